"""Throughput benchmark of the LJ hot path on one MI355X.

Workload (default "lj32m"): N = 32,000,000 particles on a 200^3-cell fcc
lattice at rho = 0.5 (L = 400), truncated LJ with rc = 2.5 and skin 0.3
(rs = 2.8), Maxwell-Boltzmann velocities at T = 1 (seed 0), dt = 0.005, NVE.
The headline run uses mixed precision (FP32 pair forces, FP64 integration and
sums) with a cell-order re-sort at every rebuild; an FP64 run on the same seed
is reported beside it.  A step is one full pass of the hot path: half kick +
drift, rebuild check (and bin / re-sort / pair-list build when due), forces,
second half kick.

Prints one JSON line on stdout; progress goes to stderr.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "particle-steps/s, 32M-atom LJ NVE: FP64 vs FP32/FP64 mixed at stated drift"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def force_bytes_per_key(mean_entries: float, mixed: bool) -> float:
    """Algorithmic HBM bytes of one force-kernel key: row offset (8) + row length
    (4) + 4 bytes per list entry + the key's own position (16 B FP32 local
    coordinates in mixed mode, 32 B FP64 in FP64 mode) + the force written
    (12 B FP32 / 24 B FP64).  Partner positions are re-reads of positions that
    are counted once as keys."""
    return 8 + 4 + 4 * mean_entries + (16 if mixed else 32) + (12 if mixed else 24)


def drift_per_1000(steps_axis, e_per_particle):
    if len(e_per_particle) < 2:
        return None
    A = np.vstack([steps_axis, np.ones_like(steps_axis)]).T
    slope = np.linalg.lstsq(A, e_per_particle, rcond=None)[0][0]
    return float(slope * 1000.0)


def run_mode(cfg, precision, steps, warmup, sample_every, seed):
    import torch

    import lj_inputs as li
    from paper_1012_2677_amd import Engine

    t0 = time.perf_counter()
    q, L = li.fcc_lattice(cfg["n_fcc"], cfg["rho"])
    v = li.maxwell_boltzmann(q.shape[0], cfg["T"], seed=seed)
    n = q.shape[0]
    e = Engine(q, v, L, rc=cfg["rc"], rs=cfg["rc"] + cfg["skin"], dt=cfg["dt"], precision=precision,
               resort_every=1, device="cuda:0", timers=True)
    del q, v
    e.prepare()
    e0 = e.energies()
    log(f"[bench] {precision}: N={n} prepared in {time.perf_counter() - t0:.1f}s, "
        f"list stride {e.plist.cell_stride}, entries {int(e.plist.status[0].item())}")
    if warmup > 0:
        e.step(warmup)
        log(f"[bench] {precision}: {warmup} warmup steps done")
    for k in range(len(e.timers.ms)):
        e.timers.ms[k] = 0.0
        e.timers.launches[k] = 0
    reb0 = e.rebuilds
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elog = e.step(steps, sample_every=sample_every)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    entries = int(e.plist.status[0].item())
    tim = e.timer_dict()
    rebuilds = e.rebuilds - reb0
    log(f"[bench] {precision}: {steps} steps in {dt:.3f}s, {rebuilds} rebuilds, timers {tim}")
    first = warmup + sample_every
    axis = np.arange(first, first + sample_every * len(elog), sample_every, dtype=np.float64)[: len(elog)]
    e_pp = elog[:, 3] / n if len(elog) else np.zeros(0)
    out = {
        "n": n,
        "L": L,
        "seconds": dt,
        "value": n * steps / dt,
        "ms_per_step": 1e3 * dt / steps,
        "rebuilds": rebuilds,
        "mean_list_entries": entries / n,
        "timers_ms": {k: [round(m, 3), c] for k, (m, c) in tim.items()},
        "energy_per_particle_start": float(e0[3] / n),
        "energy_per_particle_samples": [float(x) for x in e_pp],
        "drift_per_1000_steps": drift_per_1000(axis, e_pp),
        "max_abs_energy_change": float(np.abs(e_pp - e0[3] / n).max()) if len(e_pp) else None,
        "temperature_end": float(2.0 * elog[-1, 0] / (3.0 * (n - 1))) if len(elog) else None,
    }
    fm, fl = tim.get("force", (0.0, 0))
    if fl > 0:
        avg_ms = fm / fl
        per_launch = n * force_bytes_per_key(entries / n, precision == "mixed")
        gbs = per_launch / (avg_ms * 1e-3) / 1e9
        out["force_kernel"] = {"avg_ms": avg_ms, "launches": fl, "algorithmic_bytes_per_launch": per_launch,
                               "achieved_GBs": gbs}
    del e
    torch.cuda.empty_cache()
    return out


def cpu_baseline(cfg, seconds_target=15.0):
    """The oracle as it is (plain C, one thread) on a bounded sample of the same
    workload: the same density, temperature, dt and skin on a 256,000-particle
    box (40^3 fcc cells), timed over enough steps for ~10-30 s."""
    import oracle
    import lj_inputs as li

    q, L = li.fcc_lattice(40, cfg["rho"])
    v = li.maxwell_boltzmann(q.shape[0], cfg["T"], seed=0)
    n = q.shape[0]
    t0 = time.perf_counter()
    oracle.run(q, v, L, 2, dt=cfg["dt"], rc=cfg["rc"], rs=cfg["rc"] + cfg["skin"], sample_every=0)
    per_step = (time.perf_counter() - t0) / 2.0
    k = max(2, min(60, int(seconds_target / max(per_step, 1e-3))))
    t0 = time.perf_counter()
    oracle.run(q, v, L, k, dt=cfg["dt"], rc=cfg["rc"], rs=cfg["rc"] + cfg["skin"], sample_every=0)
    dt = time.perf_counter() - t0
    return {"value": n * k / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"N={n} (40^3 fcc cells, rho=0.5, T=1, dt=0.005, rc=2.5, skin=0.3, FP64), "
                      f"{k} velocity-Verlet steps incl. rebuilds, single thread, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="lj32m")
    ap.add_argument("--sample-every", type=int, default=100)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 companion run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--modes", default=None, help="comma list of precisions to run (default mixed,fp64)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (see DESIGN.md for how the "
              "domain decomposition would shard it). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch

    import lj_inputs as li

    cfg = dict(li.CONFIGS[args.config])
    headline = cfg["precision"]
    modes = args.modes.split(",") if args.modes else ([headline] + ([] if args.no_fp64 else
                                                                    (["fp64"] if headline != "fp64" else [])))
    sample_every = min(args.sample_every, max(1, args.steps))
    results = {}
    for m in modes:
        results[m] = run_mode(cfg, m, args.steps, args.warmup, sample_every, args.seed)
    head = results[modes[0]]
    n = head["n"]
    fk = head.get("force_kernel")
    roofline = None
    if fk:
        roofline = {"bound": "hbm", "achieved": round(fk["achieved_GBs"], 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(fk["achieved_GBs"] / HBM_PEAK_GBS, 4), "traffic": None,
                    "kernel": "k_forces_mixed" if modes[0] == "mixed" else "k_forces_fp64",
                    "avg_launch_ms": round(fk["avg_ms"], 4),
                    "algorithmic_bytes_per_launch": int(fk["algorithmic_bytes_per_launch"])}
    cpu = None if args.no_cpu else cpu_baseline(cfg)
    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if modes[0] == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: LJ NVE, N={n} on a {cfg['n_fcc']}^3-cell fcc lattice, rho=0.5, "
                               f"rc=2.5, skin=0.3, T=1 Maxwell-Boltzmann (seed {args.seed}), dt=0.005, "
                               f"{modes[0]} precision, cell re-sort at every rebuild",
                   "n": n, "box": head["L"], "precision": modes[0], "sample_every": sample_every},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "modes": results,
        "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
