"""Throughput benchmark of the LJ hot path on one MI355X.

Other workloads: --config lj4k / lj4m / lj256k / lj131m (sizes of the same
fluid), paper500k / paper32m (the paper's own benchmark conditions: |v| = 0.9
in random directions, dt = 0.001, 150 untimed + 1000 timed steps, FP64);
--ablation adds a run without re-sorting on shuffled labels.

Workload (default "lj32m"): N = 32,000,000 particles on a 200^3-cell fcc
lattice at rho = 0.5 (L = 400), truncated LJ with rc = 2.5 and skin 0.3
(rs = 2.8), Maxwell-Boltzmann velocities at T = 1 (seed 0), dt = 0.005, NVE.
The headline run uses mixed precision (FP32 pair forces, FP64 integration and
sums) with a cell-order re-sort at every rebuild; an FP64 run on the same seed
is reported beside it.  A step is one full pass of the hot path: half kick +
drift, rebuild check (and bin / re-sort / pair-list build when due), forces,
second half kick.

After the timed steps of each mode, an untimed leg runs the paper's own
protocol on the same state (150 steps, then 1000 steps with the energy sampled
every 10): its rate and the energy drift per 1000 steps fitted to its samples
are reported for every mode whatever --steps is, so that the FP64 and mixed
rates always stand beside their drifts.

The CPU baseline (the oracle, plain C) runs first, in child processes that
touch no GPU: one thread, then one process per core of the job's CPU share,
each on its own 256,000-particle box of the same fluid.

Prints one JSON line on stdout; progress goes to stderr.
"""

from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import re
import subprocess
import sys
import time

import numpy as np

METRIC = "particle-steps/s, 32M-atom LJ NVE: FP64 vs FP32/FP64 mixed at stated drift"
HBM_PEAK_GBS = 8000.0
PAPER_NODE_RATE = 105.7e6   # particle-steps/s of one 64-process POWER6 node on 64 x 500k particles (Sec. 4.5)
ROOT = os.path.dirname(os.path.abspath(__file__))
# sources that define the force kernels; a counter record is used only while they are unchanged
FORCE_SOURCES = ("paper_1012_2677_amd/csrc/md_forces.hip", "paper_1012_2677_amd/csrc/md_internal.h")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def force_bytes_per_key(mean_entries: float, mixed: bool, tiled: bool = False, half: bool = False) -> float:
    """Algorithmic HBM bytes of one key in the timed force pass, which inside a
    run is fused with the integrator (second half kick, next first half kick,
    drift): row offset (8) + row length (4) + 4 bytes per slot entry or 2 per
    tiled entry + the
    key's own coordinates (FP32 local 16 B in mixed mode; FP64 32 B in FP64
    mode, plus its 4 B packed cell with slot entries) + the integrator's streams: velocity read and
    write (48), reference position (24), position written (32; mixed mode also
    reads the FP64 position, 32, its packed cell, 4, and writes new local
    coordinates, 16).  Partner coordinates are re-reads of coordinates counted
    once as keys (in the tiled pass: staged into LDS from the same array).
    A half list (each pair once, mean_entries of them per key) is not fused:
    the force array (12 B per key in mixed mode, 24 in FP64) is written by the
    clear, read and written once by the atomics of the pair pass (counted
    once) and read by the integrator pass, 4 times in all."""
    idx = 8 + 4 + (2 if tiled else 4) * mean_entries
    fbytes = 4 * (12 if mixed else 24) if half else 0
    if mixed:
        return idx + 16 + 32 + 4 + 48 + 24 + 32 + 16 + fbytes
    return idx + 32 + (0 if tiled else 4) + 48 + 24 + 32 + fbytes


def plan_bytes_per_key(mean_entries: float) -> float:
    """Algorithmic bytes per particle of the fused force + integrator pass as
    the hot path's measurement plan counts them, whatever the list layout:
    the force row reads 4 bytes per list entry, an 8-byte row offset and the
    24-byte FP64 position; the integrator adds the position written (24), the
    velocity read and written (48) and the reference position (24), its force
    store and load and its position read vanishing in the fusion:
    4 m + 128."""
    return 4.0 * mean_entries + 8 + 24 + 24 + 48 + 24


def force_sources_sha256() -> str:
    h = hashlib.sha256()
    for rel in FORCE_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from the committed rocprofv3
    counter record (profiles/<kernel>_<workload>_hbm_traffic.md): FETCH_SIZE and
    WRITE_SIZE in KiB per dispatch, each scaled by what the counter reads for a
    plain copy of known size.  None when there is no record or the force-kernel
    sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_hbm_traffic.md")
    if not os.path.exists(path):
        return None, "no counter record"
    with open(path) as f:
        m = re.search(r"^traffic: (.*)$", f.read(), re.M)
    if not m:
        return None, "counter record has no traffic line"
    kv = dict(item.split("=", 1) for item in m.group(1).split())
    if kv.get("source_sha256") != force_sources_sha256():
        return None, "force kernel changed since the counters were taken"
    b = (float(kv["fetch_kib"]) * float(kv["fetch_scale"]) + float(kv["write_kib"]) * float(kv["write_scale"])) * 1024
    return b, path


def hbm_probe(nbytes: int = 4 << 30, reps: int = 10):
    """Achievable HBM bandwidth from the library's streaming probes (read,
    copy, triad; plain and non-temporal accesses) on arrays of nbytes each,
    the best of reps launches of each; bytes moved per launch: read nbytes,
    copy 2 nbytes, triad 3 nbytes."""
    import torch

    from paper_1012_2677_amd import _abi as A

    dev = torch.device("cuda", 0)
    a = torch.full((nbytes // 8,), 1.0, dtype=torch.float64, device=dev)
    b = torch.full_like(a, 2.0)
    c = torch.empty_like(a)
    stream = torch.cuda.current_stream(dev).cuda_stream
    out = {}
    moved = {A.MD_PROBE_READ: 1, A.MD_PROBE_COPY: 2, A.MD_PROBE_TRIAD: 3}
    names = {A.MD_PROBE_READ: "read", A.MD_PROBE_COPY: "copy", A.MD_PROBE_TRIAD: "triad"}
    for op in (A.MD_PROBE_READ, A.MD_PROBE_COPY, A.MD_PROBE_TRIAD):
        for nt in (False, True):
            kind = op | (A.MD_PROBE_NT if nt else 0)
            ms = A.md_hbm_probe(kind, a.data_ptr(), b.data_ptr(), c.data_ptr(), nbytes, reps, stream)
            out[names[op] + ("_nt" if nt else "")] = round(moved[op] * nbytes / (ms * 1e-3) / 1e9, 1)
    torch.cuda.synchronize()
    # the copies left b = a = 1 and the triads c = a + 3 b = 4
    ok = bool(torch.all(b == 1.0).item() and torch.all(c == 4.0).item())
    del a, b, c
    torch.cuda.empty_cache()
    best = max(out.values())
    return {"array_bytes": nbytes, "reps": reps, "GBs": out, "best_GBs": best, "check": ok}


def drift_per_1000(steps_axis, e_per_particle):
    if len(e_per_particle) < 2:
        return None
    A = np.vstack([steps_axis, np.ones_like(steps_axis)]).T
    slope = np.linalg.lstsq(A, e_per_particle, rcond=None)[0][0]
    return float(slope * 1000.0)


def run_mode(cfg, precision, steps, warmup, sample_every, seed, resort_every=1, shuffle=False,
             rebuild_rule="half_skin", ldc_max=8192, list_layout="auto", tile_cells=0, protocol=(150, 1000, 10),
             step_run=0):
    """One precision mode: prepare, warmup, the timed steps, then (protocol =
    (lead, steps, sample_every), lead > 0 or steps > 0) the paper's protocol
    leg on the same state: lead untimed steps, then steps timed ones with the
    energy sampled every sample_every steps, whose samples give the drift."""
    import torch

    import lj_inputs as li
    from paper_1012_2677_amd import Engine

    # the mode's footprint is its peak above what the process held before
    # (a previous mode's state, freed here first)
    gc.collect()
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    held_before = torch.cuda.memory_allocated()
    t0 = time.perf_counter()
    q, L = li.fcc_lattice(cfg["n_fcc"], cfg["rho"])
    v = li.initial_velocities(cfg, q.shape[0], seed=seed)
    if shuffle:
        # labels exchanged at random, positions and momenta kept (Sec. 3.3's
        # stand-in for a long run without re-sorting)
        q, v, _ = li.shuffle_labels(q, v, seed=seed + 1)
    n = q.shape[0]
    e = Engine(q, v, L, rc=cfg["rc"], rs=cfg["rc"] + cfg["skin"], dt=cfg["dt"], precision=precision,
               resort_every=resort_every, rebuild_rule=rebuild_rule, ldc_max=ldc_max, list_layout=list_layout,
               tile_cells=tile_cells, step_run=step_run, device="cuda:0", timers=True)
    del q, v
    e.prepare()
    e0 = e.energies()
    log(f"[bench] {precision}: N={n} prepared in {time.perf_counter() - t0:.1f}s, "
        f"list stride {e.plist.cell_stride}, entries {int(e.plist.status[0].item())}, "
        f"tiled {int(e.state.list_tiled)} (tile cells {int(e.state.tile_cells)}, stage {int(e.state.tile_stage)})")
    if warmup > 0:
        e.step(warmup)
        log(f"[bench] {precision}: {warmup} warmup steps done")
    for k in range(len(e.timers.ms)):
        e.timers.ms[k] = 0.0
        e.timers.launches[k] = 0
    reb0 = e.rebuilds
    ldc0 = e.ldc_stats
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elog = e.step(steps, sample_every=sample_every)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    dt = t2 - t1
    entries = int(e.plist.status[0].item())
    tiled = int(e.state.list_tiled)
    half = int(e.state.list.half)
    tim = e.timer_dict()
    rebuilds = e.rebuilds - reb0
    log(f"[bench] {precision}: {steps} steps in {dt:.3f}s, {rebuilds} rebuilds, timers {tim}")
    e_pp = elog[:, 3] / n if len(elog) else np.zeros(0)
    out = {
        "n": n,
        "L": L,
        "seconds": dt,
        "value": n * steps / dt,
        "ms_per_step": 1e3 * dt / steps,
        "rebuilds": rebuilds,
        "rebuild_rule": rebuild_rule,
        "ldc_checks_kept": [e.ldc_stats[0] - ldc0[0], e.ldc_stats[1] - ldc0[1]],
        "mean_list_entries": entries / n,
        "list_tiled": tiled,
        "list_half": half,
        "tile_cells": int(e.state.tile_cells),
        "step_run": int(step_run),
        "list_cell_stride": int(e.plist.cell_stride),
        "list_stride_needed": int(e.plist.status[1].item()),
        "timers_ms": {k: [round(m, 3), c] for k, (m, c) in tim.items()},
        "energy_per_particle_start": float(e0[3] / n),
        "energy_per_particle_samples": [float(x) for x in e_pp],
        "temperature_end": float(2.0 * elog[-1, 0] / (3.0 * (n - 1))) if len(elog) else None,
    }
    fm, fl = tim.get("force", (0.0, 0))
    if fl > 0:
        avg_ms = fm / fl
        per_launch = n * force_bytes_per_key(entries / n, precision == "mixed", bool(tiled), bool(half))
        plan = n * plan_bytes_per_key(entries / n)
        out["force_kernel"] = {"avg_ms": avg_ms, "launches": fl,
                               "algorithmic_bytes_per_launch": plan,
                               "achieved_GBs": plan / (avg_ms * 1e-3) / 1e9,
                               "layout_bytes_per_launch": per_launch,
                               "layout_GBs": per_launch / (avg_ms * 1e-3) / 1e9}
    lead, psteps, pevery = protocol
    if psteps > 0:
        if lead > 0:
            e.step(lead)
        torch.cuda.synchronize()
        s0 = e.step_count
        r0 = e.rebuilds
        t3 = time.perf_counter()
        plog = e.step(psteps, sample_every=pevery)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        first = (s0 // pevery + 1) * pevery
        axis = np.arange(first, first + pevery * len(plog), pevery, dtype=np.float64)[: len(plog)]
        ep = plog[:, 3] / n
        out["protocol"] = {
            "lead_steps": lead, "steps": psteps, "sample_every": pevery,
            "first_step": s0 + 1,
            "value": n * psteps / (t4 - t3),
            "MUPS": n * psteps / (t4 - t3) / 1e6,
            "ms_per_step": 1e3 * (t4 - t3) / psteps,
            "rebuilds": e.rebuilds - r0,
            "drift_per_1000_steps": drift_per_1000(axis, ep),
            "energy_per_particle_first": float(ep[0]) if len(ep) else None,
            "energy_per_particle_last": float(ep[-1]) if len(ep) else None,
            "max_abs_energy_change": float(np.abs(ep - ep[0]).max()) if len(ep) else None,
            "temperature_end": float(2.0 * plog[-1, 0] / (3.0 * (n - 1))) if len(plog) else None,
        }
        out["drift_per_1000_steps"] = out["protocol"]["drift_per_1000_steps"]
        log(f"[bench] {precision}: protocol {lead} + {psteps} steps: {out['protocol']['ms_per_step']:.3f} ms/step, "
            f"drift {out['drift_per_1000_steps']:.3e} per particle per 1000 steps")
    out["hbm_footprint_bytes"] = int(torch.cuda.max_memory_allocated() - held_before)
    # the list grows (a larger cell stride) when a tile's rows outgrow it
    out["list_cell_stride_end"] = int(e.plist.cell_stride)
    if held_before:
        out["hbm_held_before_bytes"] = int(held_before)
    del e
    gc.collect()
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    return out


def adjoint_bytes_per_key(mean_entries: float) -> float:
    """Algorithmic HBM bytes of one key in md_adjoint_kick (the fused adjoint
    kick of the reverse sweep, out accumulated and u_out written): row offset
    (8) + row length (4) + 4 per slot entry + own position (32) + packed cell
    (4) + u (24) + out read and written (48) + u_out written (24).  Partner
    positions and u are re-reads of arrays counted once as keys."""
    return 8 + 4 + 4 * mean_entries + 32 + 4 + 24 + 48 + 24


def grad_mode(cfg, steps, ckpt, seed, reps=50):
    """Gradient of the trajectory observable O = (1/K) sum_k U(q_k) with
    respect to q0, eps and sigma (TrajectoryMeanPE: forward run storing a
    checkpoint every ckpt steps, then the checkpointed reverse sweep), timed
    end to end after an untimed short one; then md_adjoint_kick alone at the
    starting positions, timed with HIP events on the stream it runs on."""
    import torch

    import lj_inputs as li
    from paper_1012_2677_amd import TrajectoryMeanPE
    from paper_1012_2677_amd.autograd import Field

    dev = torch.device("cuda", 0)
    q, L = li.fcc_lattice(cfg["n_fcc"], cfg["rho"])
    v = li.initial_velocities(cfg, q.shape[0], seed=seed)
    n = q.shape[0]
    rs, dt = cfg["rc"] + cfg["skin"], cfg["dt"]
    qt = torch.tensor(q, dtype=torch.float64, device=dev, requires_grad=True)
    vt = torch.tensor(v, dtype=torch.float64, device=dev)
    eps = torch.tensor(1.0, dtype=torch.float64, device=dev, requires_grad=True)
    sig = torch.tensor(1.0, dtype=torch.float64, device=dev, requires_grad=True)
    TrajectoryMeanPE.apply(qt, vt, eps, sig, L, ckpt, ckpt, dt, cfg["rc"], rs).backward()
    qt.grad = eps.grad = sig.grad = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    O = TrajectoryMeanPE.apply(qt, vt, eps, sig, L, steps, ckpt, dt, cfg["rc"], rs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    O.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    log(f"[bench] gradients: N={n}, {steps} steps, checkpoint every {ckpt}: forward {t1 - t0:.3f}s, "
        f"reverse sweep {t2 - t1:.3f}s, dO/deps {eps.grad.item():.6f}, dO/dsigma {sig.grad.item():.6f}")
    f = Field(n, L, 1.0, 1.0, cfg["rc"], rs, dev)
    f.params.dt = dt
    f.set_positions(qt.detach())
    g = torch.Generator(device=dev).manual_seed(seed)
    u = torch.randn((3, n), dtype=torch.float64, device=dev, generator=g)
    out = torch.zeros_like(u)
    u_out = torch.empty_like(u)
    acc = torch.zeros(2, dtype=torch.float64, device=dev)
    coef = (1.0, -0.5 * dt, -1.0 / steps, 0.5 * dt, 1.0 / steps)
    f.adjoint_kick(u, out, u_out, coef, acc)
    stream = torch.cuda.current_stream(dev)
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(reps):
        f.adjoint_kick(u, out, u_out, coef, acc)
    end.record(stream)
    torch.cuda.synchronize()
    avg_ms = start.elapsed_time(end) / reps
    entries = int(f.plist.status[0].item())
    per_call = n * adjoint_bytes_per_key(entries / n)
    gbs = per_call / (avg_ms * 1e-3) / 1e9
    log(f"[bench] md_adjoint_kick: {avg_ms:.3f} ms per call, {gbs:.0f} GB/s algorithmic")
    return {
        "n": n, "steps": steps, "checkpoint_every": ckpt,
        "forward_s": t1 - t0, "reverse_s": t2 - t1,
        "value": n * steps / (t2 - t0), "unit": "particle-steps/s (forward + reverse sweep)",
        "dO_deps": eps.grad.item(), "dO_dsigma": sig.grad.item(),
        "adjoint_kernel": {"kernel": "k_adjoint (md_adjoint_kick)", "bound": "hbm", "avg_call_ms": avg_ms,
                           "algorithmic_bytes_per_call": int(per_call), "achieved": round(gbs, 1),
                           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)},
    }


def cpu_worker(config: str, seconds_target: float, seed: int):
    """One oracle process (plain C, one thread): the fluid of `config` at the
    density, velocity law, dt and skin of the workload, on a 256,000-particle
    box (40^3 fcc cells), for enough velocity-Verlet steps (rebuilds included)
    to take about seconds_target.  Prints one JSON line."""
    import oracle
    import lj_inputs as li

    cfg = {**li.CONFIGS, **li.PAPER_CONFIGS}[config]
    q, L = li.fcc_lattice(40, cfg["rho"])
    v = li.initial_velocities(cfg, q.shape[0], seed=seed)
    n = q.shape[0]
    kw = dict(dt=cfg["dt"], rc=cfg["rc"], rs=cfg["rc"] + cfg["skin"], sample_every=0)
    t0 = time.perf_counter()
    oracle.run(q, v, L, 2, **kw)
    per_step = (time.perf_counter() - t0) / 2.0
    k = max(2, min(400, int(seconds_target / max(per_step, 1e-3))))
    t0 = time.perf_counter()
    oracle.run(q, v, L, k, **kw)
    dt = time.perf_counter() - t0
    print(json.dumps({"n": n, "steps": k, "seconds": dt, "value": n * k / dt}), flush=True)


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(config: str, cfg, seconds_target=10.0):
    """The oracle as it is, timed on this job's host cores in child processes
    that use no GPU: one process alone (one thread), then one process per core
    of the job's CPU share at once, each on its own 256,000-particle box of the
    same fluid (a bounded sample of the workload).  The all-core aggregate is
    the sum of the processes' rates."""
    affinity = len(os.sched_getaffinity(0))
    # at most 16 workers: the CPU share of one GPU of the job
    procs = max(1, min(affinity, 16))

    def launch(seed):
        return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", "--config", config,
                                 "--cpu-seconds", str(seconds_target), "--seed", str(seed)],
                                stdout=subprocess.PIPE, text=True, cwd=ROOT)

    def collect(ps):
        res = []
        for p in ps:
            out, _ = p.communicate()
            if p.returncode != 0:
                raise RuntimeError(f"cpu worker failed with status {p.returncode}")
            res.append(json.loads(out.strip().splitlines()[-1]))
        return res

    single = collect([launch(0)])[0]
    log(f"[bench] cpu oracle, one thread: {single['value']:.3e} particle-steps/s")
    t0 = time.perf_counter()
    many = collect([launch(k) for k in range(procs)])
    wall = time.perf_counter() - t0
    agg = sum(r["value"] for r in many)
    log(f"[bench] cpu oracle, {procs} processes: {agg:.3e} particle-steps/s in {wall:.1f} s")
    vel = f"|v|={cfg['speed']}" if "speed" in cfg else f"T={cfg['T']}"
    n = single["n"]
    return {"value": agg, "unit": "particle-steps/s", "cores": procs, "kind": "oracle",
            "sample": f"{procs} oracle processes at once (one thread each, plain C), each on its own N={n} box "
                      f"(40^3 fcc cells, rho={cfg['rho']}, {vel}, dt={cfg['dt']}, rc={cfg['rc']}, "
                      f"skin={cfg['skin']}, FP64) for {min(r['steps'] for r in many)}-"
                      f"{max(r['steps'] for r in many)} velocity-Verlet steps incl. rebuilds; "
                      f"rates summed; {wall:.1f} s wall",
            "cpu_model": _cpu_model(), "affinity_cores": affinity,
            "single_thread": {"value": single["value"], "steps": single["steps"], "seconds": single["seconds"],
                              "MUPS": single["value"] / 1e6},
            "MUPS_per_core": agg / procs / 1e6,
            "paper_MUPS_per_process_context": {"Xeon X5570 core (2.93 GHz)": 2.730,
                                               "POWER6 SMT process (4.7 GHz)": 1.652}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default 10; 150 for paper*)")
    ap.add_argument("--config", default="lj32m", help="lj4k, lj4m, lj32m, lj256k, lj131m, paper500k, paper32m")
    ap.add_argument("--rebuild-rule", default="half_skin", choices=["half_skin", "dutc_ldc"],
                    help="pair-list validity rule (dutc_ldc: Alg. alg_validity_check)")
    ap.add_argument("--ldc-max", type=int, default=8192, help="most particles in the large-displacement check")
    ap.add_argument("--ablation", action="store_true",
                    help="also time the headline precision without re-sorting, labels shuffled first")
    ap.add_argument("--sample-every", type=int, default=50)
    ap.add_argument("--list-layout", default="auto", choices=["auto", "slots", "half"],
                    help="list of the simulation state: tiled when possible (auto), slot entries (slots) "
                         "or each pair once with atomic partner forces (half)")
    ap.add_argument("--tile-cells", type=int, default=0, help="tile length along z in cells (0 = automatic)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--step-run", type=int, default=0,
                    help="steps queued per wait for the device (0 = automatic, 1 = a wait after every step)")
    ap.add_argument("--gradients", action="store_true",
                    help="also time the gradient of the trajectory mean PE (on by default for lj256k)")
    ap.add_argument("--ckpt", type=int, default=20, help="checkpoint interval of the gradient run")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 companion run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--modes", default=None, help="comma list of precisions to run (default mixed,fp64)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run the plain 1 GiB copy probe (the reference kernel for HBM counter scaling)")
    ap.add_argument("--protocol-lead", type=int, default=150,
                    help="untimed steps before the protocol leg (the paper's 150)")
    ap.add_argument("--protocol-steps", type=int, default=1000,
                    help="steps of the protocol leg after the timed steps (0 = none); its energy samples give "
                         "the drift per 1000 steps")
    ap.add_argument("--protocol-every", type=int, default=10, help="energy sampling interval of the protocol leg")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="target seconds per CPU oracle process")
    ap.add_argument("--cpu-worker", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker:
        # a child of cpu_baseline: the oracle only, no GPU
        cpu_worker(args.config, args.cpu_seconds, args.seed)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: there is no multi-GPU path (the domain decomposition that would "
              "shard the work over GPUs is not built). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import lj_inputs as li

    cfg = dict({**li.CONFIGS, **li.PAPER_CONFIGS}[args.config])
    # the CPU baseline first, while this process has not touched the GPU
    cpu = None if (args.no_cpu or args.calibrate_copy) else cpu_baseline(args.config, cfg, args.cpu_seconds)

    import torch

    if args.calibrate_copy:
        # the reference kernel of the HBM counter scaling: the library's plain
        # copy probe over 1 GiB (reads 1 GiB, writes 1 GiB per launch)
        from paper_1012_2677_amd import _abi as A

        a = torch.full(((1 << 30) // 8,), 1.0, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        ms = A.md_hbm_probe(A.MD_PROBE_COPY, a.data_ptr(), b.data_ptr(), None, 1 << 30, 3,
                            torch.cuda.current_stream().cuda_stream)
        print(json.dumps({"calibrate_copy": {"kernel": "md::k_probe<1, false>", "bytes_read": 1 << 30,
                                             "bytes_written": 1 << 30, "best_ms": ms}}), flush=True)
        return
    if args.warmup is None:
        args.warmup = cfg.get("warmup", 10)
    headline = cfg["precision"]
    modes = args.modes.split(",") if args.modes else ([headline] + ([] if args.no_fp64 else
                                                                    (["fp64"] if headline != "fp64" else [])))
    sample_every = min(args.sample_every, max(1, args.steps))
    protocol = (args.protocol_lead, args.protocol_steps, args.protocol_every)
    results = {}
    for m in modes:
        results[m] = run_mode(cfg, m, args.steps, args.warmup, sample_every, args.seed,
                              rebuild_rule=args.rebuild_rule, ldc_max=args.ldc_max, list_layout=args.list_layout,
                              tile_cells=args.tile_cells, protocol=protocol, step_run=args.step_run)
    head = results[modes[0]]
    n = head["n"]
    drift = {m: results[m].get("drift_per_1000_steps") for m in modes}
    if "mixed" in drift and "fp64" in drift and drift["mixed"] is not None and drift["fp64"] is not None:
        fluct = results["fp64"]["protocol"]["max_abs_energy_change"]
        drift["matched"] = bool(abs(drift["mixed"]) <= 2.0 * abs(drift["fp64"]) or
                                max(abs(drift["mixed"]), abs(drift["fp64"])) <= fluct)
        drift["criterion"] = ("|drift mixed| <= 2 |drift FP64|, or both below the FP64 run's largest energy "
                              "change over the leg")
    ablation = None
    if args.ablation:
        ab = run_mode(cfg, modes[0], args.steps, args.warmup, sample_every, args.seed, resort_every=0, shuffle=True,
                      protocol=(0, 0, 0))
        ablation = {"no_resort_shuffled": {k: ab[k] for k in ("value", "ms_per_step", "rebuilds", "timers_ms")},
                    "resort_every_rebuild_over_no_resort": head["value"] / ab["value"]}
        log(f"[bench] ablation: no re-sort, shuffled labels: {ab['ms_per_step']:.3f} ms/step "
            f"(re-sort at every rebuild is {ablation['resort_every_rebuild_over_no_resort']:.2f}x faster)")
    fk = head.get("force_kernel")
    probe = hbm_probe()
    log(f"[bench] streaming probes (GB/s): {probe['GBs']}")
    roofline = None
    if fk:
        if head.get("list_half"):
            # not one kernel: the force clear, k_pairs_half and k_integrate_half
            kname = "force_step_half" + ("" if modes[0] == "mixed" else "_fp64")
        elif modes[0] == "mixed":
            kname = "k_pairs_tiled" if head.get("list_tiled") else "k_pairs_mixed"
        else:
            kname = "k_pairs_tiled_fp64" if head.get("list_tiled") else "k_pairs_fp64"
        traffic, tsrc = counter_traffic(kname, args.config)
        roofline = {"bound": "hbm", "achieved": round(fk["achieved_GBs"], 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(fk["achieved_GBs"] / HBM_PEAK_GBS, 4),
                    "traffic": None if traffic is None else round(traffic / (fk["avg_ms"] * 1e-3) / 1e9, 1),
                    "traffic_bytes_per_launch": None if traffic is None else int(traffic),
                    "traffic_source": tsrc,
                    "kernel": kname,
                    "avg_launch_ms": round(fk["avg_ms"], 4),
                    "algorithmic_bytes_per_launch": int(fk["algorithmic_bytes_per_launch"]),
                    "algorithmic_bytes_per_particle": round(fk["algorithmic_bytes_per_launch"] / n, 2),
                    "layout_bytes_per_launch": int(fk["layout_bytes_per_launch"]),
                    "layout_GBs": round(fk["layout_GBs"], 1),
                    "layout_frac": round(fk["layout_GBs"] / HBM_PEAK_GBS, 4),
                    "achievable_GBs": probe["best_GBs"],
                    "achievable_probe": probe,
                    "frac_of_achievable": round(fk["achieved_GBs"] / probe["best_GBs"], 4)}
    grads = None
    if args.gradients or args.config == "lj256k":
        grads = grad_mode(cfg, cfg.get("steps", 200), args.ckpt, args.seed)
    vel_desc = (f"|v|={cfg['speed']} in random directions" if "speed" in cfg
                else f"T={cfg['T']} Maxwell-Boltzmann")
    # The paper's own number exists only for its own workload: 64 cubes of
    # 500,000 particles, the share of one node of its POWER6 machine
    # (105.7 M particle-updates/s, FP64, 2010 hardware).
    vs_baseline = head["value"] / PAPER_NODE_RATE if (args.config == "paper32m" and modes[0] == "fp64") else None
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
        "vs_baseline": vs_baseline,
        "dtype": "f32+f64" if modes[0] == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: LJ NVE, N={n} on a {cfg['n_fcc']}^3-cell fcc lattice, "
                               f"rho={cfg['rho']}, rc={cfg['rc']}, skin={cfg['skin']}, {vel_desc} (seed {args.seed}), "
                               f"dt={cfg['dt']}, {modes[0]} precision, cell re-sort at every rebuild, "
                               f"{args.rebuild_rule} rebuild rule",
                   "n": n, "box": head["L"], "precision": modes[0], "sample_every": sample_every},
        "roofline": roofline,
        "drift_per_1000_steps": drift,
        "cpu_baseline": cpu,
        "modes": results,
        "ablation": ablation,
        "gradients": grads,
        "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
