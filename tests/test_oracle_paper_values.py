"""Loose pins against numbers the paper prints (tests/golden/paper_benchmark.txt).

Under the benchmark conditions of Sec. 4.5 (fcc start, |v| = 0.9, dt = 0.001,
rc = 2.5, rs = 2.8, rho = 0.5) the paper counts about 23.3 pairs per particle
within rs after 1150 steps (Sec. 5, load-imbalance paragraph) and reports pair
lists that live about 50 steps (Sec. 5, lifetime paragraph).  The oracle's run
at the same conditions (a smaller box, N = 4000) must land within 5% of the
pair density; its half-skin rule (stricter than the paper's DUTC + LDC check)
must give lists of the same order of lifetime.
"""

import os

import numpy as np

import lj_inputs as li

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_benchmark.txt")


def _golden():
    vals = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return vals


def test_pair_density_under_paper_conditions(ref):
    g = _golden()
    q, L = li.fcc_lattice(10, g["rho"])
    v = li.fixed_speed_velocities(q.shape[0], g["speed"], seed=0)
    nsteps = int(g["warmup_steps"] + g["timed_steps"])
    q1, _, log, nreb = ref.run(q, v, L, nsteps, dt=g["dt"], rc=g["rc"], rs=g["rs"], sample_every=50)
    per_particle = len(ref.pairs_cells(q1, L, g["rs"])) / q.shape[0]
    paper = 0.5 * (g["pairs_max"] + g["pairs_min"]) / g["particles_per_process"]
    assert abs(per_particle - paper) < 0.05 * paper, (per_particle, paper)
    lifetime = nsteps / nreb
    assert 0.5 * g["lifetime_a"] < lifetime < 2.0 * g["lifetime_b"], lifetime
    # NVE at dt = 0.001: energy per particle constant to ~1e-5
    e = log[:, 3] / q.shape[0]
    assert np.abs(e - e[0]).max() < 1e-4
