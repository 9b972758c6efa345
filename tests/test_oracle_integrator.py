"""Pins of the oracle's velocity-Verlet run with the bookkeeping rule
(Sec. 2.3 search-length rule, Sec. 4.5 second-order symplectic integrator).

  * time reversibility: n steps, negate v, n steps returns to the start;
  * second order: the energy error scales as dt^2;
  * total momentum is conserved to rounding;
  * a dimer agrees with scipy's high-order adaptive integrator;
  * the skin list never misses an interacting pair: a run with the skin rule
    matches a run that rebuilds every step;
  * the rebuild count is consistent with the half-skin rule.
"""

import numpy as np
import pytest

import lj_inputs as li


def _min_image(d, L):
    return d - L * np.rint(d / L)


def test_reversibility(ref):
    q0, L = li.fcc_lattice(5)
    v0 = li.maxwell_boltzmann(q0.shape[0], seed=3)
    q1, v1, _, _ = ref.run(q0, v0, L, 60, dt=0.005, sample_every=0)
    q2, v2, _, _ = ref.run(q1, -v1, L, 60, dt=0.005, sample_every=0)
    assert np.abs(_min_image(q2 - q0, L)).max() < 1e-9
    assert np.abs(v2 + v0).max() < 1e-9


def test_energy_error_scales_as_dt_squared(ref):
    q0, L = li.fcc_lattice(5)
    v0 = li.maxwell_boltzmann(q0.shape[0], seed=1)
    spans = []
    for dt, k in [(0.004, 100), (0.002, 200)]:
        _, _, log, _ = ref.run(q0, v0, L, k, dt=dt, sample_every=k // 50)
        e = log[:, 3]
        spans.append(np.abs(e - e[0]).max())
    ratio = spans[0] / spans[1]
    assert 3.0 < ratio < 5.2, ratio


def test_momentum_conserved(ref):
    q0, L = li.fcc_lattice(5)
    v0 = li.maxwell_boltzmann(q0.shape[0], seed=2)
    _, v1, _, _ = ref.run(q0, v0, L, 50, sample_every=0)
    assert np.abs(v1.sum(axis=0)).max() < 1e-11


def test_dimer_against_scipy(ref):
    from scipy.integrate import solve_ivp

    L = 30.0
    q0 = np.array([[10.0, 10.0, 10.0], [11.3, 10.0, 10.0]])
    v0 = np.array([[0.4, 0.0, 0.0], [-0.4, 0.0, 0.0]])
    T = 2.0
    dt = 1e-4
    nsteps = int(round(T / dt))
    q1, v1, _, _ = ref.run(q0, v0, L, nsteps, dt=dt, sample_every=0)

    def rhs(t, y):
        x = y[1] - y[0]
        V, g = ref.pair(x * x)
        f = -g * x  # force on particle 0 along x
        return [y[2], y[3], f, -f]

    sol = solve_ivp(rhs, (0, T), [10.0, 11.3, 0.4, -0.4], method="DOP853", rtol=1e-12, atol=1e-12)
    x0, x1, u0, u1 = sol.y[:, -1]
    assert q1[0, 0] == pytest.approx(x0, abs=1e-6)
    assert q1[1, 0] == pytest.approx(x1, abs=1e-6)
    assert v1[0, 0] == pytest.approx(u0, abs=1e-6)


def test_skin_list_matches_rebuild_every_step(ref):
    q0, L = li.fcc_lattice(5)
    v0 = li.maxwell_boltzmann(q0.shape[0], seed=4)
    # rs = rc: the half-skin threshold is zero, so the list is rebuilt every
    # step with exactly the pairs inside rc
    qa, va, loga, nra = ref.run(q0, v0, L, 40, rs=2.8, sample_every=10)
    qb, vb, logb, nrb = ref.run(q0, v0, L, 40, rs=2.5, sample_every=10)
    assert nrb == 40
    assert 0 < nra < 40
    assert np.abs(_min_image(qa - qb, L)).max() < 1e-9
    assert np.abs(loga - logb).max() < 1e-8 * np.abs(logb).max()


def test_rebuild_count_plausible(ref):
    # max displacement > skin/2 = 0.15 with |v| ~ 1.6 and dt = 0.005: a rebuild
    # roughly every 5-10 steps at T = 1
    q0, L = li.fcc_lattice(10)
    v0 = li.maxwell_boltzmann(q0.shape[0], seed=0)
    _, _, log, nreb = ref.run(q0, v0, L, 100, sample_every=10)
    assert 8 <= nreb <= 25
    e = log[:, 3] / q0.shape[0]
    assert np.abs(e - e[0]).max() < 2e-3
