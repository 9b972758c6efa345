"""Pins of the oracle's force/energy/virial loop (Sec. 3.1-3.2).

  * fcc at t = 0: F = 0 by inversion symmetry; PE/N and W/N equal the exact
    shell sums (12 neighbours at sqrt2, 6 at 2, 24 at sqrt6) in rational
    arithmetic;
  * two particles: closed form along the axis, equal and opposite;
  * Newton's third law (sum of forces ~ 0) on disordered inputs;
  * F = -grad U by central differences along random directions;
  * forces do not depend on the search length once rs >= rc;
  * the per-particle sampling routine equals the full computation;
  * forces, PE and virial equal an independent O(N^2) torch enumeration
    differentiated by autograd (forces as -grad U, the virial as -dU/ds for
    displacements scaled by s), on jittered lattices at three densities.
"""

from fractions import Fraction as Fr

import numpy as np
import pytest

import lj_inputs as li
from tests.test_oracle_potential import exact_V_g


def test_fcc_energy_and_virial_exact(ref):
    q, L = li.fcc_lattice(10)
    n = q.shape[0]
    F, pe, w = ref.forces(q, L)
    shells = [(Fr(2), 12), (Fr(4), 6), (Fr(6), 24)]
    pe_exact = Fr(0)
    w_exact = Fr(0)
    for r2, cnt in shells:
        V, g = exact_V_g(r2)
        pe_exact += Fr(cnt, 2) * V
        w_exact += Fr(cnt, 2) * g * r2
    assert pe / n == pytest.approx(float(pe_exact), rel=1e-14)
    assert w / n == pytest.approx(float(w_exact), rel=1e-14)
    assert np.abs(F).max() < 1e-12
    # the values these shell sums give
    assert pe / n == pytest.approx(-2.4131626982396188, rel=1e-14)
    assert w / n == pytest.approx(-14.413251470133467, rel=1e-14)


def test_two_particles_closed_form(ref):
    L = 20.0
    for r in [0.97, 1.12, 1.6, 2.49, 2.51]:
        q = np.array([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]])
        F, pe, w = ref.forces(q, L)
        if r < 2.5:
            V, g = ref.pair(r * r)
        else:
            V, g = 0.0, 0.0
        assert pe == pytest.approx(V, rel=1e-14, abs=1e-300)
        assert F[0, 0] == pytest.approx(-g * r, rel=1e-14, abs=1e-300)
        assert F[1, 0] == pytest.approx(g * r, rel=1e-14, abs=1e-300)
        assert np.all(F[:, 1:] == 0.0)
        assert w == pytest.approx(g * r * r, rel=1e-14, abs=1e-300)


def test_two_particles_across_boundary(ref):
    L = 12.0
    q = np.array([[0.3, 6.0, 6.0], [L - 0.9, 6.0, 6.0]])  # min-image distance 1.2
    F, pe, w = ref.forces(q, L)
    V, g = ref.pair(1.2 * 1.2)
    assert pe == pytest.approx(V, rel=1e-12)
    # d = q1 - q0 = -1.2 (through the boundary): F_0 = -g d = +1.2 g
    assert F[0, 0] == pytest.approx(1.2 * g, rel=1e-12)


def test_newton_third_law(ref):
    q, L = li.jittered_fcc(8, amp=0.2)
    F, _, _ = ref.forces(q, L)
    assert np.abs(F.sum(axis=0)).max() / np.abs(F).sum() < 1e-14


def test_force_is_minus_gradient(ref):
    q, L = li.jittered_fcc(3, amp=0.15, seed=4)  # L = 6: brute-force path
    rng = np.random.default_rng(7)
    F, _, _ = ref.forces(q, L)
    h = 1e-6
    for _ in range(4):
        u = rng.standard_normal(q.shape)
        u /= np.linalg.norm(u)
        _, up, _ = ref.forces(q + h * u, L)
        _, um, _ = ref.forces(q - h * u, L)
        dU = (up - um) / (2 * h)
        assert dU == pytest.approx(-np.sum(F * u), rel=1e-6, abs=1e-8)


def test_forces_independent_of_search_length(ref):
    q, L = li.jittered_fcc(8, amp=0.2, seed=9)
    F1, pe1, w1 = ref.forces(q, L, rs=2.5000001)
    F2, pe2, w2 = ref.forces(q, L, rs=2.8)
    F3, pe3, w3 = ref.forces(q, L, rs=3.9)
    scale = np.abs(F1).max()
    assert np.abs(F1 - F2).max() < 1e-13 * scale
    assert np.abs(F1 - F3).max() < 1e-13 * scale
    assert pe1 == pytest.approx(pe2, rel=1e-14) and pe1 == pytest.approx(pe3, rel=1e-14)
    assert w1 == pytest.approx(w2, rel=1e-14) and w1 == pytest.approx(w3, rel=1e-14)


def test_sampled_forces_equal_full(ref):
    q, L = li.jittered_fcc(8, amp=0.2, seed=10)
    n = q.shape[0]
    F, pe, w = ref.forces(q, L)
    idx = np.arange(0, n, 7, dtype=np.int64)
    Fs, S, pei, wi, nb = ref.forces_sample(q, L, idx)
    assert np.abs(Fs - F[idx]).max() < 1e-13 * np.abs(F).max()
    assert np.all(S >= np.linalg.norm(Fs, axis=1) - 1e-12)
    full_idx = np.arange(n, dtype=np.int64)
    _, _, pe_all, w_all, nb_all = ref.forces_sample(q, L, full_idx)
    assert pe_all.sum() == pytest.approx(pe, rel=1e-13)
    assert w_all.sum() == pytest.approx(w, rel=1e-13)
    pairs = ref.pairs_cells(q, L, 2.8)
    assert nb_all.sum() == 2 * len(pairs)


def test_neighbor_rows_equal_pair_set(ref):
    q, L = li.jittered_fcc(6, amp=0.2, seed=12)
    n = q.shape[0]
    pairs = ref.pairs_cells(q, L, 2.8)
    rows = [[] for _ in range(n)]
    for a, b in pairs.tolist():
        rows[a].append(b)
        rows[b].append(a)
    idx = np.arange(n, dtype=np.int64)
    got = ref.neighbors_sample(q, L, idx)
    for i in range(n):
        assert got[i].tolist() == sorted(rows[i])


def _torch_energy_scaled(q, L, s, rc=2.5):
    """Brute-force truncated LJ energy (eps = sigma = 1) over all pairs with the
    minimum-image displacements scaled by s: dU/ds at s = 1 is -W."""
    import torch

    n = q.shape[0]
    i, j = torch.triu_indices(n, n, 1)
    d = q[j] - q[i]
    d = (d - L * torch.round(d / L)) * s
    r2 = (d * d).sum(-1)
    x = 1.0 / rc
    c2 = 6 * x ** 14 - 3 * x ** 8
    c0 = -7 * x ** 12 + 4 * x ** 6
    s6 = (1.0 / r2) ** 3
    V = 4 * (s6 * s6 - s6 + c2 * r2 + c0)
    return torch.where(r2 < rc * rc, V, torch.zeros_like(V)).sum()


@pytest.mark.parametrize("n_fcc,rho,seed", [(5, 0.5, 31), (6, 0.8, 32), (4, 0.3, 33)])
def test_forces_match_independent_brute_force(ref, n_fcc, rho, seed):
    # an O(N^2) enumeration in torch, differentiated by autograd, against the
    # oracle's cell-list loop with its analytic pair forces: the pair set
    # (minimum image included), the force direction and sign, PE and the
    # virial W = sum g r^2 = -dU/ds for displacements scaled by s
    import torch

    q, L = li.jittered_fcc(n_fcc, amp=0.2, rho=rho, seed=seed)
    F, pe, w = ref.forces(q, L)
    qt = torch.tensor(q, dtype=torch.float64, requires_grad=True)
    s = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    U = _torch_energy_scaled(qt, L, s)
    gq, gs = torch.autograd.grad(U, (qt, s))
    assert pe == pytest.approx(U.item(), rel=1e-12)
    assert np.abs(F + gq.numpy()).max() <= 1e-10 * np.abs(F).max()
    assert w == pytest.approx(-gs.item(), rel=1e-11)
