"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Bars (each stated at its test):
  * cell grid: bit-exact (cell_of, count, start, order);
  * pair list: the set of unordered pairs equals the oracle's exactly, every
    pair appears in both rows, rows are ordered by (stencil code, slot) and
    each code matches the partner's cell;
  * forces: max_i |F_i - F_i^ref| / S_i <= 1e-12 (FP64) and <= 1e-5 (mixed),
    where S_i = sum_j |g_ij| r_ij is the scale of the pair forces on i (the
    fcc lattice has F_i = 0, so a plain relative error is undefined);
    PE and W to 1e-12 (FP64) / 1e-6 (mixed) relative;
  * adjoint: H u to 1e-10 of max |H u|, parameter terms to 1e-10 relative.
"""

import numpy as np
import pytest
import torch

import lj_inputs as li
from tests import gpu_util as G
from tests.test_oracle_cells import ADV_L, adversarial_pairs

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
MIXED_TOL = 1e-5


def _case(name):
    if name == "fcc10":
        q, L = li.fcc_lattice(10)
        return q, [L] * 3
    if name == "jitter12":
        q, L = li.jittered_fcc(12, amp=0.2, seed=5)
        return q, [L] * 3
    if name == "uniform_ragged":
        L = 21.5
        return li.uniform_box(5003, L, seed=7), [L] * 3
    if name == "aniso":
        L = np.array([14.0, 23.0, 31.5])
        rng = np.random.default_rng(8)
        n = int(0.5 * np.prod(L)) - 3
        q = np.ascontiguousarray(rng.random((n, 3)) * L)
        return q, list(L)
    if name == "aniso_jitter":
        q, L = li.fcc_lattice_box(7, 11, 16)
        rng = np.random.default_rng(10)
        q = q + 0.2 * rng.standard_normal(q.shape)
        return li.wrap_into_box(q, L), L
    if name == "ragged_jitter":
        q, L = li.jittered_fcc(11, amp=0.2, seed=6)
        return np.ascontiguousarray(q[:-13]), [L] * 3
    if name == "small_box":
        q, L = li.jittered_fcc(5, amp=0.15, seed=9)  # L = 10: 3 cells per axis
        return q, [L] * 3
    if name == "clump":
        # 100 extra particles within 1.2 of one cell's centre: that cell holds
        # more particles than the build keeps in LDS, so its rows (and those of
        # its neighbours, whose candidates exceed the register chunks) are
        # found by the build's re-reading path
        L = 21.5
        rng = np.random.default_rng(11)
        base = li.uniform_box(5003, L, seed=7)
        c = np.array([3.5, 10.0, 17.9])
        d = rng.standard_normal((100, 3))
        d *= (1.2 * rng.random((100, 1)) ** (1.0 / 3.0)) / np.linalg.norm(d, axis=1, keepdims=True)
        return li.wrap_into_box(np.concatenate([base, c + d]), L), [L] * 3
    if name == "dense":
        # rho = 1.6 in a 3-cell box: ~59 particles per cell, every full and
        # half neighbourhood beyond the build's register chunks
        L = 10.0
        return li.uniform_box(1600, L, seed=12), [L] * 3
    if name == "slab":
        # particles in x < L/2 only: empty cells, and in the tiled list whole
        # tiles without keys next to tiles with neighbours to stage
        L = 21.5
        q = li.uniform_box(4969, L, seed=13)
        q[:, 0] *= 0.5
        return q, [L] * 3
    raise KeyError(name)


CASES = ["fcc10", "jitter12", "uniform_ragged", "aniso", "aniso_jitter", "small_box", "clump", "dense", "slab"]


@pytest.fixture(autouse=True, scope="module")
def _cuda():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1012_2677_amd  # noqa: F401  (loads libmd355.so or raises)


@pytest.mark.parametrize("name", CASES)
def test_bin_cells_bit_exact(ref, name):
    q, L = _case(name)
    s = G.Standalone(q, L)
    cell_of, count, start, order, cell_xyz = s.bin()
    r_cell, r_count, r_start, r_order = ref.bin_cells(q, L, s.grid.ncell)
    assert np.array_equal(cell_of, r_cell)
    assert np.array_equal(count, r_count)
    assert np.array_equal(start, r_start)
    assert np.array_equal(order, r_order)
    nx, ny, nz = s.grid.ncell
    cx, cy, cz = cell_xyz & 1023, (cell_xyz >> 10) & 1023, (cell_xyz >> 20) & 1023
    assert np.array_equal((cx * ny + cy) * nz + cz, cell_of)


def _check_rows_structure(s, keys, partners, codes, cell_of_slot):
    nx, ny, nz = s.grid.ncell
    kc = cell_of_slot[keys]
    pc = cell_of_slot[partners]
    kx, ky, kz = kc // (ny * nz), (kc // nz) % ny, kc % nz
    px, py, pz = pc // (ny * nz), (pc // nz) % ny, pc % nz

    def off(a, b, m):
        d = (b - a) % m
        return np.where(d == m - 1, -1, d)

    sx, sy, sz = off(kx, px, nx), off(ky, py, ny), off(kz, pz, nz)
    assert np.all(np.abs(sx) <= 1) and np.all(np.abs(sy) <= 1) and np.all(np.abs(sz) <= 1)
    assert np.array_equal(codes, (sx + 1) * 9 + (sy + 1) * 3 + (sz + 1))
    # rows ordered by neighbour cell -- the key's own cell (code 13) first, then
    # codes 14 .. 26 and 0 .. 12 -- then partner slot: strictly increasing
    # within a row
    key_change = np.concatenate([[True], keys[1:] != keys[:-1]])
    comp = ((codes - 13) % 27) * (1 << 32) + partners
    inc = np.concatenate([[True], comp[1:] > comp[:-1]])
    assert np.all(inc | key_change)


@pytest.mark.parametrize("name", CASES)
def test_pairlist_equals_oracle_set(ref, name):
    q, L = _case(name)
    s = G.Standalone(q, L)
    cell_of = s.bin()[0]
    status = s.build()
    assert status[2] == 0
    off, cnt, nbr = s.plist.rows()
    keys, partners, codes = G.decode_rows(off, cnt, nbr)
    uniq, mult = G.pair_set_from_rows(keys, partners)
    assert np.all(mult == 2)
    assert status[0] == keys.shape[0]
    refp = G.pair_codes(ref.pairs_cells(q, L, 2.8))
    assert np.array_equal(uniq, refp)
    _check_rows_structure(s, keys, partners, codes, cell_of)


def test_pairlist_adversarial_ulp(ref):
    q, expect = adversarial_pairs()
    L = [ADV_L] * 3
    s = G.Standalone(q, L)
    s.bin()
    s.build()
    keys, partners, _ = G.decode_rows(*s.plist.rows())
    uniq, mult = G.pair_set_from_rows(keys, partners)
    assert np.all(mult == 2)
    assert np.array_equal(uniq, G.pair_codes(sorted(expect)))


def test_pairlist_overflow_reported(ref):
    q, L = _case("jitter12")
    good = G.Standalone(q, L)
    good.bin()
    st = good.build()
    need = int(st[1])
    small = G.Standalone(q, L, cell_stride=64)
    small.bin()
    st2 = small.build(grow=False)
    assert st2[2] == 1
    assert int(st2[1]) == need


@pytest.mark.parametrize("name", ["fcc10", "jitter12", "ragged_jitter", "aniso", "aniso_jitter", "small_box", "clump",
                                  "dense", "slab"])
def test_forces_fp64(ref, name):
    q, L = _case(name)
    s = G.Standalone(q, L)
    s.bin()
    s.build()
    F, pw = s.forces()
    idx = np.arange(q.shape[0], dtype=np.int64)
    Fr, S, pe_i, w_i, _ = ref.forces_sample(q, L, idx)
    assert G.force_error(F, Fr, S) <= FP64_TOL
    _, pe, w = ref.forces(q, L)
    assert abs(pw[0] - pe) <= FP64_TOL * np.abs(pe_i).sum()
    assert abs(pw[1] - w) <= FP64_TOL * np.abs(w_i).sum()


# Mixed precision is judged on physical configurations: its FP32 displacement
# error is about ulp(cell side) / r, so pairs far closer than sigma (as in
# uniformly random points) exceed 1e-5 by construction.
@pytest.mark.parametrize("name", ["jitter12", "ragged_jitter", "aniso_jitter", "small_box"])
def test_forces_mixed(ref, name):
    q, L = _case(name)
    s = G.Standalone(q, L, precision="mixed")
    s.bin()
    s.build()
    F, pw = s.forces()
    idx = np.arange(q.shape[0], dtype=np.int64)
    Fr, S, pe_i, w_i, _ = ref.forces_sample(q, L, idx)
    err = G.force_error(F, Fr, S)
    assert err <= MIXED_TOL, err
    _, pe, w = ref.forces(q, L)
    assert abs(pw[0] - pe) <= 1e-6 * np.abs(pe_i).sum()
    assert abs(pw[1] - w) <= 1e-6 * np.abs(w_i).sum()


def test_forces_skip_energy_and_zero_fcc(ref):
    q, L = _case("fcc10")
    s = G.Standalone(q, L)
    s.bin()
    s.build()
    F, _ = s.forces(energy=False)
    assert np.abs(F).max() < 1e-12


def test_hvp_and_param_grad(ref):
    q, L = li.jittered_fcc(8, amp=0.15, seed=21)
    L = [L] * 3
    s = G.Standalone(q, L, eps=1.1, sigma=0.97)
    s.bin()
    s.build()
    rng = np.random.default_rng(3)
    u = rng.standard_normal(q.shape)
    Hu, dp = s.hvp(u)
    Hr, dpr = ref.hvp(q, L, u, eps=1.1, sigma=0.97)
    scale = G.hvp_scale(q, L, u, ref.pairs_cells(q, L, 2.5), eps=1.1, sigma=0.97)
    assert G.elementwise_error(Hu, Hr, scale) <= 1e-10
    assert dp == pytest.approx(dpr, rel=1e-10)
    dU = s.param_grad()
    assert dU == pytest.approx(ref.param_grad(q, L, eps=1.1, sigma=0.97), rel=1e-10)
