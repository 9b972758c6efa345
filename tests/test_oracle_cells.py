"""Pins of the oracle's grid and pair search (Sec. 2.2-2.3).

  * GridList (counting sort) equals numpy's stable argsort + bincount + cumsum
    of the cell labels (a library special case), is a permutation, is stable,
    and puts every particle inside its cell's bounds;
  * the grid pair search equals O(N^2) brute force on random, lattice and
    jittered inputs (exact set equality);
  * fcc at a = 2 has exactly 21 N pairs within 2.5 and within 2.8 (shells at
    sqrt2, 2, sqrt6 with 12 + 6 + 24 neighbours; sqrt8 > 2.8);
  * pairs placed so that r^2 lands one ulp below, on and above rs^2 are listed
    exactly when r^2 < rs^2, including across the periodic boundary;
  * ideal-gas pair count within a few standard deviations of N(N-1)/2 * v/V.
"""

import math

import numpy as np
import pytest

import lj_inputs as li


def _labels(q, L, nc):
    inv = np.array(nc, dtype=np.float64) / np.asarray(L, dtype=np.float64)
    c = np.minimum((q * inv).astype(np.int64), np.array(nc) - 1)
    return (c[:, 0] * nc[1] + c[:, 1]) * nc[2] + c[:, 2]


@pytest.mark.parametrize("case", ["fcc", "jitter", "uniform", "aniso"])
def test_gridlist_is_stable_counting_sort(ref, case):
    if case == "fcc":
        q, L = li.fcc_lattice(8)
        L = [L] * 3
    elif case == "jitter":
        q, L = li.jittered_fcc(8, amp=0.3)
        L = [L] * 3
    elif case == "uniform":
        L = [13.0, 13.0, 13.0]
        q = li.uniform_box(3000, 13.0)
    else:
        L = np.array([9.0, 14.0, 20.0])
        rng = np.random.default_rng(5)
        q = np.ascontiguousarray(rng.random((2500, 3)) * L)
    nc, ok = ref.cell_dims(L, 2.8)
    assert ok
    cell_of, count, start, order = ref.bin_cells(q, L, nc)
    lab = _labels(q, L, nc)
    ncell = int(np.prod(nc))
    assert np.array_equal(cell_of, lab)
    assert np.array_equal(count, np.bincount(lab, minlength=ncell))
    assert np.array_equal(start[:-1], np.concatenate([[0], np.cumsum(count)[:-1]]))
    assert start[-1] == q.shape[0]
    assert np.array_equal(order, np.argsort(lab, kind="stable"))
    assert np.array_equal(np.sort(order), np.arange(q.shape[0]))
    # every particle lies inside the box of its cell
    cs = np.asarray(L) / np.asarray(nc)
    c3 = np.stack(np.unravel_index(cell_of, nc), axis=1)
    assert np.all(q >= c3 * cs - 1e-12)
    assert np.all(q < (c3 + 1) * cs + 1e-12)


def test_cell_dims(ref):
    assert ref.cell_dims([20.0] * 3, 2.8) == ((7, 7, 7), True)
    assert ref.cell_dims([400.0] * 3, 2.8) == ((142, 142, 142), True)
    assert ref.cell_dims([640.0] * 3, 2.8) == ((228, 228, 228), True)
    assert ref.cell_dims([8.0] * 3, 2.8) == ((2, 2, 2), False)


def _as_set(p):
    return set(map(tuple, np.asarray(p).tolist()))


@pytest.mark.parametrize("case", [("fcc", 5), ("fcc", 6), ("jitter", 8), ("uniform", 4000), ("aniso", 2500)])
def test_grid_search_equals_brute_force(ref, case):
    kind, size = case
    if kind == "fcc":
        q, L = li.fcc_lattice(size)
        L = [L] * 3
    elif kind == "jitter":
        q, L = li.jittered_fcc(size, amp=0.25)
        L = [L] * 3
    elif kind == "uniform":
        L = [16.0] * 3
        q = li.uniform_box(size, 16.0)
    else:
        L = np.array([9.0, 14.0, 20.0])
        rng = np.random.default_rng(6)
        q = np.ascontiguousarray(rng.random((size, 3)) * L)
    pb = ref.pairs_brute(q, L, 2.8)
    pc = ref.pairs_cells(q, L, 2.8)
    assert len(pb) == len(pc)
    assert _as_set(pb) == _as_set(pc)
    assert np.all(pc[:, 0] < pc[:, 1])


@pytest.mark.parametrize("n_fcc", [5, 10])
def test_fcc_shell_count(ref, n_fcc):
    q, L = li.fcc_lattice(n_fcc)
    n = q.shape[0]
    assert len(ref.pairs_cells(q, L, 2.8)) == 21 * n
    assert len(ref.pairs_cells(q, L, 2.5)) == 21 * n
    # sqrt(8) = 2.828... is the next shell (12 more neighbours)
    assert len(ref.pairs_brute(q, L, 2.9)) == 27 * n


def predicate_r2(qi, qj, L):
    """The pinned pair predicate's r^2, evaluated with Python floats (IEEE double)
    and exact Fractions for the fused multiply-adds:
    d = q_j - q_i, d -= L * rint(d / L), r2 = fma(dz, dz, fma(dy, dy, dx * dx))."""
    from fractions import Fraction as Fr

    d = []
    for a in range(3):
        x = qj[a] - qi[a]
        k = round(x * (1.0 / L))  # round half to even, like rint
        d.append(x - L * k)
    inner = float(Fr(d[1]) * Fr(d[1]) + Fr(d[0] * d[0]))
    return float(Fr(d[2]) * Fr(d[2]) + Fr(inner))


ADV_L = 80.0


def adversarial_pairs(rs=2.8, L=ADV_L):
    """Particle pairs whose r^2 falls exactly on rs^2 and up to three ulps below
    and above it, some straddling the periodic boundary in x, y or z.

    The "free" coordinate that is tuned ulp by ulp is kept near 1 with a small
    displacement, so one ulp step moves r^2 by less than one ulp of rs^2 and
    every target is reachable.  Pairs are more than rs apart from each other.
    Returns (q[N,3], expected set of listed pairs (i, j), i < j).
    """
    rs2 = rs * rs
    targets = [rs2]
    for _ in range(3):
        targets.append(float(np.nextafter(targets[-1], 0.0)))
    t = rs2
    for _ in range(3):
        t = float(np.nextafter(t, 10.0))
        targets.append(t)
    q = []
    expect = set()
    for ti, target in enumerate(targets):
        for kind in ("inner", "xwrap", "ywrap", "zwrap"):
            s1 = 10.0 + 8.0 * ti          # 10 .. 58
            if kind == "inner":
                qi, qj, free = [s1, 1.0, 20.0], [s1 + 2.77, 1.3, 20.0], 1
            elif kind == "xwrap":
                qi, qj, free = [L - 1.3, 1.0, s1], [1.47, 1.3, s1], 1
            elif kind == "ywrap":
                qi, qj, free = [1.0, L - 1.3, s1 + 4.0], [1.3, 1.47, s1 + 4.0], 0
            else:
                qi, qj, free = [1.0, s1, L - 1.3], [1.3, s1, 1.47], 0
            # start from the real-valued solution for the free coordinate
            other = 0.0
            for ax in range(3):
                d = qj[ax] - qi[ax]
                d = d - L * round(d * (1.0 / L))
                if ax != free:
                    other += d * d
            qj[free] = qi[free] + float(np.sqrt(target - other))
            found = False
            for _ in range(100000):
                r2 = predicate_r2(qi, qj, L)
                if r2 == target:
                    found = True
                    break
                qj[free] = float(np.nextafter(qj[free], 1e3 if r2 < target else -1e3))
            assert found, (kind, target)
            assert all(0.0 <= x < L for x in qi + qj)
            i = len(q)
            q.append(qi)
            q.append(qj)
            if target < rs2:
                expect.add((i, i + 1))
    q = np.array(q, dtype=np.float64)
    # pairs must not see each other
    for a in range(0, len(q), 2):
        for b in range(0, len(q)):
            if b in (a, a + 1):
                continue
            assert predicate_r2(list(q[a]), list(q[b]), L) > 3.0 * 3.0
            assert predicate_r2(list(q[a + 1]), list(q[b]), L) > 3.0 * 3.0
    return q, expect


def test_adversarial_ulp_pairs(ref):
    q, expect = adversarial_pairs()
    L = [ADV_L] * 3
    assert len(q) == 56 and len(expect) == 12
    pb = _as_set(ref.pairs_brute(q, L, 2.8))
    pc = _as_set(ref.pairs_cells(q, L, 2.8))
    assert pb == expect
    assert pc == expect


def test_ideal_gas_pair_count(ref):
    L = 30.0
    n = 13500  # rho = 0.5
    q = li.uniform_box(n, L, seed=11)
    m = len(ref.pairs_cells(q, [L] * 3, 2.8))
    p = (4.0 / 3.0) * math.pi * 2.8 ** 3 / L ** 3
    mean = n * (n - 1) / 2 * p
    assert abs(m - mean) < 6 * math.sqrt(mean)
    # about 23 half-pairs per particle at rho = 0.5 within rs = 2.8
    assert 22.0 < m / n < 24.0
