"""CPU oracle for the Lennard-Jones MD hot path (Watanabe, Suzuki and Ito).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  It shares no code with the GPU
path.  Numerics live in the plain C file mdref.c (FP64 pair terms, long-double
sums); this module only marshals numpy arrays into it.

Arrays are numpy float64 of shape (N, 3) (the paper's q[N]); box L is a length-3
sequence.  Functions and the passages they follow:

  lj_coeffs, pair           Sec. 2.1, eq. lj_cutoff (truncated potential)
  cell_dims, bin_cells      Sec. 2.2 (inexclusive grid, GridList counting sort)
  pairs_brute, pairs_cells  Sec. 2.2-2.3 (pair finding; 13-cell half stencil)
  forces, forces_pairs      Sec. 3.1-3.2 (force loop, strict r < rc)
  forces_sample             per-particle forces by a direct 27-cell scan
  neighbors_sample          per-particle neighbour sets within rs
  run                       Sec. 2.3 + 4.5 (bookkeeping rule; velocity Verlet)
  ldc_check                 Sec. 2.3, Alg. alg_validity_check (large-displacement check)
  hvp, param_grad           Hessian-vector product / parameter derivatives
  traj_mean_pe_grad         checkpointed reverse sweep of velocity Verlet

Parity status: every function here is pinned by tests in tests/test_oracle_*.py
(closed forms in exact rational arithmetic, library special cases, brute force,
invariants and finite differences).  See each test module's header.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmdref.so")
_lib = None

_d = C.c_double
_i64 = C.c_int64
_pd = C.POINTER(C.c_double)
_pi32 = C.POINTER(C.c_int32)
_pi64 = C.POINTER(C.c_int64)
_pint = C.POINTER(C.c_int)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(
        os.path.join(_HERE, "mdref.c")
    ):
        from . import build as _b

        _b.build()
    lib = C.CDLL(_LIB_PATH)
    sig = {
        "mdref_lj_coeffs": (None, [_d, _d, _pd, _pd]),
        "mdref_pair": (None, [_d, _d, _d, _d, _pd, _pd]),
        "mdref_pair_derivs": (None, [_d, _d, _d, _d, _pd, _pd, _pd]),
        "mdref_pair_r2": (_d, [_pd, _pd, _pd]),
        "mdref_cell_dims": (C.c_int, [_pd, _d, _pint]),
        "mdref_bin": (None, [_i64, _pd, _pd, _pint, _pi32, _pi32, _pi32, _pi32]),
        "mdref_pairs_brute": (_i64, [_i64, _pd, _pd, _d, _i64, _pi32, _pi32]),
        "mdref_pairs_cells": (_i64, [_i64, _pd, _pd, _d, _i64, _pi32, _pi32]),
        "mdref_forces_pairs": (None, [_i64, _pd, _pd, _d, _d, _d, _i64, _pi32, _pi32, _pd, _pd, _pd]),
        "mdref_forces": (C.c_int, [_i64, _pd, _pd, _d, _d, _d, _d, _pd, _pd, _pd]),
        "mdref_forces_sample": (None, [_i64, _pd, _pd, _d, _d, _d, _d, _pint, _pi32, _pi32, _pi32,
                                       _i64, _pi64, _pd, _pd, _pd, _pd, _pi32]),
        "mdref_neighbors_sample": (_i64, [_pd, _pd, _d, _pint, _pi32, _pi32, _pi32, _i64, _pi64,
                                          _i64, _pi32, _pi32]),
        "mdref_run": (C.c_int, [_i64, _pd, _pd, _pd, _d, _d, _d, _d, _d, _i64, _i64, _pd, _pi64, C.c_int32,
                                _i64]),
        "mdref_ldc_check": (C.c_int, [_i64, _pd, _pd, _pd, _d, _d, _i64, _pi64, _pd]),
        "mdref_hvp": (None, [_i64, _pd, _pd, _d, _d, _d, _d, _pd, _pd, _pd]),
        "mdref_param_grad": (None, [_i64, _pd, _pd, _d, _d, _d, _d, _pd]),
        "mdref_traj_mean_pe_grad": (C.c_int, [_i64, _pd, _pd, _pd, _d, _d, _d, _d, _d, _i64, _i64,
                                              _pd, _pd, _pd]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _p(a, t=_pd):
    return a.ctypes.data_as(t)


def _q(q):
    q = np.ascontiguousarray(q, dtype=np.float64)
    assert q.ndim == 2 and q.shape[1] == 3
    return q


def _box(L):
    return np.ascontiguousarray(np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)).copy())


def lj_coeffs(sigma=1.0, rc=2.5):
    c2, c0 = C.c_double(), C.c_double()
    _load().mdref_lj_coeffs(sigma, rc, C.byref(c2), C.byref(c0))
    return c2.value, c0.value


def pair(r2, eps=1.0, sigma=1.0, rc=2.5):
    """(V, g) at squared distance r2 (no cutoff test)."""
    V, g = C.c_double(), C.c_double()
    _load().mdref_pair(float(r2), eps, sigma, rc, C.byref(V), C.byref(g))
    return V.value, g.value


def pair_derivs(r2, eps=1.0, sigma=1.0, rc=2.5):
    """(V'', dV/dsigma, dg/dsigma) at squared distance r2."""
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    _load().mdref_pair_derivs(float(r2), eps, sigma, rc, C.byref(a), C.byref(b), C.byref(c))
    return a.value, b.value, c.value


def pair_r2(qi, qj, L):
    qi = np.ascontiguousarray(qi, dtype=np.float64)
    qj = np.ascontiguousarray(qj, dtype=np.float64)
    return _load().mdref_pair_r2(_p(qi), _p(qj), _p(_box(L)))


def cell_dims(L, rs):
    nc = np.zeros(3, dtype=np.intc)
    ok = _load().mdref_cell_dims(_p(_box(L)), rs, _p(nc, _pint))
    return tuple(int(x) for x in nc), bool(ok)


def bin_cells(q, L, nc):
    """GridList of q: (cell_of[n], count[nc], start[nc+1], order[n]) int32."""
    q = _q(q)
    n = q.shape[0]
    ncv = np.asarray(nc, dtype=np.intc)
    ncell = int(np.prod(ncv.astype(np.int64)))
    cell_of = np.empty(n, np.int32)
    count = np.empty(ncell, np.int32)
    start = np.empty(ncell + 1, np.int32)
    order = np.empty(n, np.int32)
    _load().mdref_bin(n, _p(q), _p(_box(L)), _p(ncv, _pint), _p(cell_of, _pi32), _p(count, _pi32),
                      _p(start, _pi32), _p(order, _pi32))
    return cell_of, count, start, order


def _pairs(fn, q, L, rs):
    q = _q(q)
    n = q.shape[0]
    cap = 32 * n + 64
    while True:
        pi = np.empty(cap, np.int32)
        pj = np.empty(cap, np.int32)
        m = fn(n, _p(q), _p(_box(L)), rs, cap, _p(pi, _pi32), _p(pj, _pi32))
        if m < 0:
            raise ValueError("box has fewer than 3 cells per axis")
        if m <= cap:
            return np.stack([pi[:m], pj[:m]], axis=1)
        cap = int(m)


def pairs_brute(q, L, rs):
    """All pairs i < j with minimum-image r^2 < rs^2, as an (m, 2) int32 array."""
    return _pairs(_load().mdref_pairs_brute, q, L, rs)


def pairs_cells(q, L, rs):
    """Same set via the grid search (pairs as (min id, max id))."""
    return _pairs(_load().mdref_pairs_cells, q, L, rs)


def forces_pairs(q, L, pairs, eps=1.0, sigma=1.0, rc=2.5):
    q = _q(q)
    pairs = np.ascontiguousarray(pairs, dtype=np.int32)
    pi = np.ascontiguousarray(pairs[:, 0])
    pj = np.ascontiguousarray(pairs[:, 1])
    F = np.empty_like(q)
    pe, w = C.c_double(), C.c_double()
    _load().mdref_forces_pairs(q.shape[0], _p(q), _p(_box(L)), eps, sigma, rc, pi.shape[0],
                               _p(pi, _pi32), _p(pj, _pi32), _p(F), C.byref(pe), C.byref(w))
    return F, pe.value, w.value


def forces(q, L, eps=1.0, sigma=1.0, rc=2.5, rs=2.8):
    """(F[n,3], PE, W) summed over all pairs with r < rc."""
    q = _q(q)
    F = np.empty_like(q)
    pe, w = C.c_double(), C.c_double()
    rc_ = _load().mdref_forces(q.shape[0], _p(q), _p(_box(L)), eps, sigma, rc, rs, _p(F),
                               C.byref(pe), C.byref(w))
    if rc_ != 0:
        raise ValueError("box too small for the cutoff")
    return F, pe.value, w.value


def forces_sample(q, L, idx, eps=1.0, sigma=1.0, rc=2.5, rs=2.8, grid=None):
    """Per sampled particle: (F[s,3], S[s], pe_i[s], w_i[s], nb_i[s]) by a direct
    scan of the 27 surrounding cells.  grid = (nc, count, start, order) may be
    passed to reuse a GridList."""
    q = _q(q)
    if grid is None:
        nc, _ = cell_dims(L, rs)
        _, count, start, order = bin_cells(q, L, nc)
    else:
        nc, count, start, order = grid
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    s = idx.shape[0]
    F = np.empty((s, 3))
    S = np.empty(s)
    pe = np.empty(s)
    w = np.empty(s)
    nb = np.empty(s, np.int32)
    ncv = np.asarray(nc, dtype=np.intc)
    _load().mdref_forces_sample(q.shape[0], _p(q), _p(_box(L)), eps, sigma, rc, rs, _p(ncv, _pint),
                                _p(count, _pi32), _p(start, _pi32), _p(order, _pi32), s,
                                _p(idx, _pi64), _p(F), _p(S), _p(pe), _p(w), _p(nb, _pi32))
    return F, S, pe, w, nb


def neighbors_sample(q, L, idx, rs=2.8, grid=None):
    """List of sorted int32 arrays: the ids within rs of each sampled particle."""
    q = _q(q)
    if grid is None:
        nc, _ = cell_dims(L, rs)
        _, count, start, order = bin_cells(q, L, nc)
    else:
        nc, count, start, order = grid
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    s = idx.shape[0]
    cap = 128 * s + 64
    rowlen = np.empty(s, np.int32)
    ncv = np.asarray(nc, dtype=np.intc)
    while True:
        out = np.empty(cap, np.int32)
        m = _load().mdref_neighbors_sample(_p(q), _p(_box(L)), rs, _p(ncv, _pint), _p(count, _pi32),
                                           _p(start, _pi32), _p(order, _pi32), s, _p(idx, _pi64),
                                           cap, _p(rowlen, _pi32), _p(out, _pi32))
        if m <= cap:
            break
        cap = int(m)
    ends = np.cumsum(rowlen)
    return [out[e - l:e] for e, l in zip(ends, rowlen)]


RULES = {"half_skin": 0, "dutc_ldc": 1}


def run(q, v, L, nsteps, dt=0.005, eps=1.0, sigma=1.0, rc=2.5, rs=2.8, sample_every=1, rule="half_skin",
        ldc_max=8192, full_stats=False):
    """Velocity-Verlet NVE run.  rule "half_skin": rebuild when some particle
    moved more than (rs - rc)/2 since the last build; "dutc_ldc": the DUTC and
    large-displacement check of Alg. alg_validity_check with at most ldc_max
    members.  Returns (q, v, log[k, 4] = (KE, PE, W, E), rebuilds), plus a dict
    of statistics when full_stats."""
    q = _q(q).copy()
    v = _q(v).copy()
    k = nsteps // sample_every if sample_every > 0 else 0
    log = np.zeros((max(k, 1), 4))
    stats = np.zeros(4, np.int64)
    rc_ = _load().mdref_run(q.shape[0], _p(q), _p(v), _p(_box(L)), eps, sigma, rc, rs, dt, nsteps,
                            sample_every, _p(log), _p(stats, _pi64), RULES[rule], int(ldc_max))
    if rc_ != 0:
        raise ValueError("oracle run failed (geometry)")
    if full_stats:
        return q, v, log[:k], int(stats[0]), dict(rebuilds=int(stats[0]), pairs=int(stats[1]),
                                                  ldc_checks=int(stats[2]), ldc_kept=int(stats[3]))
    return q, v, log[:k], int(stats[0])


def ldc_check(q, qold, L, rc=2.5, rs=2.8, ldc_max=8192):
    """Large-displacement check of a list built at qold, at positions q
    (Alg. alg_validity_check).  Returns (valid, members, max squared
    displacement)."""
    q, qold = _q(q), _q(qold)
    nld = np.zeros(1, np.int64)
    dm2 = np.zeros(1)
    ok = _load().mdref_ldc_check(q.shape[0], _p(q), _p(qold), _p(_box(L)), rc, rs, int(ldc_max),
                                 _p(nld, _pi64), _p(dm2))
    return bool(ok), int(nld[0]), float(dm2[0])


def hvp(q, L, u, eps=1.0, sigma=1.0, rc=2.5, rs=2.8):
    """(H u [n,3], u . dF/d(eps, sigma) [2])."""
    q = _q(q)
    u = _q(u)
    Hu = np.empty_like(q)
    dp = np.empty(2)
    _load().mdref_hvp(q.shape[0], _p(q), _p(_box(L)), eps, sigma, rc, rs, _p(u), _p(Hu), _p(dp))
    return Hu, dp


def param_grad(q, L, eps=1.0, sigma=1.0, rc=2.5, rs=2.8):
    """(dU/deps, dU/dsigma)."""
    q = _q(q)
    dU = np.empty(2)
    _load().mdref_param_grad(q.shape[0], _p(q), _p(_box(L)), eps, sigma, rc, rs, _p(dU))
    return dU


def traj_mean_pe_grad(q0, v0, L, K, ckpt=20, dt=0.005, eps=1.0, sigma=1.0, rc=2.5, rs=2.8):
    """(O, dO/dq0 [n,3], dO/d(eps, sigma) [2]) for O = mean_{k=1..K} U(q_k)."""
    q0 = _q(q0)
    v0 = _q(v0)
    O = C.c_double()
    gq = np.empty_like(q0)
    gp = np.empty(2)
    rc_ = _load().mdref_traj_mean_pe_grad(q0.shape[0], _p(q0), _p(v0), _p(_box(L)), eps, sigma, rc,
                                          rs, dt, K, ckpt, C.byref(O), _p(gq), _p(gp))
    if rc_ != 0:
        raise ValueError("oracle gradient failed")
    return O.value, gq, gp
