"""GPU tests of the pair-list validity check (Sec. 2.3, Alg. alg_validity_check).

  * md_ldc_check gives the oracle's decision, member count and largest squared
    displacement bit for bit on the same positions (24 perturbed states of an
    864-particle fluid, valid and invalid, some and all particles members), and
    invalidates outright above ldc_max members;
  * md_step with the DUTC + LDC rule matches the oracle's run with the same
    rule (energies, positions, rebuild and check counts) and keeps fewer
    rebuilds than the half-skin rule;
  * no pair is ever missed: at every step of a hot run kept alive by the LDC,
    the forces equal the oracle's forces recomputed from scratch;
  * mixed precision with the rule tracks the FP64 oracle.
"""

import numpy as np
import pytest
import torch

import lj_inputs as li
from tests import gpu_util as G

pytestmark = pytest.mark.gpu

RC, RS = 2.5, 2.8


@pytest.fixture(autouse=True, scope="module")
def _cuda():
    assert torch.cuda.is_available()
    import paper_1012_2677_amd  # noqa: F401


def _perturbed(seed):
    amp = [0.02, 0.04, 0.07, 0.1][seed % 4]
    big = [0.0, 0.15, 0.3][(seed // 4) % 3]
    nbig = (seed % 3) + 1 if big else 0
    q0, L = li.jittered_fcc(6, amp=0.2, seed=seed)
    rng = np.random.default_rng(seed + 100)
    d = amp * rng.standard_normal(q0.shape)
    if nbig:
        idx = rng.choice(q0.shape[0], nbig, replace=False)
        d[idx] += big * rng.standard_normal((nbig, 3))
    return li.wrap_into_box(q0 + d, L), q0, L


def _gpu_check(q, qold, L, ldc_max):
    from paper_1012_2677_amd import _abi as A
    from paper_1012_2677_amd.engine import Workspace, make_params, stream_handle

    n = q.shape[0]
    p = make_params(n, L, rc=RC, rs=RS, ldc_max=ldc_max)
    ws = Workspace(p, "cuda:0")
    pos = torch.zeros((n, 4), dtype=torch.float64)
    pos[:, :3] = torch.from_numpy(q)
    pos = pos.to("cuda:0")
    ref = torch.from_numpy(np.ascontiguousarray(qold.T)).to("cuda:0")
    return A.md_ldc_check(p, pos.data_ptr(), ref.data_ptr(), ws.ptr, ws.nbytes, stream_handle("cuda:0"))


def test_ldc_check_matches_oracle_bitwise(ref):
    kinds = set()
    for seed in range(24):
        q, qold, L = _perturbed(seed)
        want = ref.ldc_check(q, qold, L, RC, RS, ldc_max=8192)
        got = _gpu_check(q, qold, L, 8192)
        assert got[0] == want[0] and got[1] == want[1], seed
        assert np.float64(got[2]).tobytes() == np.float64(want[2]).tobytes(), seed
        kinds.add((got[0], 0 < got[1] < q.shape[0]))
    assert {(True, True), (True, False), (False, False)} <= kinds


def test_ldc_check_member_cap():
    q, qold, L = _perturbed(17)         # 859 members, still valid
    ok, nld, _ = _gpu_check(q, qold, L, 8192)
    assert ok and 0 < nld < q.shape[0]
    ok2, nld2, _ = _gpu_check(q, qold, L, nld - 1)
    assert not ok2 and nld2 == nld
    ok3, nld3, _ = _gpu_check(q, qold, L, nld)
    assert ok3 and nld3 == nld


def _engine(q, v, L, **kw):
    from paper_1012_2677_amd import Engine

    return Engine(q, v, L, device="cuda:0", **kw)


def _min_image(d, L):
    return d - L * np.rint(d / L)


@pytest.mark.parametrize("T", [1.0, 3.0])
def test_run_with_dutc_ldc_matches_oracle(ref, T):
    q, L = li.fcc_lattice(10)
    v = li.maxwell_boltzmann(q.shape[0], T=T, seed=11)
    e = _engine(q, v, L, precision="fp64", rebuild_rule="dutc_ldc")
    log = e.step(120, sample_every=10)
    rq, rv, rlog, rreb, st = ref.run(q, v, L, 120, dt=0.005, sample_every=10, rule="dutc_ldc", full_stats=True)
    assert np.abs(log - rlog).max() <= 1e-10 * np.abs(rlog).max()
    assert np.abs(_min_image(e.positions() - rq, L)).max() < 1e-8
    assert e.rebuilds - 1 == rreb
    assert e.ldc_stats == (st["ldc_checks"], st["ldc_kept"])
    assert st["ldc_kept"] > 0
    half = ref.run(q, v, L, 120, dt=0.005, sample_every=10, full_stats=True)[4]
    assert rreb < half["rebuilds"]


def test_dutc_ldc_never_misses_a_pair(ref):
    q, L = li.fcc_lattice(8)
    v = li.maxwell_boltzmann(q.shape[0], T=3.0, seed=12)
    e = _engine(q, v, L, precision="fp64", rebuild_rule="dutc_ldc", resort_every=1)
    e.prepare()
    ids = np.arange(q.shape[0], dtype=np.int64)
    for _ in range(60):
        e.step(1)
        pos = e.positions()
        Fr, S, _, _, _ = ref.forces_sample(pos, L, ids)
        assert G.force_error(e.forces(), Fr, S) <= 1e-12
    checks, kept = e.ldc_stats
    assert kept > 0


def test_mixed_with_dutc_ldc_tracks_fp64(ref):
    q, L = li.fcc_lattice(10)
    v = li.maxwell_boltzmann(q.shape[0], T=1.0, seed=13)
    e = _engine(q, v, L, precision="mixed", rebuild_rule="dutc_ldc")
    log = e.step(100, sample_every=10)
    _, _, rlog, _ = ref.run(q, v, L, 100, dt=0.005, sample_every=10, rule="dutc_ldc")
    n = q.shape[0]
    assert np.abs(log[:, 3] - rlog[:, 3]).max() / n < 1e-5


def _sparse_pair_box():
    """A sparse box (L = 20, 7 cells of 2.857 per axis, 5 interior) holding a
    pair A-B listed across the x = 0 face (B in cell 0 at x = 0.3, A in the
    interior cell 1 at x = 3.0, distance 2.7 < rs), and isolated particles on
    a cubic lattice of spacing 4 kept more than 5 away from both."""
    L = 20.0
    g = np.arange(5) * 4.0 + 2.0
    lat = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    c = np.array([1.65, 10.0, 10.0])
    d = lat - c
    d -= L * np.rint(d / L)
    lat = lat[np.linalg.norm(d, axis=1) > 5.0]
    pair = np.array([[3.0, 10.0, 10.0], [0.3, 10.0, 10.0]])
    return np.concatenate([pair, lat]), L


@pytest.mark.parametrize("precision,layout,tile_cells", [
    ("fp64", "auto", 1), ("fp64", "slots", 0), ("mixed", "auto", 1), ("mixed", "slots", 0)])
def test_dutc_ldc_kept_list_after_large_moves_uses_minimum_images(ref, precision, layout, tile_cells):
    # Under DUTC + LDC a kept list can outlive moves larger than (cell side -
    # rc).  Here B crosses the x = 0 face (it is stored at x = L - 0.05) and A
    # moves 0.8 towards it, out of its interior build-time cell's margin: their
    # minimum-image distance is 2.25 < rc.  The check keeps the list (the pair
    # was listed, nobody else is near), so the force pass must take the minimum
    # image for the interior key A as well.
    q, L = _sparse_pair_box()
    n = q.shape[0]
    v = np.zeros_like(q)
    e = _engine(q, v, L, precision=precision, rebuild_rule="dutc_ldc", list_layout=layout,
                tile_cells=tile_cells, resort_every=1)
    e.prepare()
    e.step(1)
    assert int(e.state.list_tiled) == (1 if layout == "auto" else 0)
    r0, (c0, k0) = e.rebuilds, e.ldc_stats
    qold = e.positions()
    slot_of_id = torch.empty_like(e.id.long())
    slot_of_id[e.id.long()] = torch.arange(n, device=e.id.device)
    sa, sb = int(slot_of_id[0]), int(slot_of_id[1])
    e.pos[sa, 0] = 2.2
    e.pos[sb, 0] = L - 0.05
    qnew = e.positions()
    ok, members, _ = ref.ldc_check(qnew, qold, L)
    assert ok and members == n
    e.state.dutc_buffer = 0.0      # the DUTC buffer is used up: the check decides
    e.step(1)
    assert e.rebuilds == r0 and e.ldc_stats == (c0 + 1, k0 + 1)
    pos = e.positions()
    assert np.allclose(pos, qnew)
    Fr, S, _, _, _ = ref.forces_sample(pos, L, np.arange(n, dtype=np.int64))
    assert np.linalg.norm(Fr[0]) > 0.01 and S[0] > 0.01
    assert G.force_error(e.forces(), Fr, S) <= (1e-12 if precision == "fp64" else 1e-5)
