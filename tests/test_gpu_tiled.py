"""GPU tests of the tiled list layout of the simulation state (FP64 and mixed).

The state's list is tiled when the slots are in cell order: entries are 16-bit
indices into the staged neighbourhood of the key's tile, and the force pass
reads partners from LDS.  These tests check:

  * when the library chooses the tiled layout, and that it falls back to slot
    entries when a tile's neighbourhood is too large to stage;
  * index work, bit-exact: every tiled row, decoded on the host from the
    documented layout, equals the slot-layout row of the same key entry by
    entry, and both equal the oracle's neighbour sets;
  * forces after md_prepare against the FP64 oracle (1e-12 in FP64, 1e-5 in
    mixed, of the pair-force scale) for several tile lengths, including tiles
    that wrap the box in z;
  * runs with the tiled list match the oracle's run (FP64: energy log to
    1e-10 relative, same rebuilds; mixed: energy per particle to 1e-5) and the
    slot-layout run;
  * FP64 tiles on the box faces after particles crossed the faces since the
    build;
  * anisotropic boxes with 3-cell axes (3 neighbour columns, one-cell tiles);
  * crowded cells (a clump, a rho = 1.6 box), where the build re-reads its
    candidates from memory, and a half-empty box (tiles without keys): rows
    still equal the slot rows and the oracle's.
"""

import numpy as np
import pytest
import torch

import lj_inputs as li
from tests import gpu_util as G

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True, scope="module")
def _cuda():
    assert torch.cuda.is_available()
    import paper_1012_2677_amd  # noqa: F401


def _engine(q, v, L, **kw):
    from paper_1012_2677_amd import Engine

    return Engine(q, v, L, device="cuda:0", **kw)


def _jittered(n_fcc, seed, rho=0.5, amp=0.15):
    q, L = li.jittered_fcc(n_fcc, amp=amp, seed=seed, rho=rho)
    q, _, _ = li.shuffle_labels(q, seed=seed)
    return q, L


def test_layout_selection():
    q, L = li.fcc_lattice(10)
    v = li.maxwell_boltzmann(q.shape[0], seed=0)
    for precision, cap in (("mixed", 3500), ("fp64", 1950)):
        e = _engine(q, v, L, precision=precision)
        e.prepare()
        assert int(e.state.list_tiled) == 1
        assert int(e.state.tile_cells) == 5          # clipped to nz - 2 with 7 cells per axis
        assert 0 < int(e.state.tile_stage) <= cap
    for kw in (dict(precision="fp64", resort_every=0), dict(precision="mixed", resort_every=0),
               dict(precision="mixed", list_layout="slots"), dict(precision="fp64", list_layout="slots"),
               dict(precision="mixed", cell_stride=1153)):
        f = _engine(q, v, L, **kw)
        f.prepare()
        assert int(f.state.list_tiled) == 0, kw


@pytest.mark.parametrize("waves", ["cell", "tile"])
@pytest.mark.parametrize("precision,tile_cells", [("mixed", 0), ("mixed", 1), ("mixed", 2), ("mixed", 3),
                                                  ("fp64", 0), ("fp64", 4)])
def test_tiled_rows_equal_slot_rows_and_oracle(ref, precision, tile_cells, waves):
    # both ways of spreading the build (a wave per cell, a wave per tile)
    q, L = _jittered(10, seed=11)
    v = li.maxwell_boltzmann(q.shape[0], seed=11)
    t = _engine(q, v, L, precision=precision, tile_cells=tile_cells, build_waves=waves)
    s = _engine(q, v, L, precision=precision, list_layout="slots")
    t.prepare()
    s.prepare()
    assert int(t.state.list_tiled) == 1 and int(s.state.list_tiled) == 0
    assert torch.equal(t.id, s.id)
    n = q.shape[0]
    slots = np.arange(n)
    kt, pt = G.rows_for_slots_state(t, slots)
    ks, ps = G.rows_for_slots_state(s, slots)
    assert np.array_equal(kt, ks)
    assert np.array_equal(pt, ps)
    # and the oracle's neighbour sets, by particle id
    ids = t.id.cpu().numpy()
    qp = t.positions()
    rows = ref.neighbors_sample(qp, L, ids, rs=2.8)
    for k in range(n):
        assert np.array_equal(np.sort(ids[pt[kt == k]]), rows[k])


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("tile_cells", [0, 1, 2, 4, 5, 1023])
def test_tiled_forces_match_oracle(ref, precision, tile_cells):
    q, L = _jittered(10, seed=3)
    v = li.maxwell_boltzmann(q.shape[0], seed=3)
    e = _engine(q, v, L, precision=precision, tile_cells=tile_cells)
    e.prepare()
    assert int(e.state.list_tiled) == 1
    idx = np.arange(q.shape[0], dtype=np.int64)
    Fr, S, pe_i, w_i, _ = ref.forces_sample(e.positions(), L, idx)
    en = e.energies()   # per-particle shares of the oracle sum to the totals
    if precision == "fp64":
        assert G.force_error(e.forces(), Fr, S) <= 1e-12
        assert en[1] == pytest.approx(pe_i.sum(), rel=1e-12)
        assert en[2] == pytest.approx(w_i.sum(), rel=1e-12)
    else:
        assert G.force_error(e.forces(), Fr, S) <= 1e-5
        assert abs(en[1] - pe_i.sum()) / q.shape[0] < 1e-5
        assert abs(en[2] - w_i.sum()) / q.shape[0] < 1e-4


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_tiled_run_tracks_oracle_and_slot_run(ref, precision):
    q, L = li.fcc_lattice(10)
    v = li.maxwell_boltzmann(q.shape[0], T=1.0, seed=0)
    t = _engine(q, v, L, precision=precision)
    s = _engine(q, v, L, precision=precision, list_layout="slots")
    lt = t.step(100, sample_every=10)
    ls = s.step(100, sample_every=10)
    assert int(t.state.list_tiled) == 1
    rq, _, rlog, rreb = ref.run(q, v, L, 100, dt=0.005, sample_every=10)
    n = q.shape[0]
    if precision == "fp64":
        for log in (lt, ls):
            assert np.abs(log - rlog).max() <= 1e-10 * np.abs(rlog).max()
        d = t.positions() - rq
        assert np.abs(d - L * np.rint(d / L)).max() < 1e-8
        assert t.rebuilds - 1 == rreb
    else:
        for log in (lt, ls):
            assert np.abs(log[:, 3] - rlog[:, 3]).max() / n < 1e-5
            assert np.abs(log[:, 1] - rlog[:, 1]).max() / n < 1e-5
        assert np.abs(lt - ls).max() / n < 1e-5
    assert t.rebuilds == s.rebuilds


@pytest.mark.parametrize("tile_cells", [3, 4])
def test_fp64_boundary_tiles_after_particles_cross_the_box_faces(ref, tile_cells):
    # 11 cells per axis, tiles of 3 and 4 cells (the z faces cut different
    # tiles).  Particles within 0.02 of a face in x or z are sent across it, so
    # that two steps later (no rebuild) the list holds partners whose
    # coordinates wrapped since the build; the step's forces and those of the
    # energy pass match the oracle at the current positions.
    q, L = _jittered(16, seed=5, amp=0.05)   # no close pairs: no rebuild in two steps
    n = q.shape[0]
    v = li.maxwell_boltzmann(n, T=1.0, seed=5)
    moved = 0
    for ax in (0, 2):
        lo, hi = q[:, ax] < 0.02, q[:, ax] > L - 0.02
        v[lo, ax] = -2.0
        v[hi, ax] = 2.0
        moved += int(lo.sum() + hi.sum())
    assert moved > 100
    e = _engine(q, v, L, precision="fp64", tile_cells=tile_cells)
    e.step(2)
    assert int(e.state.list_tiled) == 1 and int(e.state.tile_cells) == tile_cells
    assert e.rebuilds == 1
    crossed = np.abs(e.positions() - q).max(axis=1) > 0.5 * L
    assert crossed.sum() > 100
    idx = np.arange(n, dtype=np.int64)
    Fr, S, pe_i, w_i, _ = ref.forces_sample(e.positions(), L, idx)
    assert G.force_error(e.forces(), Fr, S) <= 1e-12
    en = e.energies()
    assert G.force_error(e.forces(), Fr, S) <= 1e-12
    assert en[1] == pytest.approx(pe_i.sum(), rel=1e-12)
    assert en[2] == pytest.approx(w_i.sum(), rel=1e-12)


@pytest.mark.parametrize("precision,tile_cells", [("mixed", 18), ("fp64", 10)])
def test_oversized_tiles_fall_back_to_slot_entries(ref, precision, tile_cells):
    # a dense solid (rho = 1) with long tiles: the staged neighbourhood of a
    # tile (~9 * (tile_cells + 2) cells * 23 particles) exceeds what the force
    # pass stages (3500 particles in mixed, 1950 in FP64)
    q, L = li.fcc_lattice(36, rho=1.0)
    v = li.maxwell_boltzmann(q.shape[0], T=0.2, seed=1)
    e = _engine(q, v, L, precision=precision, tile_cells=tile_cells)
    e.prepare()
    assert int(e.state.list_tiled) == 0
    e.step(5)
    idx = np.random.default_rng(0).choice(q.shape[0], 300, replace=False).astype(np.int64)
    Fr, S, _, _, _ = ref.forces_sample(e.positions(), L, idx)
    assert G.force_error(e.forces()[idx], Fr, S) <= (1e-12 if precision == "fp64" else 1e-5)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("cells", [(5, 8, 14), (14, 5, 5), (5, 5, 20)])
def test_tiled_anisotropic_boxes(ref, precision, cells):
    # 3-column axes (the neighbour columns cx - 1 and cx + 1 are the only two
    # others), a 3-cell z axis (tiles of one cell), long z columns; jittered
    q, L = li.fcc_lattice_box(*cells)
    rng = np.random.default_rng(sum(cells))
    q = q + rng.normal(0.0, 0.1, q.shape)
    q = q - np.asarray(L) * np.floor(q / np.asarray(L))
    v = li.maxwell_boltzmann(q.shape[0], seed=1)
    t = _engine(q, v, L, precision=precision)
    s = _engine(q, v, L, precision=precision, list_layout="slots")
    t.prepare()
    s.prepare()
    assert int(t.state.list_tiled) == 1
    slots = np.arange(q.shape[0])
    kt, pt = G.rows_for_slots_state(t, slots)
    ks, ps = G.rows_for_slots_state(s, slots)
    assert np.array_equal(kt, ks) and np.array_equal(pt, ps)
    idx = np.arange(q.shape[0], dtype=np.int64)
    Fr, S, _, _, _ = ref.forces_sample(t.positions(), L, idx)
    assert G.force_error(t.forces(), Fr, S) <= (1e-12 if precision == "fp64" else 1e-5)
    # a short run keeps matching the slot-entry run
    lt = t.step(20, sample_every=10)
    ls = s.step(20, sample_every=10)
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert np.abs(lt - ls).max() <= tol * max(1.0, np.abs(ls).max())


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_standalone_force_pass_refuses_a_tiled_state_list(precision):
    # the library marks the state's list as tiled; md_forces then returns
    # MD_ERR_ARG instead of reading tile offsets as slots.  A slot-layout
    # state list is accepted and gives the state's own forces.
    from paper_1012_2677_amd import _abi as A
    from paper_1012_2677_amd.engine import Workspace

    q, L = _jittered(8, seed=5)
    v = li.maxwell_boltzmann(q.shape[0], seed=5)
    dt = torch.float32 if precision == "mixed" else torch.float64
    for layout, tiled in (("auto", 1), ("slots", 0)):
        e = _engine(q, v, L, precision=precision, list_layout=layout)
        e.prepare()
        assert int(e.state.list.tiled) == tiled == int(e.state.list_tiled)
        ws = Workspace(e.params, G.device())
        F = torch.zeros((3, q.shape[0]), dtype=dt, device=G.device())
        args = (e.params, e.state.pos, e.state.cells, e.state.list, F.data_ptr(), None, ws.ptr, ws.nbytes,
                e.stream())
        if tiled:
            with pytest.raises(A.MdError) as err:
                A.md_forces(*args)
            assert err.value.code == A.MD_ERR_ARG
            continue
        A.md_forces(*args)
        torch.cuda.synchronize()
        got = F.double().cpu().numpy()
        want = e.force.double().cpu().numpy()
        tol = 1e-12 if precision == "fp64" else 1e-5
        assert np.abs(got - want).max() <= tol * np.abs(want).max()


@pytest.mark.parametrize("waves", ["cell", "tile"])
@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("name", ["clump", "dense", "slab"])
def test_tiled_rows_in_crowded_or_empty_cells(ref, precision, name, waves):
    # cells beyond the build's LDS key buffer and neighbourhoods beyond its
    # register chunks (the tiled rows come from the path that re-reads the
    # candidates), or empty cells and tiles without keys: rows must still
    # equal the slot rows and the oracle's sets
    from tests.test_gpu_parity import _case

    q, L = _case(name)
    v = np.zeros_like(q)
    t = _engine(q, v, L, precision=precision, build_waves=waves)
    s = _engine(q, v, L, precision=precision, list_layout="slots")
    t.prepare()
    s.prepare()
    assert int(t.state.list_tiled) == 1 and int(s.state.list_tiled) == 0
    assert torch.equal(t.id, s.id)
    n = q.shape[0]
    slots = np.arange(n)
    kt, pt = G.rows_for_slots_state(t, slots)
    ks, ps = G.rows_for_slots_state(s, slots)
    assert np.array_equal(kt, ks)
    assert np.array_equal(pt, ps)
    ids = t.id.cpu().numpy()
    rows = ref.neighbors_sample(t.positions(), L, ids, rs=2.8)
    for k in range(n):
        assert np.array_equal(np.sort(ids[pt[kt == k]]), rows[k])
    if precision == "fp64":
        idx = np.arange(n, dtype=np.int64)
        Fr, S, _, _, _ = ref.forces_sample(t.positions(), L, idx)
        assert G.force_error(t.forces(), Fr, S) <= 1e-12


def _radius_pairs(rs=2.8, L=48.0):
    """Pairs in interior cells whose pinned r^2 lies within three ulp steps of
    the free coordinate below and above rs^2 (r^2 < rs^2 listed), along x, y, z
    and a diagonal, each pair at its own anchor more than rs from the others."""
    from tests.test_oracle_cells import predicate_r2

    rs2 = rs * rs
    dirs = [((2.77, 0.3, 0.2), 0), ((0.3, 2.77, 0.1), 1), ((0.2, 0.1, 2.78), 2), ((1.6, 1.6, 1.62), 0)]
    anchors = iter([(x, y, z) for x in (6.0, 14.0, 22.0, 30.0, 38.0) for y in (6.0, 14.0, 22.0, 30.0, 38.0)
                    for z in (6.0, 14.0, 22.0, 30.0)])
    q, expect = [], set()
    for d, free in dirs:
        a0 = next(anchors)
        qi = list(a0)
        qj = [a0[k] + d[k] for k in range(3)]
        other = sum((qj[k] - qi[k]) ** 2 for k in range(3) if k != free)
        qj[free] = qi[free] + float(np.sqrt(rs2 - other))
        # step the free coordinate to the last value with r^2 < rs^2
        while predicate_r2(qi, qj, L) >= rs2:
            qj[free] = float(np.nextafter(qj[free], -1e3))
        while True:
            nxt = float(np.nextafter(qj[free], 1e3))
            if predicate_r2(qi, qj[:free] + [nxt] + qj[free + 1:], L) >= rs2:
                break
            qj[free] = nxt
        vals = [qj[free]]
        for _ in range(2):
            vals.insert(0, float(np.nextafter(vals[0], -1e3)))
        for _ in range(3):
            vals.append(float(np.nextafter(vals[-1], 1e3)))
        for v in vals:
            a = list(next(anchors))
            pi = [a[k] for k in range(3)]
            pj = [a[k] + (qj[k] - qi[k]) for k in range(3)]
            # the same offset from another anchor: re-tune the free coordinate's
            # difference exactly (anchors are integers, so the offsets carry over)
            pj[free] = a[free] + (v - qi[free])
            i = len(q)
            q += [pi, pj]
            if predicate_r2(pi, pj, L) < rs2:
                expect.add((i, i + 1))
    q = np.array(q, dtype=np.float64)
    for p in range(0, len(q), 2):
        r2 = [predicate_r2(list(q[p]), list(q[b]), L) for b in range(len(q)) if b not in (p, p + 1)]
        assert min(r2) > 3.0 * 3.0
    return q, expect, L


@pytest.mark.parametrize("waves", ["cell", "tile"])
def test_tiled_rows_decide_pairs_at_the_search_radius_bit_exactly(waves):
    # interior pairs a few ulps of r^2 inside and outside rs^2 (the tiled
    # build's own code path, with both ways of spreading its waves) must be
    # decided as the pinned predicate decides them, as the slot rows are
    from tests.test_oracle_cells import predicate_r2

    q, expect, L = _radius_pairs()
    n = q.shape[0]
    rs2 = 2.8 * 2.8
    near = sum(1 for p in range(0, n, 2) if abs(predicate_r2(list(q[p]), list(q[p + 1]), L) - rs2) < 1e-13)
    assert len(expect) >= 8 and n - 2 * len(expect) >= 16 and near >= 16
    for precision in ("fp64", "mixed"):
        t = _engine(q, np.zeros_like(q), L, precision=precision, build_waves=waves)
        s = _engine(q, np.zeros_like(q), L, precision=precision, list_layout="slots")
        t.prepare()
        s.prepare()
        assert int(t.state.list_tiled) == 1
        slots = np.arange(n)
        kt, pt = G.rows_for_slots_state(t, slots)
        ks, ps = G.rows_for_slots_state(s, slots)
        assert np.array_equal(kt, ks) and np.array_equal(pt, ps)
        ids = t.id.cpu().numpy()
        got = {(int(min(ids[k], ids[p])), int(max(ids[k], ids[p]))) for k, p in zip(kt, pt)}
        assert got == expect, precision
