"""GPU tests of the whole step loop (md_prepare / md_step / md_energy / md_resort).

  * a 4000-particle FP64 run (dt = 0.005, 100 steps, fcc start, T = 1) matches
    the oracle's run: energy log to 1e-10 relative, final positions to 1e-8,
    same number of rebuilds;
  * the list never misses a pair: at every step of a short run the forces on
    the GPU state equal the oracle's forces recomputed from scratch (<= 1e-12);
  * a particle moved from the host by more than half the skin forces a
    rebuild on the next step, and the forces after it miss no pair;
  * mixed precision tracks the FP64 oracle (energy per particle to 1e-5);
  * the paper's benchmark conditions (|v| = 0.9, dt = 0.001) in FP64 and mixed,
    and a never re-sorted run on shuffled labels, match the oracle;
  * runs are bitwise deterministic;
  * the re-sort is an exact permutation;
  * error paths: non-finite force, positions outside the box, list overflow
    with resumption;
  * steps queued in runs with the rebuild decision on the device give bitwise
    the run of one wait per step, and a non-finite force stops a run.
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


def _min_image(d, L):
    return d - L * np.rint(d / L)


@pytest.mark.parametrize("resort_every", [1, 0])
def test_trajectory_fp64_matches_oracle(ref, resort_every):
    q, L = li.fcc_lattice(10)
    v = li.maxwell_boltzmann(q.shape[0], T=1.0, seed=0)
    e = _engine(q, v, L, precision="fp64", resort_every=resort_every)
    log = e.step(100, sample_every=10)
    rq, rv, rlog, rreb = ref.run(q, v, L, 100, dt=0.005, sample_every=10)
    assert log.shape == rlog.shape == (10, 4)
    assert np.abs(log - rlog).max() <= 1e-10 * np.abs(rlog).max()
    assert np.abs(_min_image(e.positions() - rq, L)).max() < 1e-8
    assert np.abs(e.velocities() - rv).max() < 1e-8
    # the GPU counts the initial build as a rebuild
    assert e.rebuilds - 1 == rreb


def test_no_missed_pair_every_step(ref):
    q, L = li.fcc_lattice(10)
    v = li.maxwell_boltzmann(q.shape[0], T=1.0, seed=1)
    e = _engine(q, v, L, precision="fp64", resort_every=1)
    e.prepare()
    idx = np.arange(q.shape[0], dtype=np.int64)
    rebuilds = e.rebuilds
    seen_reuse = 0
    for _ in range(25):
        e.step(1)
        pos = e.positions()
        Fr, S, _, _, _ = ref.forces_sample(pos, L, idx)
        assert G.force_error(e.forces(), Fr, S) <= 1e-12
        seen_reuse += e.rebuilds == rebuilds
        rebuilds = e.rebuilds
    assert seen_reuse >= 10  # most steps reuse the list


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_host_move_beyond_half_skin_rebuilds_next_step(ref, precision):
    # a particle moved from the host by more than half the skin between two
    # calls is caught by the displacement check of the next step: the list is
    # rebuilt before that step's force pass, and no pair is missed
    q, L = li.fcc_lattice(10)
    v = li.maxwell_boltzmann(q.shape[0], T=0.5, seed=8)
    e = _engine(q, v, L, precision=precision, resort_every=1)
    e.prepare()
    e.step(2)
    r0 = e.rebuilds
    e.step(1)
    assert e.rebuilds == r0  # slow start: the list is still valid
    skin = 2.8 - 2.5
    slot = 17
    x = float(e.pos[slot, 0].item()) + 0.7 * skin
    e.pos[slot, 0] = x - L * np.floor(x / L)
    e.step(1)
    assert e.rebuilds == r0 + 1
    idx = np.arange(q.shape[0], dtype=np.int64)
    Fr, S, _, _, _ = ref.forces_sample(e.positions(), L, idx)
    assert G.force_error(e.forces(), Fr, S) <= (1e-12 if precision == "fp64" else 1e-5)


def test_mixed_tracks_fp64(ref):
    q, L = li.fcc_lattice(10)
    v = li.maxwell_boltzmann(q.shape[0], T=1.0, seed=0)
    e = _engine(q, v, L, precision="mixed", resort_every=1)
    log = e.step(100, sample_every=10)
    _, _, rlog, _ = ref.run(q, v, L, 100, dt=0.005, sample_every=10)
    n = q.shape[0]
    assert np.abs(log[:, 3] - rlog[:, 3]).max() / n < 1e-5
    assert np.abs(log[:, 1] - rlog[:, 1]).max() / n < 1e-5


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_paper_conditions_match_oracle(ref, precision):
    # the paper's benchmark conditions (Sec. 4.5) on a 4000-particle cube:
    # |v| = 0.9 in random directions, dt = 0.001, 150 + 100 steps
    cfg = li.PAPER_CONFIGS["paper500k"]
    q, L = li.fcc_lattice(10, cfg["rho"])
    v = li.initial_velocities(cfg, q.shape[0], seed=5)
    rs = cfg["rc"] + cfg["skin"]
    e = _engine(q, v, L, precision=precision, rc=cfg["rc"], rs=rs, dt=cfg["dt"], resort_every=1)
    log = e.step(250, sample_every=25)
    rq, rv, rlog, rreb = ref.run(q, v, L, 250, dt=cfg["dt"], rc=cfg["rc"], rs=rs, sample_every=25)
    n = q.shape[0]
    if precision == "fp64":
        assert np.abs(log - rlog).max() <= 1e-10 * np.abs(rlog).max()
        assert np.abs(_min_image(e.positions() - rq, L)).max() < 1e-8
        assert e.rebuilds - 1 == rreb
    else:
        assert np.abs(log[:, 3] - rlog[:, 3]).max() / n < 1e-5
        assert np.abs(log[:, 1] - rlog[:, 1]).max() / n < 1e-5


def test_no_resort_on_shuffled_labels_matches_oracle(ref):
    # the re-sort ablation's configuration: labels shuffled, never re-sorted
    q, L = li.fcc_lattice(10)
    v = li.maxwell_boltzmann(q.shape[0], T=1.0, seed=6)
    qs, vs, perm = li.shuffle_labels(q, v, seed=7)
    e = _engine(qs, vs, L, precision="fp64", resort_every=0)
    log = e.step(60, sample_every=20)
    rq, rv, rlog, _ = ref.run(qs, vs, L, 60, dt=0.005, sample_every=20)
    assert np.abs(log - rlog).max() <= 1e-10 * np.abs(rlog).max()
    assert np.abs(_min_image(e.positions() - rq, L)).max() < 1e-8
    assert np.array_equal(e.id.cpu().numpy(), np.arange(q.shape[0]))


def test_energy_call_matches_log(ref):
    q, L = li.fcc_lattice(10)
    v = li.maxwell_boltzmann(q.shape[0], seed=4)
    e = _engine(q, v, L)
    log = e.step(20, sample_every=20)
    en = e.energies()
    assert np.allclose(en, log[-1], rtol=1e-13, atol=0)
    F, pe, w = ref.forces(e.positions(), L)
    assert en[1] == pytest.approx(pe, rel=1e-12)
    assert en[2] == pytest.approx(w, rel=1e-12)
    assert en[0] == pytest.approx(0.5 * np.sum(e.velocities() ** 2), rel=1e-12)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_bitwise_deterministic(precision):
    q, L = li.fcc_lattice(12)
    v = li.maxwell_boltzmann(q.shape[0], seed=2)
    a = _engine(q, v, L, precision=precision)
    b = _engine(q, v, L, precision=precision)
    la = a.step(60, sample_every=20)
    lb = b.step(60, sample_every=20)
    assert np.array_equal(la, lb)
    assert np.array_equal(a.positions(), b.positions())
    assert np.array_equal(a.forces(), b.forces())


def test_resort_is_exact_permutation(ref):
    from paper_1012_2677_amd import _abi as A

    q, L = li.jittered_fcc(10, amp=0.2, seed=3)
    q, _, perm = li.shuffle_labels(q, seed=3)
    v = li.maxwell_boltzmann(q.shape[0], seed=3)
    e = _engine(q, v, L, resort_every=1)
    s = e.state
    A.md_bin_cells(e.params, s.pos, s.cells, s.ws, s.ws_bytes, e.stream())
    order = e.grid.order.cpu().numpy()
    A.md_resort(e.params, s, e.stream())
    e._sync_pointers()
    torch.cuda.synchronize()
    pos = e.pos[:, :3].cpu().numpy()
    ids = e.id.cpu().numpy()
    assert np.array_equal(pos, q[order])
    assert np.array_equal(ids, order)
    assert np.array_equal(e.vel.cpu().numpy().T, v[order])
    assert np.array_equal(e.pos_ref.cpu().numpy().T, q[order])
    # slots are now in cell order
    r_cell, _, _, _ = ref.bin_cells(pos, L, e.grid.ncell)
    assert np.all(np.diff(r_cell) >= 0)
    assert np.array_equal(e.grid.cell_of.cpu().numpy(), r_cell)


def test_nonfinite_reported():
    from paper_1012_2677_amd import MdError, _abi as A

    q, L = li.fcc_lattice(6)
    q = q.copy()
    q[1] = q[0]  # two coincident particles
    v = np.zeros_like(q)
    e = _engine(q, v, L)
    with pytest.raises(MdError) as err:
        e.prepare()
    assert err.value.code == A.MD_ERR_NONFINITE


def test_positions_outside_box_rejected():
    from paper_1012_2677_amd import MdError, _abi as A

    q, L = li.fcc_lattice(6)
    q = q.copy()
    q[5, 0] = L + 0.5
    e = _engine(q, np.zeros_like(q), L)
    with pytest.raises(MdError) as err:
        e.prepare()
    assert err.value.code == A.MD_ERR_ARG


def _close_logs(log, rlog, precision, n):
    if precision == "fp64":
        return np.abs(log - rlog).max() <= 1e-10 * np.abs(rlog).max()
    return np.abs(log[:, 1] - rlog[:, 1]).max() / n < 1e-5 and np.abs(log[:, 3] - rlog[:, 3]).max() / n < 1e-5


@pytest.mark.parametrize("waves", ["cell", "tile"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_capacity_overflow_resumes(ref, precision, waves):
    q, L = li.fcc_lattice(10)
    v = li.maxwell_boltzmann(q.shape[0], seed=0)
    e = _engine(q, v, L, cell_stride=64, precision=precision, build_waves=waves)
    log = e.step(30, sample_every=10)
    assert e.plist.cell_stride > 64
    _, _, rlog, _ = ref.run(q, v, L, 30, sample_every=10)
    assert _close_logs(log, rlog, precision, q.shape[0])


@pytest.mark.parametrize("waves", ["cell", "tile"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_overflow_mid_run_resumes(ref, precision, waves):
    q, L = li.fcc_lattice(10)
    v = li.maxwell_boltzmann(q.shape[0], seed=5)
    e = _engine(q, v, L, precision=precision, build_waves=waves)
    e.prepare()
    need = int(e.plist.status[1].item())
    # shrink the list to the lattice's exact need: a later rebuild of the
    # disordered fluid overflows, md_step stops in phase 1 and is resumed
    e.plist.resize(need)
    e.plist.fill(e.state.list)
    e.state.list_valid = 0
    log = e.step(60, sample_every=10)
    assert e.plist.cell_stride > need
    _, _, rlog, _ = ref.run(q, v, L, 60, sample_every=10)
    assert log.shape == rlog.shape
    assert _close_logs(log, rlog, precision, q.shape[0])


@pytest.mark.parametrize("precision,resort_every", [("fp64", 0), ("fp64", 1), ("mixed", 1)])
def test_step_record_matches_single_steps(precision, resort_every):
    # md_step_record's frame k is the positions at which step k evaluated its
    # forces, in the original particle order, and built[k] marks the steps
    # that rebuilt the list; the same run taken one md_step at a time (whose
    # kicks run in separate passes, so roundings may differ in the last bits)
    # gives the same positions and the same rebuilds
    q, L = li.fcc_lattice(10)
    v = li.maxwell_boltzmann(q.shape[0], T=1.0, seed=14)
    a = _engine(q, v, L, precision=precision, resort_every=resort_every)
    b = _engine(q, v, L, precision=precision, resort_every=resort_every)
    a.prepare()
    b.prepare()
    _, frames, built = a.step_record(30)
    assert frames.shape == (30, q.shape[0], 4)
    fr = frames.cpu().numpy()
    assert np.all(fr[:, :, 3] == 0.0)
    for k in range(30):
        r0 = b.rebuilds
        b.step(1)
        assert built[k] == (b.rebuilds > r0), k
        d = fr[k, :, :3] - b.positions()
        assert np.abs(d - L * np.rint(d / L)).max() < 1e-9, k
    assert built.any() and not built.all()


@pytest.mark.parametrize("precision,layout,resort_every", [("fp64", "auto", 1), ("mixed", "auto", 1),
                                                           ("fp64", "slots", 0), ("mixed", "slots", 1)])
def test_queued_runs_equal_a_wait_per_step(precision, layout, resort_every):
    # md_step queues the steps in runs and takes the rebuild decision on the
    # device; runs of one step (a wait after each), of 16 steps (the passes
    # after each stop run gated), and of the automatic length give bitwise the
    # same run: energy log, positions, velocities, forces and rebuild count,
    # and every force pass that ran is timed once
    q, L = li.fcc_lattice(10)
    v = li.maxwell_boltzmann(q.shape[0], T=1.0, seed=21)
    out = {}
    for run in (1, 16, 0):
        e = _engine(q, v, L, precision=precision, list_layout=layout, resort_every=resort_every, step_run=run,
                    timers=True)
        log = e.step(120, sample_every=3)
        e.step(7, sample_every=1)     # a second call resumes the first's state
        out[run] = (log, e.positions(), e.velocities(), e.forces(), e.rebuilds, e.timer_dict())
    ref = out[1]
    assert ref[4] > 10
    for run in (16, 0):
        got = out[run]
        assert np.array_equal(got[0], ref[0]), run
        for k in (1, 2, 3):
            assert np.array_equal(got[k], ref[k]), (run, k)
        assert got[4] == ref[4], run
        for name in ("force", "reduce", "build"):
            assert got[5][name][1] == ref[5][name][1], (run, name)
    assert ref[5]["force"][1] == 127          # one per step (md_prepare is not timed)


def test_queued_runs_stop_on_a_nonfinite_force():
    # a particle placed on top of another, with the same velocity and force,
    # from the host: the next step rebuilds (the move is beyond half the skin), its
    # force is not finite, the run of 16 stops there and its later passes do
    # nothing; the step count says which step it was
    from paper_1012_2677_amd import MdError, _abi as A

    q, L = li.fcc_lattice(8)
    v = li.maxwell_boltzmann(q.shape[0], seed=3)
    e = _engine(q, v, L, step_run=16)
    e.step(5)
    r0 = e.rebuilds
    e.pos[1, :3] = e.pos[0, :3]
    e.vel[:, 1] = e.vel[:, 0]
    e.force[:, 1] = e.force[:, 0]     # so that the first half kick and drift keep them together
    with pytest.raises(MdError) as err:
        e.step(20)
    assert err.value.code == A.MD_ERR_NONFINITE
    assert e.step_count == 6
    assert e.rebuilds == r0 + 1
