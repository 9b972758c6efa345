"""GPU tests of the half list: each pair once (Sec. 2.4, the key/partner list
with Newton's third law), the partner's share of the force added by atomics.

  * index work, bit-exact: every half row equals the full row of the same key
    with the partners of stencil codes 0 .. 12, and the own cell's partners
    of smaller slot, removed (same entries in the same order); the unordered
    pairs of the half list are the oracle's pair set, each exactly once; rows
    keep the (code, slot) order and each code names the partner's cell;
  * forces from md_forces on a half list against the FP64 oracle (1e-12 in
    FP64, 1e-5 in mixed, of the pair-force scale), PE and W as for full
    lists (1e-12 / 1e-6 of the sum of magnitudes);
  * runs of the simulation state with the half list against the oracle's run
    (FP64: energy log to 1e-10 relative, same rebuilds; mixed: energy per
    particle to 1e-5), with the half-skin and the DUTC + LDC rules;
  * the Hessian and adjoint passes refuse a half list.
The atomics make the rounding of each force sum depend on their order, so
nothing here compares two runs bit for bit.
"""

import numpy as np
import pytest
import torch

import lj_inputs as li
from tests import gpu_util as G
from tests.test_gpu_parity import CASES, FP64_TOL, MIXED_TOL, _case, _check_rows_structure
from tests.test_oracle_cells import ADV_L, adversarial_pairs

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True, scope="module")
def _cuda():
    assert torch.cuda.is_available()
    import paper_1012_2677_amd  # noqa: F401


def _half_of_full(keys, partners, codes):
    return (codes > 13) | ((codes == 13) & (partners > keys))


@pytest.mark.parametrize("name", CASES)
def test_half_rows_are_full_rows_filtered(ref, name):
    q, L = _case(name)
    full = G.Standalone(q, L)
    half = G.Standalone(q, L, list_layout="half")
    cell_of = full.bin()[0]
    half.bin()
    assert full.build()[2] == 0
    st = half.build()
    assert st[2] == 0
    assert int(half.plist.l.half) == 1 and int(full.plist.l.half) == 0
    kf, pf, cf = G.decode_rows(*full.plist.rows())
    kh, ph, ch = G.decode_rows(*half.plist.rows())
    keep = _half_of_full(kf, pf, cf)
    assert np.array_equal(kh, kf[keep])
    assert np.array_equal(ph, pf[keep])
    assert np.array_equal(ch, cf[keep])
    assert st[0] == kh.shape[0]
    uniq, mult = G.pair_set_from_rows(kh, ph)
    assert np.all(mult == 1)
    assert np.array_equal(uniq, G.pair_codes(ref.pairs_cells(q, L, 2.8)))
    _check_rows_structure(half, kh, ph, ch, cell_of)


def test_half_list_adversarial_ulp(ref):
    q, expect = adversarial_pairs()
    s = G.Standalone(q, [ADV_L] * 3, list_layout="half")
    s.bin()
    s.build()
    keys, partners, _ = G.decode_rows(*s.plist.rows())
    uniq, mult = G.pair_set_from_rows(keys, partners)
    assert np.all(mult == 1)
    assert np.array_equal(uniq, G.pair_codes(sorted(expect)))


@pytest.mark.parametrize("precision,name", [("fp64", n) for n in ("fcc10", "jitter12", "ragged_jitter", "aniso",
                                                                  "aniso_jitter", "small_box", "clump", "dense",
                                                                  "slab")]
                         + [("mixed", n) for n in ("jitter12", "ragged_jitter", "aniso_jitter", "small_box")])
def test_half_forces_match_oracle(ref, precision, name):
    q, L = _case(name)
    s = G.Standalone(q, L, precision=precision, list_layout="half")
    s.bin()
    s.build()
    F, pw = s.forces()
    F2, _ = s.forces(energy=False)
    idx = np.arange(q.shape[0], dtype=np.int64)
    Fr, S, pe_i, w_i, _ = ref.forces_sample(q, L, idx)
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    assert G.force_error(F, Fr, S) <= tol
    assert G.force_error(F2, Fr, S) <= tol
    _, pe, w = ref.forces(q, L)
    etol = FP64_TOL if precision == "fp64" else 1e-6
    assert abs(pw[0] - pe) <= etol * np.abs(pe_i).sum()
    assert abs(pw[1] - w) <= etol * np.abs(w_i).sum()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("rule", ["half_skin", "dutc_ldc"])
def test_half_run_tracks_oracle(ref, precision, rule):
    from paper_1012_2677_amd import Engine

    q, L = li.fcc_lattice(10)
    v = li.maxwell_boltzmann(q.shape[0], T=1.0, seed=0)
    e = Engine(q, v, L, precision=precision, list_layout="half", rebuild_rule=rule, device="cuda:0")
    log = e.step(100, sample_every=10)
    assert int(e.state.list.half) == 1 and int(e.state.list_tiled) == 0
    rq, _, rlog, rreb = ref.run(q, v, L, 100, dt=0.005, sample_every=10, rule=rule)
    n = q.shape[0]
    if precision == "fp64":
        assert np.abs(log - rlog).max() <= 1e-10 * np.abs(rlog).max()
        d = e.positions() - rq
        assert np.abs(d - L * np.rint(d / L)).max() < 1e-8
        assert e.rebuilds - 1 == rreb
    else:
        assert np.abs(log[:, 3] - rlog[:, 3]).max() / n < 1e-5
        assert np.abs(log[:, 1] - rlog[:, 1]).max() / n < 1e-5
    # the state's forces after the run are those of its positions, on the
    # per-particle metric |dF_i| / S_i of every other force check
    pos = e.positions()
    Fr, S, _, _, _ = ref.forces_sample(pos, L, np.arange(n, dtype=np.int64))
    assert G.force_error(e.forces(), Fr, S) <= (FP64_TOL if precision == "fp64" else MIXED_TOL)


def test_adjoint_passes_refuse_a_half_list():
    from paper_1012_2677_amd import _abi as A

    q, L = _case("jitter12")
    s = G.Standalone(q, L, list_layout="half")
    s.bin()
    s.build()
    u = np.random.default_rng(0).standard_normal(q.shape)
    for call in (lambda: s.hvp(u), lambda: s.param_grad()):
        with pytest.raises(A.MdError) as err:
            call()
        assert err.value.code == A.MD_ERR_ARG
