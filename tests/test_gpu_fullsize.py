"""Parity at full workload sizes, in the launch configuration the benchmark
times (re-sort at every rebuild; mixed precision at 32M and 131M, FP64 at 4M),
on sampled particles the oracle can check one by one:

  * the pair-list rows of the sampled particles equal the oracle's neighbour
    sets within rs (exact set equality, ids; the tiled list, decoded on the
    host);
  * the forces on the sampled particles equal the oracle's to the precision
    bar (1e-5 mixed, 1e-12 FP64, relative to the pair-force scale S_i);
  * the list's total entry count equals twice the number of pairs implied by
    the per-particle neighbour counts of the sample (statistical check only).

The state is first advanced some steps (a disordered fluid with several
rebuilds and re-sorts behind it), then md_prepare rebuilds the list at the
current positions.  The half list (each pair once) gets the same row and
force checks at 32M, its rows cut from the oracle's sets by the half rule.

The adjoint passes (md_hvp, md_param_grad, md_adjoint_kick) are compared with
the oracle element by element at the gradient workload's full size (256,000
particles of an equilibrating fluid), one oracle pass each.
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


def _sample_ids(n, k, seed):
    rng = np.random.default_rng(seed)
    ids = rng.choice(n, size=k, replace=False)
    return np.unique(np.concatenate([ids, [0, 1, n - 2, n - 1]])).astype(np.int64)


def _check_state(ref, e, L, ids, tol):
    q = e.positions()
    nc, _ = ref.cell_dims(L, e.params.rs)
    _, count, start, order = ref.bin_cells(q, L, nc)
    grid = (nc, count, start, order)
    # rows
    ids_dev = e.id.long()
    slot_of_id = torch.empty_like(ids_dev)
    slot_of_id[ids_dev] = torch.arange(e.n, device=ids_dev.device)
    slots = slot_of_id[torch.as_tensor(ids, device=ids_dev.device)]
    kidx, pslot = G.rows_for_slots_state(e, slots.cpu().numpy())
    pid = e.id.cpu().numpy()[pslot]
    ref_rows = ref.neighbors_sample(q, L, ids, rs=e.params.rs, grid=grid)
    for k in range(len(ids)):
        got = np.sort(pid[kidx == k])
        assert np.array_equal(got, ref_rows[k]), (ids[k], len(got), len(ref_rows[k]))
    # forces
    F = e.forces()[ids]
    Fr, S, _, _, nb = ref.forces_sample(q, L, ids, rc=e.params.rc, rs=e.params.rs, grid=grid)
    err = G.force_error(F, Fr, S)
    assert err <= tol, err
    mean_nb = nb.mean()
    total = int(e.plist.status[0].item())
    assert abs(total / e.n - mean_nb) < 0.05 * mean_nb
    return err


@pytest.mark.parametrize("config,precision,tol,steps", [
    ("lj32m", "mixed", 1e-5, 40),
    ("lj32m", "fp64", 1e-12, 40),
    ("lj4m", "fp64", 1e-12, 40),
])
def test_full_size_sampled_parity(ref, config, precision, tol, steps):
    from paper_1012_2677_amd import Engine

    cfg = li.CONFIGS[config]
    q, L = li.fcc_lattice(cfg["n_fcc"])
    v = li.maxwell_boltzmann(q.shape[0], cfg["T"], seed=0)
    n = q.shape[0]
    e = Engine(q, v, L, rc=cfg["rc"], rs=cfg["rc"] + cfg["skin"], dt=cfg["dt"], precision=precision,
               resort_every=1, device="cuda:0")
    del q, v
    e.step(steps)
    assert e.rebuilds > 3
    e.prepare()
    # the tiled list (the benchmark's configuration)
    assert int(e.state.list_tiled) == 1
    _check_state(ref, e, L, _sample_ids(n, 2048, 1), tol)


def test_largest_workload_sampled_parity(ref):
    """131,072,000 particles (the largest single-GPU workload), mixed."""
    from paper_1012_2677_amd import Engine

    cfg = li.CONFIGS["lj131m"]
    q, L = li.fcc_lattice(cfg["n_fcc"])
    v = li.maxwell_boltzmann(q.shape[0], cfg["T"], seed=0)
    n = q.shape[0]
    e = Engine(q, v, L, rc=cfg["rc"], rs=cfg["rc"] + cfg["skin"], dt=cfg["dt"], precision="mixed",
               resort_every=1, device="cuda:0")
    del q, v
    e.step(12)
    e.prepare()
    assert int(e.state.list_tiled) == 1
    _check_state(ref, e, L, _sample_ids(n, 1024, 2), 1e-5)


def _cell_offset(a, b, n):
    d = (b - a) % n
    return np.where(d == n - 1, -1, d)


def test_half_list_full_size_sampled_parity(ref):
    """32,000,000 particles, mixed, half list (each pair once): the rows of
    sampled keys equal the oracle's neighbour sets cut by the half rule
    (partners in cells of stencil code above 13, or in the key's cell with a
    larger slot), in (code, slot) order; the forces on the sampled particles,
    which collect the atomics of every key, equal the oracle's (1e-5)."""
    from paper_1012_2677_amd import Engine

    cfg = li.CONFIGS["lj32m"]
    q, L = li.fcc_lattice(cfg["n_fcc"])
    v = li.maxwell_boltzmann(q.shape[0], cfg["T"], seed=0)
    n = q.shape[0]
    e = Engine(q, v, L, rc=cfg["rc"], rs=cfg["rc"] + cfg["skin"], dt=cfg["dt"], precision="mixed",
               resort_every=1, list_layout="half", device="cuda:0")
    del q, v
    e.step(20)
    e.prepare()
    assert int(e.state.list.half) == 1 and int(e.state.list_tiled) == 0
    ids = _sample_ids(n, 2048, 3)
    q = e.positions()
    nc, _ = ref.cell_dims(L, e.params.rs)
    _, count, start, order = ref.bin_cells(q, L, nc)
    grid = (nc, count, start, order)
    id_of_slot = e.id.cpu().numpy()
    slot_of_id = np.empty(n, np.int64)
    slot_of_id[id_of_slot] = np.arange(n)
    cxyz = e.grid.cell_xyz.cpu().numpy()
    slots = slot_of_id[ids]
    kidx, pslot, codes = G.rows_for_slots(e.plist, slots)
    ref_rows = ref.neighbors_sample(q, L, ids, rs=e.params.rs, grid=grid)
    for k in range(len(ids)):
        sk = slots[k]
        sj = slot_of_id[ref_rows[k]]
        a, b = cxyz[sk], cxyz[sj]
        sx = _cell_offset(a & 1023, b & 1023, nc[0])
        sy = _cell_offset((a >> 10) & 1023, (b >> 10) & 1023, nc[1])
        sz = _cell_offset((a >> 20) & 1023, (b >> 20) & 1023, nc[2])
        code = (sx + 1) * 9 + (sy + 1) * 3 + (sz + 1)
        keep = (code > 13) | ((code == 13) & (sj > sk))
        want = np.lexsort((sj[keep], code[keep]))
        row = kidx == k
        assert np.array_equal(pslot[row], sj[keep][want]), ids[k]
        assert np.array_equal(codes[row], code[keep][want]), ids[k]
    F = e.forces()[ids]
    Fr, S, _, _, _ = ref.forces_sample(q, L, ids, rc=e.params.rc, rs=e.params.rs, grid=grid)
    assert G.force_error(F, Fr, S) <= 1e-5


def test_adjoint_full_size_elementwise(ref):
    """256,000 particles (the gradient workload), FP64: md_hvp, md_param_grad
    and md_adjoint_kick against oracle.hvp / oracle.param_grad / oracle.forces
    on every particle, with the per-particle scales of the pair terms
    (gradients of one configuration: 1e-10)."""
    from paper_1012_2677_amd import Engine

    cfg = li.CONFIGS["lj256k"]
    q, L = li.fcc_lattice(cfg["n_fcc"])
    v = li.maxwell_boltzmann(q.shape[0], cfg["T"], seed=4)
    n = q.shape[0]
    e = Engine(q, v, L, rc=cfg["rc"], rs=cfg["rc"] + cfg["skin"], dt=cfg["dt"], precision="fp64",
               resort_every=1, device="cuda:0")
    e.step(40)
    assert e.rebuilds > 3
    q = e.positions()
    del e
    eps, sig = 1.05, 0.98
    s = G.Standalone(q, L, eps=eps, sigma=sig)
    s.params.dt = cfg["dt"]
    s.bin()
    assert s.build()[2] == 0
    rng = np.random.default_rng(5)
    u = rng.standard_normal(q.shape)
    out0 = rng.standard_normal(q.shape)
    pairs = ref.pairs_cells(q, L, cfg["rc"])
    hs = G.hvp_scale(q, L, u, pairs, eps=eps, sigma=sig)
    Hr, dpr = ref.hvp(q, L, u, eps=eps, sigma=sig)
    Hu, dp = s.hvp(u)
    assert G.elementwise_error(Hu, Hr, hs) <= 1e-10
    assert dp == pytest.approx(dpr, rel=1e-10)
    dUr = ref.param_grad(q, L, eps=eps, sigma=sig)
    assert s.param_grad() == pytest.approx(dUr, rel=1e-10)
    # the fused kick of the reverse sweep: out = out0 - h H u - w F,
    # u_out = u + dt out, acc = h u . dF/dtheta + w dU/dtheta
    h, w = 0.5 * cfg["dt"], 1.0 / 200
    out, u_out, acc = s.adjoint_kick(u, out0, (1.0, -h, -w, h, w))
    Fr, S, _, _, _ = ref.forces_sample(q, L, np.arange(n, dtype=np.int64), eps=eps, sigma=sig)
    want = out0 - h * Hr - w * Fr
    scale = np.linalg.norm(out0, axis=1) + h * hs + w * S
    assert G.elementwise_error(out, want, scale) <= 1e-10
    assert G.elementwise_error(u_out, u + cfg["dt"] * want, np.linalg.norm(u, axis=1) + cfg["dt"] * scale) <= 1e-10
    assert acc == pytest.approx(h * dpr + w * dUr, rel=1e-10)
