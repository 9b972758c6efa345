"""GPU tests of the differentiable layer (LJEnergy, TrajectoryMeanPE).

  * LJEnergy: U, F and the gradients of L = a U + gF . F with respect to q,
    eps and sigma equal the CPU oracle's (H u from the oracle's Hessian-vector
    product, parameter terms from its derivative routines) to 1e-10;
  * LJEnergy: central finite differences (h = 1e-6) of U along a random
    direction and in eps, sigma;
  * TrajectoryMeanPE: O and its gradients equal the oracle's checkpointed
    reverse sweep on a 500-particle system (1e-8 relative), also when the
    sweep's list overflows and a segment is swept again;
  * TrajectoryMeanPE at the full differentiable workload (N = 256,000, 200
    steps, checkpoints every 20, dt = 0.005): central finite differences with
    h = 1e-6 along a random direction in q0 and in eps, sigma.
"""

import numpy as np
import pytest
import torch

import lj_inputs as li

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True, scope="module")
def _cuda():
    assert torch.cuda.is_available()
    import paper_1012_2677_amd  # noqa: F401


DEV = "cuda:0"


def _t(x, grad=False):
    return torch.tensor(x, dtype=torch.float64, device=DEV, requires_grad=grad)


def test_ljenergy_matches_oracle(ref):
    from paper_1012_2677_amd import LJEnergy

    q, L = li.jittered_fcc(8, amp=0.15, seed=41)
    eps0, sig0 = 1.1, 0.97
    qt, eps, sig = _t(q, True), _t(eps0, True), _t(sig0, True)
    U, F = LJEnergy.apply(qt, eps, sig, L)
    Fr, pe, _ = ref.forces(q, L, eps=eps0, sigma=sig0)
    assert U.item() == pytest.approx(pe, rel=1e-12)
    assert np.abs(F.detach().cpu().numpy() - Fr).max() <= 1e-12 * np.abs(Fr).max()
    rng = np.random.default_rng(5)
    gF = rng.standard_normal(q.shape)
    a = 0.7
    loss = a * U + (F * _t(gF)).sum()
    loss.backward()
    Hu, dp = ref.hvp(q, L, gF, eps=eps0, sigma=sig0)
    dU = ref.param_grad(q, L, eps=eps0, sigma=sig0)
    gq_ref = -a * Fr - Hu
    assert np.abs(qt.grad.cpu().numpy() - gq_ref).max() <= 1e-10 * np.abs(gq_ref).max()
    assert eps.grad.item() == pytest.approx(a * dU[0] + dp[0], rel=1e-10)
    assert sig.grad.item() == pytest.approx(a * dU[1] + dp[1], rel=1e-10)


def test_ljenergy_finite_differences():
    from paper_1012_2677_amd import LJEnergy

    q, L = li.jittered_fcc(10, amp=0.15, seed=42)
    qt, eps, sig = _t(q, True), _t(1.0, True), _t(1.0, True)
    U, _ = LJEnergy.apply(qt, eps, sig, L)
    U.backward()
    rng = np.random.default_rng(6)
    u = rng.standard_normal(q.shape)
    h = 1e-6

    def energy(qq, e=1.0, s=1.0):
        with torch.no_grad():
            return LJEnergy.apply(_t(qq), _t(e), _t(s), L)[0].item()

    fd = (energy(q + h * u) - energy(q - h * u)) / (2 * h)
    assert np.sum(qt.grad.cpu().numpy() * u) == pytest.approx(fd, rel=1e-6)
    fde = (energy(q, 1.0 + h) - energy(q, 1.0 - h)) / (2 * h)
    fds = (energy(q, 1.0, 1.0 + h) - energy(q, 1.0, 1.0 - h)) / (2 * h)
    assert eps.grad.item() == pytest.approx(fde, rel=1e-7)
    assert sig.grad.item() == pytest.approx(fds, rel=1e-7)


def test_trajectory_gradient_matches_oracle(ref):
    from paper_1012_2677_amd import TrajectoryMeanPE

    q, L = li.fcc_lattice(5)
    v = li.maxwell_boltzmann(q.shape[0], seed=43)
    K, ck = 40, 10
    qt, eps, sig = _t(q, True), _t(1.0, True), _t(1.0, True)
    O = TrajectoryMeanPE.apply(qt, _t(v), eps, sig, L, K, ck)
    O.backward()
    Or, gqr, gpr = ref.traj_mean_pe_grad(q, v, L, K, ckpt=ck)
    assert O.item() == pytest.approx(Or, rel=1e-12)
    gq = qt.grad.cpu().numpy()
    assert np.abs(gq - gqr).max() <= 1e-8 * np.abs(gqr).max()
    assert eps.grad.item() == pytest.approx(gpr[0], rel=1e-8)
    assert sig.grad.item() == pytest.approx(gpr[1], rel=1e-8)


def test_trajectory_gradient_redoes_a_segment_whose_list_overflowed(ref, monkeypatch):
    # the reverse sweep reads its lists' overflow flags once per segment; a
    # field list made too small from the start overflows, the segment is swept
    # again from its saved adjoints with a grown list, and the gradients are
    # those of the oracle
    from paper_1012_2677_amd import TrajectoryMeanPE, autograd

    made = []

    class TinyList(autograd.PairList):
        def __init__(self, params, ncell, device, cell_stride=None, entry_bits=32):
            super().__init__(params, ncell, device, 8, entry_bits)
            made.append(self)

    monkeypatch.setattr(autograd, "PairList", TinyList)
    q, L = li.fcc_lattice(5)
    v = li.maxwell_boltzmann(q.shape[0], seed=44)
    K, ck = 30, 10
    qt, eps, sig = _t(q, True), _t(1.0, True), _t(1.0, True)
    O = TrajectoryMeanPE.apply(qt, _t(v), eps, sig, L, K, ck)
    O.backward()
    assert made and made[0].cell_stride > 8      # the field's list grew
    Or, gqr, gpr = ref.traj_mean_pe_grad(q, v, L, K, ckpt=ck)
    gq = qt.grad.cpu().numpy()
    assert np.abs(gq - gqr).max() <= 1e-8 * np.abs(gqr).max()
    assert eps.grad.item() == pytest.approx(gpr[0], rel=1e-8)
    assert sig.grad.item() == pytest.approx(gpr[1], rel=1e-8)


def test_trajectory_gradient_full_size_finite_differences():
    from paper_1012_2677_amd import TrajectoryMeanPE

    cfg = li.CONFIGS["lj256k"]
    q, L = li.fcc_lattice(cfg["n_fcc"])
    v = li.maxwell_boltzmann(q.shape[0], cfg["T"], seed=0)
    K, ck, dt = cfg["steps"], 20, cfg["dt"]
    qt, eps, sig = _t(q, True), _t(1.0, True), _t(1.0, True)
    vt = _t(v)
    O = TrajectoryMeanPE.apply(qt, vt, eps, sig, L, K, ck, dt)
    O.backward()
    h = 1e-6
    rng = np.random.default_rng(7)
    u = rng.standard_normal(q.shape)

    def obs(qq, e=1.0, s=1.0):
        with torch.no_grad():
            return TrajectoryMeanPE.apply(_t(qq), vt, _t(e), _t(s), L, K, ck, dt).item()

    gq = qt.grad.cpu().numpy()
    # the lattice start is in [0, L); the perturbed copies are folded back in
    fd = (obs(li.wrap_into_box(q + h * u, L)) - obs(li.wrap_into_box(q - h * u, L))) / (2 * h)
    assert np.sum(gq * u) == pytest.approx(fd, rel=1e-5)
    fde = (obs(q, 1.0 + h) - obs(q, 1.0 - h)) / (2 * h)
    fds = (obs(q, 1.0, 1.0 + h) - obs(q, 1.0, 1.0 - h)) / (2 * h)
    assert eps.grad.item() == pytest.approx(fde, rel=1e-6)
    assert sig.grad.item() == pytest.approx(fds, rel=1e-6)
