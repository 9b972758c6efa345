"""Pins of the oracle's adjoint routines.

  * H u equals central differences of the force field, -(F(q+hu) - F(q-hu))/2h;
  * H u equals torch's float64 CPU autograd Hessian-vector product of a
    brute-force energy (a library routine differentiating an independent
    torch expression of the potential);
  * dU/d(eps, sigma) and u . dF/d(eps, sigma) equal central differences;
  * the checkpointed trajectory gradient equals central finite differences of
    the observable along random directions and in eps, sigma, and equals torch
    autograd through an unrolled velocity-Verlet run on a tiny system;
  * checkpoint spacing does not change the result.
"""

import numpy as np
import pytest
import torch

import lj_inputs as li


def torch_energy(q, L, eps, sigma, rc=2.5):
    """Brute-force truncated LJ energy in torch (float64), minimum image."""
    n = q.shape[0]
    i, j = torch.triu_indices(n, n, 1)
    d = q[j] - q[i]
    d = d - L * torch.round(d / L)
    r2 = (d * d).sum(-1)
    x = sigma / rc
    c2 = 6 * x ** 14 - 3 * x ** 8
    c0 = -7 * x ** 12 + 4 * x ** 6
    s6 = (sigma * sigma / r2) ** 3
    V = 4 * eps * (s6 * s6 - s6 + c2 * r2 / (sigma * sigma) + c0)
    return torch.where(r2 < rc * rc, V, torch.zeros_like(V)).sum()


@pytest.fixture(scope="module")
def small():
    q, L = li.jittered_fcc(3, amp=0.15, seed=21)  # N = 108, L = 6
    return q, L


def test_hvp_finite_differences(ref, small):
    q, L = small
    rng = np.random.default_rng(1)
    u = rng.standard_normal(q.shape)
    Hu, _ = ref.hvp(q, L, u)
    h = 1e-6
    Fp, _, _ = ref.forces(q + h * u, L)
    Fm, _, _ = ref.forces(q - h * u, L)
    fd = -(Fp - Fm) / (2 * h)
    assert np.abs(Hu - fd).max() < 1e-5 * np.abs(Hu).max()


def test_hvp_torch_autograd(ref, small):
    q, L = small
    rng = np.random.default_rng(2)
    u = rng.standard_normal(q.shape)
    Hu, _ = ref.hvp(q, L, u)
    qt = torch.tensor(q, dtype=torch.float64)
    ut = torch.tensor(u, dtype=torch.float64)
    _, hv = torch.autograd.functional.hvp(lambda x: torch_energy(x, L, 1.0, 1.0), qt, ut)
    assert np.abs(Hu - hv.numpy()).max() < 1e-10 * np.abs(Hu).max()
    # the gradient agrees as well (dU/dq = -F)
    qg = qt.clone().requires_grad_(True)
    torch_energy(qg, L, 1.0, 1.0).backward()
    F, _, _ = ref.forces(q, L)
    assert np.abs(qg.grad.numpy() + F).max() < 1e-11 * np.abs(F).max()


def test_param_grad_finite_differences(ref, small):
    q, L = small
    dU = ref.param_grad(q, L, eps=1.1, sigma=0.95)
    h = 1e-6
    _, ep, _ = ref.forces(q, L, eps=1.1 + h, sigma=0.95)
    _, em, _ = ref.forces(q, L, eps=1.1 - h, sigma=0.95)
    assert dU[0] == pytest.approx((ep - em) / (2 * h), rel=1e-7)
    _, sp, _ = ref.forces(q, L, eps=1.1, sigma=0.95 + h)
    _, sm, _ = ref.forces(q, L, eps=1.1, sigma=0.95 - h)
    assert dU[1] == pytest.approx((sp - sm) / (2 * h), rel=1e-6)


def test_force_parameter_vjp(ref, small):
    q, L = small
    rng = np.random.default_rng(3)
    u = rng.standard_normal(q.shape)
    _, dp = ref.hvp(q, L, u, eps=1.2, sigma=1.05)
    h = 1e-6
    for k, (de, ds) in enumerate([(h, 0.0), (0.0, h)]):
        Fp, _, _ = ref.forces(q, L, eps=1.2 + de, sigma=1.05 + ds)
        Fm, _, _ = ref.forces(q, L, eps=1.2 - de, sigma=1.05 - ds)
        fd = np.sum(u * (Fp - Fm)) / (2 * h)
        assert dp[k] == pytest.approx(fd, rel=1e-6)


def _observable(ref, q0, v0, L, K, eps, sigma, dt):
    O, _, _ = ref.traj_mean_pe_grad(q0, v0, L, K, ckpt=K, dt=dt, eps=eps, sigma=sigma)
    return O


def test_trajectory_gradient_finite_differences(ref):
    q0, L = li.jittered_fcc(3, amp=0.1, seed=31)
    v0 = li.maxwell_boltzmann(q0.shape[0], seed=31)
    K, dt = 30, 0.005
    O, gq, gp = ref.traj_mean_pe_grad(q0, v0, L, K, ckpt=7, dt=dt, eps=1.0, sigma=1.0)
    h = 1e-6
    rng = np.random.default_rng(4)
    for _ in range(3):
        u = rng.standard_normal(q0.shape)
        u /= np.linalg.norm(u)
        fd = (_observable(ref, q0 + h * u, v0, L, K, 1.0, 1.0, dt)
              - _observable(ref, q0 - h * u, v0, L, K, 1.0, 1.0, dt)) / (2 * h)
        assert np.sum(gq * u) == pytest.approx(fd, rel=1e-5, abs=1e-7)
    fde = (_observable(ref, q0, v0, L, K, 1.0 + h, 1.0, dt)
           - _observable(ref, q0, v0, L, K, 1.0 - h, 1.0, dt)) / (2 * h)
    fds = (_observable(ref, q0, v0, L, K, 1.0, 1.0 + h, dt)
           - _observable(ref, q0, v0, L, K, 1.0, 1.0 - h, dt)) / (2 * h)
    assert gp[0] == pytest.approx(fde, rel=1e-5)
    assert gp[1] == pytest.approx(fds, rel=1e-5)


def test_trajectory_gradient_torch_unrolled(ref):
    q0, L = li.jittered_fcc(3, amp=0.1, seed=32)
    v0 = li.maxwell_boltzmann(q0.shape[0], seed=32)
    K, dt = 12, 0.005
    O, gq, gp = ref.traj_mean_pe_grad(q0, v0, L, K, ckpt=5, dt=dt)
    q = torch.tensor(q0, requires_grad=True)
    eps = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    sig = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    v = torch.tensor(v0)

    def force(x):
        with torch.enable_grad():
            e = torch_energy(x, L, eps, sig)
            (g,) = torch.autograd.grad(e, x, create_graph=True)
        return -g

    x = q
    F = force(x)
    tot = 0.0
    for _ in range(K):
        v = v + 0.5 * dt * F
        x = x + dt * v
        F = force(x)
        v = v + 0.5 * dt * F
        tot = tot + torch_energy(x, L, eps, sig)
    Ot = tot / K
    Ot.backward()
    assert O == pytest.approx(Ot.item(), rel=1e-12)
    assert np.abs(gq - q.grad.numpy()).max() < 1e-9 * np.abs(gq).max()
    assert gp[0] == pytest.approx(eps.grad.item(), rel=1e-9)
    assert gp[1] == pytest.approx(sig.grad.item(), rel=1e-9)


def test_checkpoint_spacing_invariant(ref):
    q0, L = li.jittered_fcc(3, amp=0.1, seed=33)
    v0 = li.maxwell_boltzmann(q0.shape[0], seed=33)
    a = ref.traj_mean_pe_grad(q0, v0, L, 20, ckpt=20)
    b = ref.traj_mean_pe_grad(q0, v0, L, 20, ckpt=3)
    assert a[0] == b[0]
    assert np.array_equal(a[1], b[1])
    assert np.array_equal(a[2], b[2])
