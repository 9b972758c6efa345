"""GPU tests of degenerate inputs, in every list layout and both precisions.

  * One particle: no pairs; zero force and PE; velocity Verlet with F = 0
    moves it ballistically, q(t) = wrap(q0 + v t), with v and KE unchanged,
    through several rebuilds and re-sorts of a one-particle system.
  * One isolated pair at r = 1.5 across the periodic boundary in x: the
    forces are -g d and +g d with (V, g) from the oracle's pair function,
    PE = V(r) and W = g r^2 (FP64 to 1e-13 relative, mixed to 1e-5); the list
    holds the pair twice in the full layouts and once in the half list (row
    lengths; the tiled list's status total also counts its padding entries).
"""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

LAYOUTS = ["auto", "slots", "half"]


@pytest.fixture(autouse=True, scope="module")
def _cuda():
    assert torch.cuda.is_available()
    import paper_1012_2677_amd  # noqa: F401


def _engine(q, v, L, **kw):
    from paper_1012_2677_amd import Engine

    return Engine(q, v, L, device="cuda:0", **kw)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("layout", LAYOUTS)
def test_single_particle_moves_ballistically(precision, layout):
    L, dt, steps = 10.0, 0.005, 60
    q = np.array([[9.9, 0.05, 5.0]])
    v = np.array([[1.0, -2.0, 0.5]])
    e = _engine(q, v, L, precision=precision, list_layout=layout, dt=dt)
    log = e.step(steps, sample_every=10)
    assert int(e.plist.status[0].item()) == 0
    assert e.rebuilds > 2            # it crossed half the skin several times
    assert np.all(e.forces() == 0.0)
    assert np.all(log[:, 1] == 0.0) and np.all(log[:, 2] == 0.0)
    assert np.allclose(log[:, 0], 0.5 * np.sum(v * v), rtol=0, atol=1e-15)
    assert np.array_equal(e.velocities(), v)
    want = np.mod(q + steps * dt * v, L)
    d = e.positions() - want
    assert np.abs(d - L * np.rint(d / L)).max() < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("layout", LAYOUTS)
def test_isolated_pair_across_the_boundary(ref, precision, layout):
    L = 10.0
    q = np.array([[0.2, 5.0, 5.0], [8.7, 5.0, 5.0]])   # minimum-image distance 1.5 along x
    v = np.zeros_like(q)
    e = _engine(q, v, L, precision=precision, list_layout=layout)
    e.prepare()
    # row lengths count the pairs; the tiled list also pads each row of odd
    # length with the tile's stand-in entry, which its status total includes
    assert int(e.plist.counts.sum().item()) == (1 if layout == "half" else 2)
    assert int(e.plist.status[0].item()) == {"auto": 4, "slots": 2, "half": 1}[layout]
    assert int(e.state.list_tiled) == (1 if layout == "auto" else 0)
    V, g = ref.pair(1.5 * 1.5)
    d = np.array([-1.5, 0.0, 0.0])                       # q_1 - q_0, minimum image
    want = np.stack([-g * d, g * d])
    F = e.forces()
    en = e.energies()
    tol = 1e-13 if precision == "fp64" else 1e-5
    scale = abs(g) * 1.5
    assert np.abs(F - want).max() <= tol * scale
    assert abs(en[1] - V) <= tol * abs(V)
    assert abs(en[2] - g * 2.25) <= tol * abs(g * 2.25)
