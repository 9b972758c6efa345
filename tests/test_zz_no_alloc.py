"""md_forces_noalloc, the variant of md_forces that allocates nothing (its
scratch is a fixed array inside the library), gives md_forces' results bit
for bit: two calls in a row on one device, the second on a smaller input, in
FP64 and mixed precision, with and without energies; and the oracle's forces
to each precision's bar.  Above its particle limit it refuses before any
launch."""

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


def _noalloc(s, energy):
    A = s.A
    dt = torch.float32 if s.params.precision == A.MD_MIXED else torch.float64
    F = torch.zeros((3, s.n), dtype=dt, device=G.device())
    pw = torch.zeros(2, dtype=torch.float64, device=G.device())
    A.md_forces_noalloc(s.params, s.pos.data_ptr(), s.grid.c, s.plist.l, F.data_ptr(),
                        pw.data_ptr() if energy else None, s.stream)
    torch.cuda.synchronize()
    return F.double().cpu().numpy().T.copy(), pw.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_forces_equal_md_forces_on_two_calls(ref, precision):
    tol = 1e-12 if precision == "fp64" else 1e-5
    # the second call takes a smaller input than the first
    for n_fcc, seed in ((12, 31), (8, 32)):
        q, L = li.jittered_fcc(n_fcc, amp=0.2, seed=seed)
        s = G.Standalone(q, [L] * 3, precision=precision)
        s.bin()
        assert s.build()[2] == 0
        for energy in (True, False):
            F_ref, pw_ref = s.forces(energy=energy)
            F, pw = _noalloc(s, energy)
            assert np.array_equal(F, F_ref), (n_fcc, energy)
            if energy:
                assert np.array_equal(pw, pw_ref), (n_fcc, pw, pw_ref)
        Fr, S, _, _, _ = ref.forces_sample(q, [L] * 3, np.arange(q.shape[0], dtype=np.int64))
        assert G.force_error(F, Fr, S) <= tol


def test_noalloc_refuses_more_particles_than_its_scratch_holds():
    from paper_1012_2677_amd import _abi as A
    from paper_1012_2677_amd.engine import make_params

    n = A.MD_NOALLOC_MAX_N + 1
    p = make_params(n, 200.0)
    fake = 1 << 20   # never dereferenced: the size check fails first
    cells = A.MdCells()
    cells.cell_of = cells.cell_xyz = cells.count = cells.start = cells.order = fake
    plist = A.MdPairlist()
    with pytest.raises(A.MdError) as e:
        A.md_forces_noalloc(p, fake, cells, plist, fake, None, None)
    assert e.value.code == A.MD_ERR_ARG and "at most" in str(e.value)
