"""The streaming probes behind the achievable-bandwidth figure do the work
they are credited with: after a copy b equals a, after a triad c = a + 3 b, on
a size that is not a multiple of the launch grid's slot (ragged tail)."""

import pytest
import torch

pytestmark = pytest.mark.gpu


def test_probe_copy_and_triad_results():
    from paper_1012_2677_amd import _abi as A

    dev = torch.device("cuda", 0)
    n = (1 << 20) + 8 * 37          # doubles; bytes a multiple of 64
    g = torch.Generator(device=dev).manual_seed(0)
    a = torch.randn(n, dtype=torch.float64, device=dev, generator=g)
    b = torch.randn(n, dtype=torch.float64, device=dev, generator=g)
    c = torch.zeros_like(a)
    s = torch.cuda.current_stream(dev).cuda_stream
    for nt in (0, A.MD_PROBE_NT):
        b0 = b.clone()
        ms = A.md_hbm_probe(A.MD_PROBE_TRIAD | nt, a.data_ptr(), b.data_ptr(), c.data_ptr(), 8 * n, 2, s)
        assert ms > 0
        assert torch.allclose(c, a + 3.0 * b0, rtol=1e-15, atol=1e-15)   # one rounding or two
        ms = A.md_hbm_probe(A.MD_PROBE_READ | nt, a.data_ptr(), b.data_ptr(), None, 8 * n, 2, s)
        assert ms > 0 and torch.equal(b, b0)
        ms = A.md_hbm_probe(A.MD_PROBE_COPY | nt, a.data_ptr(), b.data_ptr(), None, 8 * n, 2, s)
        assert torch.equal(b, a)
        b.copy_(b0)
