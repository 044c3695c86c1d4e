"""The allocation-free KI2 entry point (gsyeig_symv_noalloc) against the
context-based gsyeig_symv, through the C ABI: the same kernels in the same
order, so the results must agree bit for bit -- on two calls in a row, the
second with a smaller (ragged) input, and with a padded leading dimension.
Sizes beyond the fixed scratch are rejected without touching the GPU."""
import sys

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def test_symv_noalloc_equals_symv():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1111_6374_amd as gs

    st = torch.cuda.current_stream()
    rc, ctx = gs.gsyeig_create(st.cuda_stream)
    assert rc == 0
    try:
        assert gs.GSYEIG_NOALLOC_MAX_N == 16384
        for n, lda in ((16384, 16384), (3001, 3001), (700, 768), (16384, 16384)):
            say("symv_noalloc", n, lda)
            g = torch.Generator(device="cuda")
            g.manual_seed(1000 + n)
            R = torch.randn(n, n, generator=g, dtype=torch.float64, device="cuda")
            A = torch.full((n, lda), float("nan"), dtype=torch.float64, device="cuda")
            A[:, :n] = R + R.t()  # symmetric; padding columns never read
            del R
            x = torch.randn(n, generator=g, dtype=torch.float64, device="cuda")
            y0 = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
            y1 = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
            assert gs.gsyeig_symv(ctx, n, A, lda, x, y0) == 0
            assert gs.gsyeig_symv_noalloc(st.cuda_stream, n, A, lda, x, y1) == 0
            torch.cuda.synchronize()
            assert torch.equal(y0, y1), n
            # and the operation itself (a plain FP64 product as reference)
            ref = A[:, :n] @ x
            assert torch.max(torch.abs(y1 - ref)).item() <= 1e-13 * n * torch.max(torch.abs(ref)).item()
        big = gs.GSYEIG_NOALLOC_MAX_N + 1
        assert gs.gsyeig_symv_noalloc(st.cuda_stream, big, 1, big, 1, 1) == gs.GSYEIG_ETOOBIG
        assert gs.gsyeig_symv_noalloc(st.cuda_stream, 0, 1, 1, 1, 1) == -2
    finally:
        gs.gsyeig_destroy(ctx)
