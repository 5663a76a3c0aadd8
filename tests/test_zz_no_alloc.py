"""The allocation-free Gram entry point (tdmap_edm_gram_noalloc) against
tdmap_edm, the entry point that takes a caller's workspace.

Both run the same kernels, so the outputs must be equal bit for bit: that
is checked on two calls in a row on one GPU, the second with a smaller
input (the static array keeps the first call's contents, which the second
must not depend on), for both Gram precisions and each kernel choice, and
with guard cells around the output.  The size limit and the argument checks
are host-side and run without a GPU.
"""
import ctypes

import numpy as np
import pytest

from paper_1308_1419_amd import synth, tdmap

torch = pytest.importorskip("torch")

PRECS = {"bf16_gram": tdmap.BF16_GRAM, "bf16x3_gram": tdmap.BF16X3_GRAM}
SCRATCH = 32 << 20


def _noalloc(Xd, prec, rho, out):
    N, d = Xd.shape
    tdmap.tdmap_edm_gram_noalloc(Xd.data_ptr(), N, d, Xd.stride(0), out.data_ptr(),
                                 PRECS[prec], rho, torch.cuda.current_stream().cuda_stream)


def _guarded(T, shift):
    buf = torch.full((T + 8,), float("nan"), dtype=torch.float32, device="cuda")
    return buf, buf[shift: shift + T]


@pytest.mark.gpu
@pytest.mark.parametrize("prec", list(PRECS))
@pytest.mark.parametrize("rho", [0, 128, 256])
def test_noalloc_equals_workspace_entry_point(prec, rho):
    assert torch.cuda.is_available(), "GPU test collected on a machine without a GPU"
    cases = [(3000, 64, 1, 0), (700, 17, 2, 3)]  # (N, d, seed, output shift)
    for N, d, seed, shift in cases:
        X, _ = synth.gaussian_with_near_duplicates(N, d, seed=seed, frac=0.05)
        Xd = torch.from_numpy(X).cuda()
        T = N * (N + 1) // 2
        ref = tdmap.edm(Xd, layout="packed", strategy="ltm", rho=rho, precision=prec)
        buf, out = _guarded(T, shift)
        _noalloc(Xd, prec, rho, out)
        torch.cuda.synchronize()
        assert torch.equal(out.view(torch.int32), ref.view(torch.int32)), (N, d, prec, rho)
        assert bool(torch.isnan(buf[:shift]).all()) and bool(torch.isnan(buf[shift + T:]).all())


@pytest.mark.gpu
@pytest.mark.parametrize("prec", list(PRECS))
def test_noalloc_at_the_largest_workload(prec):
    # the 100000-point, d = 64 workload fits the static array in both
    # precisions; the second call is smaller
    assert torch.cuda.is_available(), "GPU test collected on a machine without a GPU"
    for N, d, seed in [(100000, 64, synth.workload_seed(3)), (5000, 100, 7)]:
        X, _ = synth.gaussian_with_near_duplicates(N, d, seed=seed)
        Xd = torch.from_numpy(X).cuda()
        ref = tdmap.edm(Xd, layout="packed", strategy="ltm", rho=256, precision=prec)
        out = torch.empty_like(ref)
        _noalloc(Xd, prec, 256, out)
        torch.cuda.synchronize()
        assert torch.equal(out.view(torch.int32), ref.view(torch.int32)), (N, d, prec)
        del ref, out


def test_noalloc_size_limit_and_arguments():
    # host-side checks: nothing is launched for these calls
    lib = tdmap._load()
    for prec in PRECS.values():
        for N, d in [(100000, 64), (1000, 128), (1, 1)]:
            assert lib.tdmap_workspace_size(tdmap.OP_EDM, N, d, 0, 0, prec) <= SCRATCH
        # the smallest N past the array for d = 64
        N = 260000 if prec == tdmap.BF16_GRAM else 130000
        assert lib.tdmap_workspace_size(tdmap.OP_EDM, N, 64, 0, 0, prec) > SCRATCH
        fake = ctypes.c_void_p(16)
        assert lib.tdmap_edm_gram_noalloc(fake, N, 64, 64, fake, prec, 0, None) == \
            tdmap.ERR_UNSUPPORTED
        assert lib.tdmap_edm_gram_noalloc(fake, 100, 64, 64, fake, prec, 64, None) == \
            tdmap.ERR_UNSUPPORTED
        assert lib.tdmap_edm_gram_noalloc(None, 100, 64, 64, fake, prec, 0, None) == \
            tdmap.ERR_INVALID
        assert lib.tdmap_edm_gram_noalloc(fake, 100, 64, 32, fake, prec, 0, None) == \
            tdmap.ERR_INVALID
        assert lib.tdmap_edm_gram_noalloc(None, 0, 64, 64, None, prec, 0, None) == tdmap.OK
    assert lib.tdmap_edm_gram_noalloc(ctypes.c_void_p(16), 100, 64, 64, ctypes.c_void_p(16),
                                      tdmap.FP32, 0, None) == tdmap.ERR_INVALID
