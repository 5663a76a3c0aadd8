"""GPU parity of the Gram-form EDM on MFMA (precisions BF16_GRAM and the
split BF16X3_GRAM).

Bars, per pair (i, j), against the FP64 oracle distance D of the FP32 points:
* every pair: |D_gpu - D| <= gram_bound(||x_i||, ||x_j||, D, d, split) (the
  stated bound of a pair that is not recomputed, for the precision used) or
  within the FP32 rule 1e-6 D (a recomputed pair);
* the diagonal is exactly 0 and every planted near-duplicate pair (those
  sit far below the recompute threshold) meets the FP32 rule.
"""
import numpy as np
import pytest

from oracle import edm as oedm
from oracle import native
from paper_1308_1419_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1308_1419_amd import tdmap  # noqa: E402

REL = oedm.fp32_rel_tol()


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test collected on a machine without a GPU")


PRECS = ["bf16_gram", "bf16x3_gram"]


def _check_rows(X, rows, got_rows, split=False):
    """got_rows[r] holds row rows[r] (i+1 values) of the GPU triangle."""
    d = X.shape[1]
    X64 = X.astype(np.float64)
    norms = np.linalg.norm(X64, axis=1)
    ref_rows = native.edm_rows(X, rows)
    stats = {"max_abs": 0.0, "max_rel": 0.0, "n": 0, "sq_rel": 0.0, "fp32_rule": 0}
    for i, got, ref in zip(rows, got_rows, ref_rows):
        got = np.asarray(got, dtype=np.float64)
        assert got[i] == 0.0, f"diagonal ({i},{i}) = {got[i]}"
        bound = oedm.gram_bound(norms[i], norms[: i + 1], ref, d, split=split)
        err = np.abs(got - ref)
        ok = (err <= bound) | (err <= REL * ref)
        assert np.all(ok), f"row {i}: {int((~ok).sum())} pairs out of bound, worst " \
                           f"{err[~ok].max()} vs {bound[~ok].min()}"
        nz = ref > 0
        stats["max_abs"] = max(stats["max_abs"], float(err.max()))
        if nz.any():
            rel = err[nz] / ref[nz]
            stats["max_rel"] = max(stats["max_rel"], float(rel.max()))
            stats["sq_rel"] += float(np.dot(rel, rel))
        stats["fp32_rule"] += int(np.sum(err <= REL * ref))
        stats["n"] += len(ref)
    stats["rms_rel"] = (stats["sq_rel"] / max(stats["n"], 1)) ** 0.5
    return stats


# feature counts covering every padded width the kernels are compiled for
# (16, 32, 64, 128) and the run-time loop (48, 112, 144), at the ends of
# each width's range
DS = [1, 3, 16, 17, 32, 33, 64, 100, 113, 128, 129]
NS = [1, 2, 15, 16, 17, 63, 64, 65, 127, 128, 129, 255, 256, 257, 300, 1000]
# Gram tile edges: 0 = the autotuned choice, plus each kernel on its own
RHOS = [0, 128, 256]


def _gram(Xd, prec, rho=0, out=None):
    return tdmap.edm(Xd, layout="packed", strategy="ltm", rho=rho, precision=prec, out=out)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("N", NS)
@pytest.mark.parametrize("d", DS)
def test_gram_small(N, d, prec):
    _require_gpu()
    X, pairs = synth.gaussian_with_near_duplicates(N, d, seed=500 + N + d, frac=0.05)
    Xd = torch.from_numpy(X).cuda()
    D = _gram(Xd, prec)
    torch.cuda.synchronize()
    Dh = D.cpu().numpy()
    rows = list(range(N))
    got_rows = [Dh[oedm.tri(i): oedm.tri(i) + i + 1] for i in rows]
    _check_rows(X, rows, got_rows, split=prec == "bf16x3_gram")
    ref = oedm.edm64_packed(X)
    for c, s in pairs:
        i, j = max(c, s), min(c, s)
        k = oedm.tri(i) + j
        assert abs(Dh[k] - ref[k]) <= REL * ref[k], (i, j, Dh[k], ref[k])


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("rho", RHOS)
@pytest.mark.parametrize("shift", [0, 1, 2, 3])
@pytest.mark.parametrize("N,d", [(300, 64), (1000, 17), (517, 128)])
def test_gram_output_offsets(N, d, shift, rho, prec):
    # outputs that start 4, 8 or 12 bytes past a 16-byte boundary: the
    # kernels take the alignment of every row from the real address; the
    # cells before and after the triangle stay untouched
    _require_gpu()
    X, pairs = synth.gaussian_with_near_duplicates(N, d, seed=900 + N + d, frac=0.05)
    Xd = torch.from_numpy(X).cuda()
    T = oedm.tri(N)
    buf = torch.full((T + 8,), float("nan"), dtype=torch.float32, device="cuda")
    out = buf[shift: shift + T]
    _gram(Xd, prec, rho=rho, out=out)
    torch.cuda.synchronize()
    Bh = buf.cpu().numpy()
    assert np.all(np.isnan(Bh[:shift])) and np.all(np.isnan(Bh[shift + T:]))
    Dh = Bh[shift: shift + T]
    got_rows = [Dh[oedm.tri(i): oedm.tri(i) + i + 1] for i in range(N)]
    _check_rows(X, list(range(N)), got_rows, split=prec == "bf16x3_gram")


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("rho", [128, 256])
@pytest.mark.parametrize("N,d", [(1000, 64), (777, 32), (600, 100)])
def test_gram_kernels_bitwise_equal(N, d, rho, prec):
    # the tile and strip kernels share the operand rounding, the MFMA
    # products in one order and the epilogue: their outputs are equal bit
    # for bit, also against the autotuned call
    _require_gpu()
    X, _ = synth.gaussian_with_near_duplicates(N, d, seed=31 + N, frac=0.05)
    Xd = torch.from_numpy(X).cuda()
    a = _gram(Xd, prec, rho=0)
    b = _gram(Xd, prec, rho=rho)
    torch.cuda.synchronize()
    assert torch.equal(a.view(torch.int32), b.view(torch.int32))


def _bf16(x):
    """FP32 -> BF16 round to nearest even, returned as FP32 values (the
    rounding the Gram prologue applies)."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("rho", [128, 256])
def test_gram_recompute_count(prec, rho):
    # the instrumented launch writes the same output as the timed one and
    # counts the pairs that took the FP32 recompute; those are the pairs
    # with G <= (n_i + n_j) / 4 for the represented (BF16 or hi + lo)
    # points, which FP64 decides for every pair farther than 1e-4 (n_i + n_j)
    # from the threshold (FP32 accumulation error is about 4e-6 of it here)
    _require_gpu()
    N, d = 1000, 64
    X, pairs = synth.gaussian_with_near_duplicates(N, d, seed=123, frac=0.05)
    Xd = torch.from_numpy(X).cuda()
    D, cnt = tdmap.gram_recompute_count(Xd, prec, rho=rho)
    ref = _gram(Xd, prec, rho=rho)
    torch.cuda.synchronize()
    assert torch.equal(D.view(torch.int32), ref.view(torch.int32))
    hi = _bf16(X)
    rep = hi.astype(np.float64)
    if prec == "bf16x3_gram":
        rep = rep + _bf16(X - hi).astype(np.float64)
    n = np.sum(rep * rep, axis=1)
    G = n[:, None] + n[None, :] - 2.0 * rep @ rep.T
    thr = 0.25 * (n[:, None] + n[None, :])
    lower = np.tril(np.ones((N, N), dtype=bool))
    surely = lower & (G - thr < -1e-4 * (n[:, None] + n[None, :]))
    maybe = lower & (G - thr <= 1e-4 * (n[:, None] + n[None, :]))
    c = int(cnt.item())
    assert int(surely.sum()) <= c <= int(maybe.sum()), (c, int(surely.sum()), int(maybe.sum()))
    # the diagonal and the planted pairs are all below the threshold
    assert c >= N + len(pairs)


@pytest.mark.parametrize("prec", PRECS)
def test_gram_rejects_other_layouts(prec):
    _require_gpu()
    X = torch.from_numpy(synth.uniform_points(100, 64, seed=1)).cuda()
    with pytest.raises(tdmap.TdmapError):
        tdmap.edm(X, layout="full", strategy="ltm", rho=0, precision=prec)
    with pytest.raises(tdmap.TdmapError):
        tdmap.edm(X, layout="packed", strategy="bb", rho=0, precision=prec)
    with pytest.raises(tdmap.TdmapError):
        tdmap.edm(X, layout="strict", strategy="ltm", rho=0, precision=prec)


def test_split_is_far_more_accurate():
    # the same points through both precisions: the split form's largest
    # error is far below the BF16 form's
    _require_gpu()
    N, d = 2000, 64
    X, _ = synth.gaussian_with_near_duplicates(N, d, seed=77)
    Xd = torch.from_numpy(X).cuda()
    ref = oedm.edm64_packed(X)
    errs = {}
    for prec in PRECS:
        D = tdmap.edm(Xd, layout="packed", strategy="ltm", rho=0, precision=prec)
        torch.cuda.synchronize()
        errs[prec] = float(np.abs(D.cpu().numpy().astype(np.float64) - ref).max())
    assert errs["bf16x3_gram"] * 50 < errs["bf16_gram"], errs


@pytest.mark.parametrize("prec", PRECS)
def test_gram_workload_full_size(prec):
    # the 100000-point, d = 64 workload at the launch the benchmark times:
    # 2048 seeded rows, the rows of all 1000 planted near-duplicate pairs and
    # the tile-edge rows, whole, against the C oracle; every planted pair
    # against the FP32 rule; the whole diagonal exactly 0
    _require_gpu()
    N, d = 100000, 64
    X, pairs = synth.gaussian_with_near_duplicates(N, d, seed=synth.workload_seed(3))
    Xd = torch.from_numpy(X).cuda()
    D = tdmap.edm(Xd, layout="packed", strategy="ltm", rho=0, precision=prec)
    torch.cuda.synchronize()
    diag = torch.arange(N, device="cuda", dtype=torch.int64)
    diag = diag * (diag + 1) // 2 + diag
    assert bool(torch.all(D.index_select(0, diag) == 0)), "non-zero diagonal cell"
    rows = set(synth.sample_rows(N, 2048, seed=11))
    rows.update(int(max(c, s)) for c, s in pairs)
    rows.update({0, 1, 63, 64, 127, 128, 255, 256, 99967, 99968, N - 1})
    rows = sorted(rows)
    got_rows = []
    for i in rows:
        k = oedm.tri(i)
        got_rows.append(D[k: k + i + 1].cpu().numpy())
    stats = _check_rows(X, rows, got_rows, split=prec == "bf16x3_gram")
    print(f"{prec} N=100000 d=64: {stats['n']} pairs checked, max abs err {stats['max_abs']:.3e}, "
          f"max rel err {stats['max_rel']:.3e}, rms rel err {stats['rms_rel']:.3e}, "
          f"{stats['fp32_rule']} pairs within 1e-6 relative", flush=True)
    # every planted pair meets the FP32 rule
    idx = torch.as_tensor([oedm.tri(int(max(c, s))) + int(min(c, s)) for c, s in pairs],
                          device="cuda")
    got = D.index_select(0, idx).cpu().numpy().astype(np.float64)
    X64 = X.astype(np.float64)
    ref = np.linalg.norm(X64[pairs[:, 0]] - X64[pairs[:, 1]], axis=1)
    assert np.all(np.abs(got - ref) <= REL * ref)
