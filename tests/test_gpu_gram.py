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


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("N", [1, 2, 15, 16, 17, 63, 64, 65, 127, 128, 129, 255, 256, 257, 300, 1000])
@pytest.mark.parametrize("d", [1, 3, 16, 33, 64, 100])
def test_gram_small(N, d, prec):
    _require_gpu()
    X, pairs = synth.gaussian_with_near_duplicates(N, d, seed=500 + N + d, frac=0.05)
    Xd = torch.from_numpy(X).cuda()
    D = tdmap.edm(Xd, layout="packed", strategy="ltm", rho=0, precision=prec)
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
    # the 100000-point, d = 64 workload: sampled rows (seeded rows, the rows
    # of every planted near-duplicate pair, the first and last rows) against
    # the C oracle; the diagonal of every sampled row is exactly 0
    _require_gpu()
    N, d = 100000, 64
    X, pairs = synth.gaussian_with_near_duplicates(N, d, seed=synth.workload_seed(3))
    Xd = torch.from_numpy(X).cuda()
    D = tdmap.edm(Xd, layout="packed", strategy="ltm", rho=0, precision=prec)
    torch.cuda.synchronize()
    rows = set(synth.sample_rows(N, 512, seed=11))
    rows.update(int(max(c, s)) for c, s in pairs[:200])
    rows.update({63, 64, 127, 128, 99967, 99968})
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
