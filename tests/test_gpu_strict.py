"""GPU parity of the problem without the diagonal (Sec. II-A, Eq. (10)).

Two pieces, both called through the C ABI:
* tdmap_map_blocks_nodiag, the no-diagonal block map, bit-exact against the
  oracle's integer form (every lambda below 2^16, every row start below
  2^32 with its neighbours, and the whole 32-bit range by succession);
* the strict packed layout (cell (i, j), j < i, at i(i-1)/2 + j) written by
  the tiles and by the linear sweep, whose position -> cell map is Eq. (10):
  FP32 distances within 1e-6 relative of the FP64 oracle, nothing written
  past the N(N-1)/2 cells, and bit for bit the off-diagonal cells of the
  packed layout (one per-pair function); its gradient equals the packed
  layout's gradient bit for bit (deterministic mode), whose diagonal is
  ignored, and matches the FP64 oracle to the gradient tolerance.
"""
import numpy as np
import pytest

from oracle import edm as oedm
from oracle import maps as omaps
from oracle import native
from paper_1308_1419_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1308_1419_amd import tdmap  # noqa: E402

SENTINEL = np.int32(0x7FC0DEAD)
REL = oedm.fp32_rel_tol()


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test collected on a machine without a GPU")


def _strict_size(N):
    return N * (N - 1) // 2 if N > 0 else 0


def _check_rel(got, ref, where=""):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, where
    zero = ref == 0
    assert np.all(got[zero] == 0), f"{where}: non-zero where the exact distance is 0"
    err = np.abs(got - ref)
    bad = err > REL * ref
    if np.any(bad):
        k = int(np.argmax(err / np.where(ref > 0, ref, 1)))
        raise AssertionError(f"{where}: {int(bad.sum())} cells out of tolerance, worst "
                             f"at {k}: got {got.flat[k]!r} ref {ref.flat[k]!r}")


def _guarded(n, guard=64):
    buf = torch.empty(n + guard, dtype=torch.float32, device="cuda")
    buf.view(torch.int32).fill_(int(SENTINEL))
    return buf, buf[:n]


def _guard_ok(buf, guard=64):
    return bool(np.all(buf[-guard:].cpu().numpy().view(np.int32) == SENTINEL))


def _check_grad(got, ref, where=""):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max()
    if scale == 0:
        assert np.all(got == 0), where
        return
    err = np.abs(got - ref)
    assert err.max() <= 1e-4 * scale, f"{where}: max err {err.max()} scale {scale}"
    assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref), where


# --------------------------------------------------------------------------
# the no-diagonal map
# --------------------------------------------------------------------------

def test_map_nodiag_exact_below_2_16():
    _require_gpu()
    count = 1 << 16
    ij = tdmap.map_blocks_nodiag(0, count).cpu().numpy().astype(np.int64)
    ref = np.array([omaps.g_oracle_nodiag(lam) for lam in range(count)], dtype=np.int64)
    assert np.array_equal(ij, ref)


def test_map_nodiag_row_boundaries_exact():
    _require_gpu()
    # row i >= 2 starts at S(i) = i(i-1)/2; the last start below 2^32 is row 92682
    for i in list(range(2, 2000)) + list(range(46000, 46400)) + list(range(92000, 92683)):
        t = i * (i - 1) // 2
        ij = tdmap.map_blocks_nodiag(t - 1, 3).cpu().numpy().astype(np.int64)
        assert tuple(ij[0]) == omaps.g_oracle_nodiag(t - 1) == (i - 1, i - 2)
        assert tuple(ij[1]) == omaps.g_oracle_nodiag(t) == (i, 0)
        assert tuple(ij[2]) == omaps.g_oracle_nodiag(t + 1)
    last = (1 << 32) - 1
    ij = tdmap.map_blocks_nodiag(last, 1).cpu().numpy().astype(np.int64)
    assert tuple(ij[0]) == omaps.g_oracle_nodiag(last)


def test_map_nodiag_whole_32bit_range_by_succession():
    _require_gpu()
    chunk = 1 << 27
    out = torch.empty((chunk, 2), dtype=torch.int32, device="cuda")
    for c in range((1 << 32) // chunk):
        lam0 = c * chunk
        tdmap.map_blocks_nodiag(lam0, chunk, out=out)
        i = out[:, 0].to(torch.int64)
        j = out[:, 1].to(torch.int64)
        assert (int(i[0]), int(j[0])) == omaps.g_oracle_nodiag(lam0)
        same_row = (i[1:] == i[:-1]) & (j[1:] == j[:-1] + 1)
        next_row = (i[1:] == i[:-1] + 1) & (j[1:] == 0) & (j[:-1] == i[:-1] - 1)
        assert bool(torch.all(same_row | next_row)), f"chunk {c}"
        assert bool(torch.all((j >= 0) & (j < i)))
        last = lam0 + chunk - 1
        assert (int(i[-1]), int(j[-1])) == omaps.g_oracle_nodiag(last)
    torch.cuda.synchronize()


# --------------------------------------------------------------------------
# strict layout, forward
# --------------------------------------------------------------------------

@pytest.mark.parametrize("strategy", ["ltm", "bb"])
@pytest.mark.parametrize("rho", [64, 128, 256])
@pytest.mark.parametrize("N", [1, 2, 3, 5, 64, 257, 300, 1037])
def test_edm_strict_tiles(strategy, rho, N):
    _require_gpu()
    X = synth.uniform_points(N, 3, seed=500 + N)
    Xd = torch.from_numpy(X).cuda()
    buf, D = _guarded(_strict_size(N))
    tdmap.edm(Xd, layout="strict", strategy=strategy, rho=rho, out=D)
    torch.cuda.synchronize()
    _check_rel(D.cpu().numpy(), oedm.edm64_strict(X), f"strict {strategy} {rho} N={N}")
    assert _guard_ok(buf), "wrote past the end"


@pytest.mark.parametrize("d", [1, 2, 3, 4])
@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 31, 64, 1000, 1025, 1037, 2900])
def test_edm_strict_sweep(N, d):
    # rho = 1: positions mapped to cells by Eq. (10), written in address order
    _require_gpu()
    X = synth.uniform_points(N, d, seed=600 + N + d)
    Xd = torch.from_numpy(X).cuda()
    buf, D = _guarded(_strict_size(N))
    tdmap.edm(Xd, layout="strict", strategy="ltm", rho=1, out=D)
    torch.cuda.synchronize()
    _check_rel(D.cpu().numpy(), oedm.edm64_strict(X), f"strict sweep N={N} d={d}")
    assert _guard_ok(buf), "wrote past the end"
    R = tdmap.edm(Xd, layout="strict", strategy="ltm", rho=64)
    assert torch.equal(D.view(torch.int32), R.view(torch.int32))


def test_edm_strict_single_point_has_no_cells():
    _require_gpu()
    X = torch.from_numpy(synth.uniform_points(1, 3, seed=1)).cuda()
    for rho in (0, 1, 64, 256):
        D = tdmap.edm(X, layout="strict", strategy="ltm", rho=rho)
        assert D.numel() == 0
    torch.cuda.synchronize()


@pytest.mark.parametrize("rho", [0, 1, 64, 128, 256])
def test_edm_strict_equals_packed_off_diagonal(rho):
    _require_gpu()
    N = 2049
    X = synth.uniform_points(N, 3, seed=77)
    Xd = torch.from_numpy(X).cuda()
    S = tdmap.edm(Xd, layout="strict", strategy="ltm", rho=rho)
    P = tdmap.edm(Xd, layout="packed", strategy="ltm", rho=16)
    torch.cuda.synchronize()
    rows = torch.arange(N, device="cuda", dtype=torch.int64)
    diag = rows * (rows + 1) // 2 + rows
    keep = torch.ones(P.numel(), dtype=torch.bool, device="cuda")
    keep[diag] = False
    assert torch.equal(P[keep].view(torch.int32), S.view(torch.int32))


# --------------------------------------------------------------------------
# strict layout, backward
# --------------------------------------------------------------------------

def _packed_from_strict(dS, N, diag_value):
    dP = np.empty(oedm.tri(N), dtype=np.float32)
    for i in range(N):
        s = i * (i - 1) // 2
        dP[oedm.tri(i): oedm.tri(i) + i] = dS[s: s + i]
        dP[oedm.tri(i) + i] = diag_value
    return dP


@pytest.mark.parametrize("rho", [64, 128, 256])
@pytest.mark.parametrize("N,d", [(1, 3), (2, 3), (37, 2), (300, 3), (1037, 4)])
def test_backward_strict(rho, N, d):
    _require_gpu()
    X = synth.uniform_points(N, d, seed=700 + N + d)
    rng = np.random.default_rng(N + 1)
    dS = rng.standard_normal(_strict_size(N)).astype(np.float32)
    dP = _packed_from_strict(dS, N, diag_value=123.0)  # the diagonal is ignored
    Xd = torch.from_numpy(X).cuda()
    if N > 1:
        dS_d = torch.from_numpy(dS).cuda()
    else:
        dS_d = torch.empty(0, dtype=torch.float32, device="cuda")
    g_s = tdmap.edm_backward(Xd, dS_d, layout="strict", rho=rho, deterministic=True)
    g_p = tdmap.edm_backward(Xd, torch.from_numpy(dP).cuda(), layout="packed", rho=rho,
                             deterministic=True)
    torch.cuda.synchronize()
    assert torch.equal(g_s.view(torch.int32), g_p.view(torch.int32))
    _check_grad(g_s.cpu().numpy(), oedm.edm_backward64(X, dP), f"strict N={N} rho={rho}")
    g_a = tdmap.edm_backward(Xd, dS_d, layout="strict", rho=rho, deterministic=False)
    torch.cuda.synchronize()
    _check_grad(g_a.cpu().numpy(), oedm.edm_backward64(X, dP), f"strict atomic N={N}")


# --------------------------------------------------------------------------
# 30000 points (the full-size workload's points), strict layout
# --------------------------------------------------------------------------

def test_big_strict_sampled_rows_and_sweep_vs_tiles():
    _require_gpu()
    N = 30000
    X = synth.uniform_points(N, 3, seed=synth.workload_seed(2))
    Xd = torch.from_numpy(X).cuda()
    A = tdmap.edm(Xd, layout="strict", strategy="ltm", rho=1)
    B = tdmap.edm(Xd, layout="strict", strategy="ltm", rho=256)
    torch.cuda.synchronize()
    assert torch.equal(A.view(torch.int32), B.view(torch.int32))
    rows = synth.sample_rows(N, 64, seed=6) + [1, 2, 255, 256, 1023, 1024, 1025, 29999]
    rows = sorted(set(r for r in rows if r >= 1))
    exp = native.edm_rows(X, rows)
    for i, e in zip(rows, exp):
        s = i * (i - 1) // 2
        _check_rel(A[s: s + i].cpu().numpy(), e[:i], f"row {i}")
    del A, B
    torch.cuda.empty_cache()
