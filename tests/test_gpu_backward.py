"""GPU parity of the EDM gradient (tdmap_edm_backward) and the autograd
Function against the FP64 oracle.

Tolerance (FP32 kernel, FP64 oracle, same dD input):
    max |dX_gpu - dX_64| <= 1e-4 * max |dX_64|   and
    ||dX_gpu - dX_64||_2 <= 1e-5 * ||dX_64||_2.
The deterministic mode must also reproduce its own bits.
"""
import numpy as np
import pytest

from oracle import edm as oedm
from oracle import native
from paper_1308_1419_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1308_1419_amd import tdmap  # noqa: E402


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test collected on a machine without a GPU")


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


def _full_from_packed(dD, N, fill=np.nan):
    F = np.full((N, N), fill, dtype=np.float32)
    for i in range(N):
        F[i, : i + 1] = dD[oedm.tri(i): oedm.tri(i) + i + 1]
    return F


@pytest.mark.parametrize("rho", [64, 128, 256, 0])
@pytest.mark.parametrize("det", [True, False])
@pytest.mark.parametrize("N,d", [(1, 3), (2, 3), (3, 1), (37, 2), (300, 3), (1000, 4), (1100, 3),
                                 (1300, 2)])
def test_backward_packed(rho, det, N, d):
    _require_gpu()
    X = synth.uniform_points(N, d, seed=40 + N + d)
    rng = np.random.default_rng(N)
    dD = rng.standard_normal(oedm.tri(N)).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    got = tdmap.edm_backward(Xd, torch.from_numpy(dD).cuda(), layout="packed", rho=rho,
                             deterministic=det)
    torch.cuda.synchronize()
    _check_grad(got.cpu().numpy(), oedm.edm_backward64(X, dD), f"N={N} d={d}")


@pytest.mark.parametrize("det", [True, False])
def test_backward_full_layout_ignores_upper_triangle(det):
    _require_gpu()
    N, d = 517, 3
    X = synth.uniform_points(N, d, seed=8)
    rng = np.random.default_rng(3)
    dD = rng.standard_normal(oedm.tri(N)).astype(np.float32)
    F = _full_from_packed(dD, N)           # NaN above the diagonal
    Fp = np.full((N, N + 3), np.nan, dtype=np.float32)
    Fp[:, :N] = F                            # and a pitch that is not N
    Xd = torch.from_numpy(X).cuda()
    for rho in (64, 128, 256):
        got = tdmap.edm_backward(Xd, torch.from_numpy(Fp).cuda(), layout="full", rho=rho,
                                 deterministic=det, ldd=N + 3)
        torch.cuda.synchronize()
        g = got.cpu().numpy()
        assert np.all(np.isfinite(g))
        _check_grad(g, oedm.edm_backward64(X, dD), f"full rho={rho}")


def test_backward_deterministic_bitwise():
    _require_gpu()
    N = 3000
    X = synth.uniform_points(N, 3, seed=12)
    dD = np.random.default_rng(5).standard_normal(oedm.tri(N)).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    dDd = torch.from_numpy(dD).cuda()
    for rho in (64, 128, 256):
        a = tdmap.edm_backward(Xd, dDd, rho=rho, deterministic=True)
        b = tdmap.edm_backward(Xd, dDd, rho=rho, deterministic=True)
        torch.cuda.synchronize()
        assert torch.equal(a.view(torch.int32), b.view(torch.int32))


@pytest.mark.parametrize("rho", [0, 64, 128, 256])
def test_backward_unaligned_dD_pointer(rho):
    # every tile reads dD with 4-byte loads: a view one float past a 16-byte
    # boundary gives the gradient of the same values
    _require_gpu()
    N = 700
    X = synth.uniform_points(N, 3, seed=14)
    dD = np.random.default_rng(6).standard_normal(oedm.tri(N)).astype(np.float32)
    buf = torch.empty(oedm.tri(N) + 1, dtype=torch.float32, device="cuda")
    buf[1:] = torch.from_numpy(dD).cuda()
    view = buf[1:]
    Xd = torch.from_numpy(X).cuda()
    got = tdmap.edm_backward(Xd, view, rho=rho, deterministic=True)
    torch.cuda.synchronize()
    _check_grad(got.cpu().numpy(), oedm.edm_backward64(X, dD), "unaligned dD")


def test_backward_tuned_decision_serves_unaligned_dD():
    # one tuner decision per (d, size) class; a call with an unaligned dD
    # after a call that tuned on an aligned one replays it correctly
    _require_gpu()
    N, d = 900, 3
    X = synth.uniform_points(N, d, seed=15)
    dD = np.random.default_rng(7).standard_normal(oedm.tri(N)).astype(np.float32)
    buf = torch.empty(oedm.tri(N) + 4, dtype=torch.float32, device="cuda")
    Xd = torch.from_numpy(X).cuda()
    tdmap.tdmap_autotune_reset()
    buf[: oedm.tri(N)] = torch.from_numpy(dD).cuda()
    tdmap.edm_backward(Xd, buf[: oedm.tri(N)], rho=0, deterministic=True)
    torch.cuda.synchronize()
    ts = tdmap.tdmap_tuned_rho(tdmap.OP_BACKWARD, 0, 0, d, N)
    assert ts in (64, 128, 256)
    buf[1: oedm.tri(N) + 1] = torch.from_numpy(dD).cuda()
    got = tdmap.edm_backward(Xd, buf[1: oedm.tri(N) + 1], rho=0, deterministic=True)
    torch.cuda.synchronize()
    assert tdmap.tdmap_tuned_rho(tdmap.OP_BACKWARD, 0, 0, d, N) == ts
    _check_grad(got.cpu().numpy(), oedm.edm_backward64(X, dD), "unaligned dD after an aligned tune")


def test_backward_coincident_points_and_zero_gradient():
    _require_gpu()
    X = synth.uniform_points(200, 3, seed=6)
    X[7] = X[2]
    X[150] = X[149]
    dD = np.zeros(oedm.tri(200), dtype=np.float32)
    dD[oedm.tri(7) + 2] = 5.0
    dD[oedm.tri(150) + 149] = -3.0
    for i in range(200):
        dD[oedm.tri(i) + i] = 1e3
    Xd = torch.from_numpy(X).cuda()
    for det in (True, False):
        got = tdmap.edm_backward(Xd, torch.from_numpy(dD).cuda(), rho=64, deterministic=det)
        torch.cuda.synchronize()
        assert np.all(got.cpu().numpy() == 0.0)


def test_autograd_stress_small_matches_fp64():
    # the small stress case, n = 64: L = sum_{j<i} (D_ij - delta_ij)^2
    _require_gpu()
    X, Xp = synth.stress_inputs(64, 3, seed=synth.workload_seed(4))
    delta = oedm.edm64_packed(Xp)
    L64, g64 = oedm.stress_grad64(X, delta)
    fd = oedm.central_differences(lambda Z: _stress_fp64(Z, delta), X, h=1e-6)
    assert np.max(np.abs(fd - g64)) <= 1e-7 * np.abs(g64).max()
    EDM = tdmap.EDM()
    Xt = torch.from_numpy(X).cuda().requires_grad_(True)
    dl = torch.from_numpy(delta.astype(np.float32)).cuda()
    D = EDM.apply(Xt)
    L = ((D - dl) ** 2).sum()
    L.backward()
    torch.cuda.synchronize()
    assert abs(float(L.detach()) - L64) <= 1e-5 * L64
    _check_grad(Xt.grad.cpu().numpy(), g64, "autograd n=64")


@pytest.mark.parametrize("rho", [1, 16, 64, 256])
def test_autograd_forward_block_sizes(rho):
    # any forward block size runs its backward: sizes the backward has no
    # tile for (the one-cell sweep, the paper's 16 x 16 blocks) fall back to
    # the autotuned backward tile
    _require_gpu()
    X, Xp = synth.stress_inputs(64, 3, seed=synth.workload_seed(4))
    delta = oedm.edm64_packed(Xp)
    L64, g64 = oedm.stress_grad64(X, delta)
    EDM = tdmap.EDM()
    Xt = torch.from_numpy(X).cuda().requires_grad_(True)
    dl = torch.from_numpy(delta.astype(np.float32)).cuda()
    D = EDM.apply(Xt, rho)
    L = ((D - dl) ** 2).sum()
    L.backward()
    torch.cuda.synchronize()
    assert abs(float(L.detach()) - L64) <= 1e-5 * L64
    _check_grad(Xt.grad.cpu().numpy(), g64, f"autograd rho={rho}")


def test_autograd_rejects_unknown_block_size():
    _require_gpu()
    Xt = torch.zeros((8, 3), dtype=torch.float32, device="cuda", requires_grad=True)
    with pytest.raises(ValueError):
        tdmap.EDM().apply(Xt, 12)


def _stress_fp64(Z, delta):
    N = Z.shape[0]
    tot = 0.0
    for i in range(N):
        r = np.sqrt(((Z[i] - Z[:i]) ** 2).sum(1)) - delta[oedm.tri(i): oedm.tri(i) + i]
        tot += float((r * r).sum())
    return tot


def test_stress_workload_full_size():
    # the 20000-point stress workload: forward, torch loss, backward; the
    # kernel is compared with the FP64 gradient of the same FP32 dD, and the
    # whole chain with the FP64 stress gradient
    _require_gpu()
    N = 20000
    X, Xp = synth.stress_inputs(N, 3, seed=synth.workload_seed(4))
    Xd = torch.from_numpy(X).cuda()
    delta = tdmap.edm(torch.from_numpy(Xp).cuda(), layout="packed", rho=0)
    D = tdmap.edm(Xd, layout="packed", rho=0)
    dD = 2.0 * (D - delta)
    for det in (True, False):
        dX = tdmap.edm_backward(Xd, dD, layout="packed", rho=0, deterministic=det)
        torch.cuda.synchronize()
        ref = native.edm_backward(X, dD.cpu().numpy())
        _check_grad(dX.cpu().numpy(), ref, f"N=20000 det={det}")
    # end to end against the FP64 stress gradient (delta from the FP64 oracle)
    delta64 = np.concatenate(native.edm_rows(Xp, range(N)))
    D64 = np.concatenate(native.edm_rows(X, range(N)))
    dD64 = 2.0 * (D64 - delta64)
    # the C oracle takes the cell gradient in FP32; the rounding of dD64 to
    # FP32 changes the gradient by far less than the tolerance
    g64 = native.edm_backward(X, dD64.astype(np.float32))
    dX = tdmap.edm_backward(Xd, 2.0 * (D - torch.from_numpy(delta64.astype(np.float32)).cuda()),
                            rho=0, deterministic=True)
    torch.cuda.synchronize()
    _check_grad(dX.cpu().numpy(), g64, "stress end to end")
