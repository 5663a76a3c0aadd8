"""GPU parity at the size limits: launches that the library splits because a
single HIP launch would pass 2^32 work-items, and packed indices past 2^32.

* tdmap_map_blocks over 2^31 + 2^20 block indices ending at 2^32 (two
  launches): bit-exact against the oracle at both ends and at the launch
  boundary, and a row-major succession everywhere in between.
* N = 93000 points in the packed layout (4,324,546,500 cells, so packed
  positions pass 2^32): the one-cell-per-thread LTM launch needs two
  launches at every rho in {8, 16, 32}; its output, and that of the
  256-cell strips, equals the linear sweep's bit for bit, and the sweep
  (64-bit g(lambda)) is checked against the FP64 oracle on rows around both
  launch boundaries, around position 2^32, and at seeded rows.
"""
import math

import numpy as np
import pytest

from oracle import edm as oedm
from oracle import maps as omaps
from oracle import native
from paper_1308_1419_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1308_1419_amd import tdmap  # noqa: E402

REL = oedm.fp32_rel_tol()


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test collected on a machine without a GPU")


def _check_rel(got, ref, where=""):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, where
    assert np.all(got[ref == 0] == 0), where
    err = np.abs(got - ref)
    assert np.all(err <= REL * ref), f"{where}: worst {err.max()}"


def test_map_blocks_split_launch_to_2_32():
    _require_gpu()
    count = (1 << 31) + (1 << 20)
    lam0 = (1 << 32) - count
    out = torch.empty((count, 2), dtype=torch.int32, device="cuda")
    tdmap.map_blocks(lam0, count, out=out)
    torch.cuda.synchronize()
    # both ends and the first lambda of the second launch (2^31 lanes each)
    for t in (0, 1, (1 << 31) - 1, 1 << 31, (1 << 31) + 1, count - 1):
        i, j = (int(v) & 0xFFFFFFFF for v in out[t].tolist())
        assert (i, j) == omaps.g_oracle(lam0 + t), t
    chunk = 1 << 27
    for c0 in range(0, count, chunk):
        c1 = min(count, c0 + chunk + 1)  # overlap by one to join the slices
        i = out[c0:c1, 0].to(torch.int64)
        j = out[c0:c1, 1].to(torch.int64)
        same_row = (i[1:] == i[:-1]) & (j[1:] == j[:-1] + 1)
        next_row = (i[1:] == i[:-1] + 1) & (j[1:] == 0) & (j[:-1] == i[:-1])
        assert bool(torch.all(same_row | next_row)), c0
        assert bool(torch.all(j <= i)), c0
    del out
    torch.cuda.empty_cache()


N_BIG = 93000


@pytest.fixture(scope="module")
def big_packed():
    _require_gpu()
    X = synth.uniform_points(N_BIG, 3, seed=synth.workload_seed(2) + 7)
    Xd = torch.from_numpy(X).cuda()
    total = N_BIG * (N_BIG + 1) // 2
    assert total > (1 << 32)
    S = torch.empty(total, dtype=torch.float32, device="cuda")
    tdmap.edm(Xd, layout="packed", strategy="ltm", rho=1, out=S)
    torch.cuda.synchronize()
    yield X, Xd, S
    del S
    torch.cuda.empty_cache()


def _rows_at(pos):
    """Row of packed position pos."""
    return (math.isqrt(8 * pos + 1) - 1) // 2


def test_sweep_past_2_32_against_oracle(big_packed):
    X, Xd, S = big_packed
    rows = set(synth.sample_rows(N_BIG, 24, seed=12))
    r32 = _rows_at(1 << 32)
    rows.update({r32 - 1, r32, r32 + 1, 1023, 1024, N_BIG - 1})
    for rho in (8, 16, 32):
        # the first row of the tile row where the second launch starts
        max_blocks = ((1 << 32) - 1) // (rho * rho)
        I, _ = omaps.g_oracle(max_blocks)
        rows.update({I * rho - 1, I * rho, I * rho + rho - 1})
    rows = sorted(r for r in rows if 0 <= r < N_BIG)
    ref = native.edm_rows(X, rows)
    for i, e in zip(rows, ref):
        k = oedm.tri(i)
        _check_rel(S[k: k + i + 1].cpu().numpy(), e, f"row {i}")


def test_strips_past_2_32_equal_sweep(big_packed):
    # the 256-cell strips (8-row work-groups, 64-bit packed offsets past
    # 2^32) write the same bits as the linear sweep
    X, Xd, S = big_packed
    C = torch.empty_like(S)
    tdmap.edm(Xd, layout="packed", strategy="ltm", rho=256, out=C)
    torch.cuda.synchronize()
    assert torch.equal(C.view(torch.int32), S.view(torch.int32))
    del C
    torch.cuda.empty_cache()


@pytest.mark.parametrize("rho", [8, 16, 32])
def test_split_cell_launch_equals_sweep(big_packed, rho):
    X, Xd, S = big_packed
    nb = -(-N_BIG // rho)
    assert nb * (nb + 1) // 2 * rho * rho > (1 << 32)  # needs two launches
    C = torch.empty_like(S)
    tdmap.edm(Xd, layout="packed", strategy="ltm", rho=rho, out=C)
    torch.cuda.synchronize()
    assert torch.equal(C.view(torch.int32), S.view(torch.int32))
    del C
    torch.cuda.empty_cache()
