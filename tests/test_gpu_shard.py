"""Sharded EDM (tdmap_edm_shard): the block index space of a launch cut into
num_shards equal ranges, one per device in a multi-device run.

The union of the shards' writes must be tdmap_edm's output bit for bit, and
the shards must write disjoint cells: checked by writing every shard into
one NaN-prefilled buffer and comparing it with the unsharded call, and by
counting each shard's cells on its own.
"""
import numpy as np
import pytest

from oracle import edm as oedm
from paper_1308_1419_amd import synth, tdmap

torch = pytest.importorskip("torch")

CASES = [  # (layout, rho, precision, N, d)
    ("full", 256, "fp32", 1037, 3),
    ("full", 128, "fp32", 700, 2),
    ("full", 64, "fp32", 513, 4),
    ("packed", 256, "fp32", 1000, 3),
    ("strict", 256, "fp32", 999, 1),
    ("packed", 128, "fp32", 640, 3),
    ("packed", 256, "bf16_gram", 1000, 64),
    ("packed", 128, "bf16_gram", 777, 32),
    ("packed", 256, "bf16x3_gram", 600, 100),
]


def _cells(N, layout):
    return {"full": N * N, "packed": oedm.tri(N), "strict": N * (N - 1) // 2}[layout]


def _written(N, layout):
    return {"full": oedm.tri(N), "packed": oedm.tri(N), "strict": N * (N - 1) // 2}[layout]


def _buffer(N, layout):
    shape = (N, N) if layout == "full" else (_cells(N, layout),)
    return torch.full(shape, float("nan"), dtype=torch.float32, device="cuda")


@pytest.mark.gpu
@pytest.mark.parametrize("layout,rho,prec,N,d", CASES)
@pytest.mark.parametrize("P", [1, 2, 3, 7])
def test_shards_union_is_the_whole_output(layout, rho, prec, N, d, P):
    assert torch.cuda.is_available(), "GPU test collected on a machine without a GPU"
    if prec == "fp32":
        X = synth.uniform_points(N, d, seed=40 + N)
    else:
        X, _ = synth.gaussian_with_near_duplicates(N, d, seed=40 + N, frac=0.05)
    Xd = torch.from_numpy(X).cuda()
    ref = _buffer(N, layout)
    tdmap.edm(Xd, layout=layout, strategy="ltm", rho=rho, precision=prec, out=ref)
    got = _buffer(N, layout)
    counts = []
    for s in range(P):
        tdmap.edm_shard(Xd, s, P, layout=layout, rho=rho, precision=prec, out=got)
        alone = _buffer(N, layout)
        tdmap.edm_shard(Xd, s, P, layout=layout, rho=rho, precision=prec, out=alone)
        counts.append(int((~torch.isnan(alone)).sum().item()))
    torch.cuda.synchronize()
    assert torch.equal(got.view(torch.int32), ref.view(torch.int32)), (layout, rho, prec, P)
    # disjoint: the shards' cell counts add up to the triangle (a shard may
    # hold only blocks past the last point, and then writes nothing)
    assert sum(counts) == _written(N, layout), (counts, _written(N, layout))


def test_shard_arguments_are_checked_before_launch():
    lib = tdmap._load()
    f = 16
    args = (f, 100, 3, 3, f, 100, tdmap.FULL, tdmap.LTM, 256, tdmap.FP32, None, 0)
    assert lib.tdmap_edm_shard(*args, -1, 2, None) == tdmap.ERR_INVALID
    assert lib.tdmap_edm_shard(*args, 2, 2, None) == tdmap.ERR_INVALID
    assert lib.tdmap_edm_shard(*args, 0, 0, None) == tdmap.ERR_INVALID
    for rho in (0, 1, 8, 16, 32):
        a = list(args)
        a[8] = rho
        assert lib.tdmap_edm_shard(*a, 0, 2, None) == tdmap.ERR_UNSUPPORTED, rho
    a = list(args)
    a[7] = tdmap.BB
    assert lib.tdmap_edm_shard(*a, 0, 2, None) == tdmap.ERR_UNSUPPORTED
    a = list(args)
    a[9] = tdmap.BF16_GRAM
    a[6] = tdmap.PACKED
    a[8] = 64
    assert lib.tdmap_edm_shard(*a, 0, 2, None) == tdmap.ERR_UNSUPPORTED
