"""GPU parity of the batched persistent EDM (tdmap_edm_batched).

Bars: every set's packed triangle within 1e-6 relative of the FP64 oracle
(exact zeros on the diagonal); bit-identical to tdmap_edm on the set alone
(one per-pair function); every output cell written and nothing past the
last set touched.
"""
import numpy as np
import pytest

from oracle import edm as oedm
from oracle import native
from paper_1308_1419_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1308_1419_amd import tdmap  # noqa: E402

SENTINEL = 0x7FC0DEAD
REL = oedm.fp32_rel_tol()


def _require_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test collected on a machine without a GPU")


def _check_rel(got, ref, where=""):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, where
    assert np.all(got[ref == 0] == 0), where
    bad = np.abs(got - ref) > REL * ref
    assert not np.any(bad), f"{where}: {int(bad.sum())} cells out of tolerance"


def _run(sizes, d, rho, seed, guard=256):
    rng = np.random.default_rng(seed)
    sizes = np.asarray(sizes, dtype=np.int64)
    point_off = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=point_off[1:])
    out_off = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes * (sizes + 1) // 2, out=out_off[1:])
    X = rng.random((int(point_off[-1]), d), dtype=np.float32)
    total = int(out_off[-1])
    buf = torch.empty(total + guard, dtype=torch.float32, device="cuda")
    buf.view(torch.int32).fill_(SENTINEL)
    # the ABI wants a non-NULL X_cat even when every set is empty
    Xd = torch.from_numpy(X).cuda() if len(X) else torch.zeros((1, d), device="cuda")
    tdmap.edm_batched(Xd, torch.from_numpy(point_off).cuda(), torch.from_numpy(out_off).cuda(),
                      rho=rho, out=buf[:total] if total else buf)
    torch.cuda.synchronize()
    return X, point_off, out_off, buf


@pytest.mark.parametrize("rho", [1, 64, 128, 0])
@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_batched_ragged_sets(rho, d):
    _require_gpu()
    sizes = [5, 0, 1, 2, 63, 64, 65, 0, 200, 129, 300, 7, 255, 256, 257, 520, 0, 1030]
    X, po, oo, buf = _run(sizes, d, rho, seed=d * 10 + rho)
    got = buf.cpu().numpy()
    ref = oedm.edm64_batched(X, po)
    _check_rel(got[: len(ref)], ref, f"rho={rho} d={d}")
    assert np.all(got.view(np.int32)[len(ref):] == SENTINEL), "wrote past the last set"
    # bitwise equal to single-set calls
    Xd = torch.from_numpy(X).cuda()
    for s, n in enumerate(sizes):
        if n == 0:
            continue
        one = tdmap.edm(Xd[po[s]: po[s + 1]].contiguous(), layout="packed", strategy="ltm", rho=16)
        torch.cuda.synchronize()
        assert torch.equal(one.view(torch.int32), buf[oo[s]: oo[s + 1]].view(torch.int32)), s


@pytest.mark.parametrize("rho", [1, 64, 128])
def test_batched_empty_and_single(rho):
    _require_gpu()
    X, po, oo, buf = _run([0, 0, 0], 3, rho, seed=1)
    assert np.all(buf.cpu().numpy().view(np.int32) == SENTINEL)
    X, po, oo, buf = _run([1], 3, rho, seed=2)
    assert buf[0].item() == 0.0
    assert np.all(buf.cpu().numpy().view(np.int32)[1:] == SENTINEL)
    # no sets at all is a no-op
    tdmap.tdmap_edm_batched(0, 3, 0, 0, 0, 0, 64, 0, 0, 0)


@pytest.mark.parametrize("rho", [1, 64, 0])
def test_batched_many_small_sets(rho):
    # sizes 0..139: the sweep crosses many set boundaries inside one thread
    _require_gpu()
    rng = np.random.default_rng(9)
    sizes = rng.integers(0, 140, size=3000)
    sizes[:40] = [0, 1, 2, 1, 0, 0, 3, 1, 1, 2] * 4
    X, po, oo, buf = _run(sizes, 3, rho, seed=3)
    got = buf.cpu().numpy()
    ref = oedm.edm64_batched(X, po)
    _check_rel(got[: len(ref)], ref, f"3000 small sets rho={rho}")
    assert np.all(got.view(np.int32)[len(ref):] == SENTINEL)


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_batched_sets_beyond_lds(d):
    # the linear sweep stages a set's points in 64 KB of LDS (16384 / d
    # points); a larger set, and the chunk at the end of every set, take the
    # path that maps each position on its own and reads global memory.
    # Sets at the cap, one past it and far past it, between small and empty
    # ones; every walk writes the same bits as the tiles.
    _require_gpu()
    cap = 16384 // d
    sizes = [300, cap + 1, 0, 1, cap, 777, 2, cap + 1000, 9]
    X, po, oo, buf = _run(sizes, d, 1, seed=40 + d)
    total = int(oo[-1])
    assert bool(torch.all(buf.view(torch.int32)[total:] == SENTINEL)), "wrote past the last set"
    Xd = torch.from_numpy(X).cuda()
    other = torch.empty(total, dtype=torch.float32, device="cuda")
    tdmap.edm_batched(Xd, torch.from_numpy(po).cuda(), torch.from_numpy(oo).cuda(), rho=64, out=other)
    torch.cuda.synchronize()
    assert torch.equal(other.view(torch.int32), buf[:total].view(torch.int32))
    for s, n in enumerate(sizes):
        if n == 0:
            continue
        pts = X[po[s]: po[s + 1]]
        rows = range(n) if n <= 2000 else sorted({0, 1, n // 3, n // 2, n - 2, n - 1}
                                                  | set(range(cap - 3, min(cap + 3, n))))
        ref = native.edm_rows(pts, rows)
        for r, row in zip(rows, ref):
            a = int(oo[s]) + r * (r + 1) // 2
            _check_rel(buf[a: a + r + 1].cpu().numpy(), row, f"d={d} set {s} (n={n}) row {r}")


def test_batched_unaligned_output():
    # every walk takes an output at any 4-byte offset; the tuner's choice
    # is shared by aligned and unaligned calls
    _require_gpu()
    sizes = [700, 3, 0, 1500, 64]
    X, po, oo, buf = _run(sizes, 3, 64, seed=77)
    total = int(oo[-1])
    Xd = torch.from_numpy(X).cuda()
    pod, ood = torch.from_numpy(po).cuda(), torch.from_numpy(oo).cuda()
    for rho in (1, 64, 128, 0):
        for shift in (1, 2, 3):
            other = torch.empty(total + 8, dtype=torch.float32, device="cuda")
            other.view(torch.int32).fill_(SENTINEL)
            tdmap.edm_batched(Xd, pod, ood, rho=rho, out=other[shift: shift + total])
            torch.cuda.synchronize()
            assert torch.equal(other[shift: shift + total].view(torch.int32),
                               buf[:total].view(torch.int32)), (rho, shift)
            bits = other.view(torch.int32)
            assert bool(torch.all(bits[:shift] == SENTINEL)) and bool(torch.all(bits[shift + total:] == SENTINEL))


def test_batched_output_offsets_not_from_zero():
    # out_off[0] > 0: set 0 starts inside D_cat; every walk writes exactly
    # [out_off[0], out_off[S]) and agrees bitwise
    _require_gpu()
    sizes = np.array([900, 0, 5, 1300], dtype=np.int64)
    rng = np.random.default_rng(21)
    po = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    shift = 37
    oo = (shift + np.concatenate([[0], np.cumsum(sizes * (sizes + 1) // 2)])).astype(np.int64)
    X = rng.random((int(po[-1]), 3), dtype=np.float32)
    Xd = torch.from_numpy(X).cuda()
    pod, ood = torch.from_numpy(po).cuda(), torch.from_numpy(oo).cuda()
    total = int(oo[-1])
    ref = oedm.edm64_batched(X, po)
    first = None
    for rho in (1, 64, 128):
        buf = torch.empty(total + 64, dtype=torch.float32, device="cuda")
        buf.view(torch.int32).fill_(SENTINEL)
        tdmap.edm_batched(Xd, pod, ood, rho=rho, out=buf[:total])
        torch.cuda.synchronize()
        bits = buf.view(torch.int32)
        assert bool(torch.all(bits[:shift] == SENTINEL)), f"rho={rho} wrote before out_off[0]"
        assert bool(torch.all(bits[total:] == SENTINEL)), f"rho={rho} wrote past the last set"
        _check_rel(buf[shift:total].cpu().numpy(), ref, f"rho={rho}")
        if first is None:
            first = bits[:total].clone()
        assert torch.equal(bits[:total], first), rho


def test_batched_workload_full_size():
    # the 4096-set workload (n uniform in [64, 4096]); 256 seeded sets plus
    # the smallest and the largest are compared with the C oracle, every
    # cell is checked to be written, and nothing past the end
    _require_gpu()
    data = synth.batched_sets(4096, 64, 4096, 3, seed=synth.workload_seed(5))
    X, po, oo, sizes = data["X"], data["point_off"], data["out_off"], data["sizes"]
    total = int(oo[-1])
    buf = torch.empty(total + 1024, dtype=torch.float32, device="cuda")
    buf.view(torch.int32).fill_(SENTINEL)
    Xd = torch.from_numpy(X).cuda()
    pod, ood = torch.from_numpy(po).cuda(), torch.from_numpy(oo).cuda()
    tdmap.edm_batched(Xd, pod, ood, rho=0, out=buf[:total])
    torch.cuda.synchronize()
    # every persistent walk (linear sweep, 64- and 128-cell tiles) writes
    # the same bits
    other = torch.empty(total, dtype=torch.float32, device="cuda")
    chosen = tdmap.tdmap_tuned_rho(tdmap.OP_BATCHED, 0, int(po[-1]) // 4096, 3, 4096)
    assert chosen in (1, 64, 128)
    for rho in (1, 64, 128):
        if rho == chosen:
            continue
        tdmap.edm_batched(Xd, pod, ood, rho=rho, out=other)
        torch.cuda.synchronize()
        assert torch.equal(other.view(torch.int32), buf[:total].view(torch.int32)), rho
    del other
    bits = buf.view(torch.int32)
    assert not bool(torch.any(bits[:total] == SENTINEL)), "a cell was not written"
    assert bool(torch.all(bits[total:] == SENTINEL)), "wrote past the last set"
    rng = np.random.default_rng(7)
    pick = set(rng.choice(4096, size=256, replace=False).tolist())
    pick.update({int(np.argmin(sizes)), int(np.argmax(sizes))})
    for s in sorted(pick):
        pts = X[po[s]: po[s + 1]]
        ref = np.concatenate(native.edm_rows(pts, range(len(pts))))
        got = buf[oo[s]: oo[s + 1]].cpu().numpy()
        _check_rel(got, ref, f"set {s} (n={sizes[s]})")


def test_batched_tuner_keys_on_set_size():
    # two batches with the same number of sets but sizes in different ranges
    # are tuned apart: a decision made on small sets is not reused for large
    # ones
    _require_gpu()
    tdmap.tdmap_autotune_reset()
    S = 32
    batches = {}
    for name, lo, hi in (("small", 8, 16), ("large", 600, 1200)):
        data = synth.batched_sets(S, lo, hi, 3, seed=41 + lo)
        batches[name] = data
    mean = {k: int(v["point_off"][-1]) // S for k, v in batches.items()}
    assert mean["small"].bit_length() != mean["large"].bit_length()

    def run(data):
        Xd = torch.from_numpy(data["X"]).cuda()
        pod = torch.from_numpy(data["point_off"]).cuda()
        ood = torch.from_numpy(data["out_off"]).cuda()
        D = tdmap.edm_batched(Xd, pod, ood, rho=0)
        torch.cuda.synchronize()
        return D

    run(batches["small"])
    assert tdmap.tdmap_tuned_rho(tdmap.OP_BATCHED, 0, mean["small"], 3, S) in (1, 64, 128)
    assert tdmap.tdmap_tuned_rho(tdmap.OP_BATCHED, 0, mean["large"], 3, S) == 0
    D = run(batches["large"])
    assert tdmap.tdmap_tuned_rho(tdmap.OP_BATCHED, 0, mean["large"], 3, S) in (1, 64, 128)
    data = batches["large"]
    ref = oedm.edm64_batched(data["X"], data["point_off"])
    _check_rel(D.cpu().numpy(), ref, "large batch after tuning")
