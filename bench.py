"""Benchmark of the triangular-domain EDM on one MI355X.

One step = one lower-triangular EDM of 30000 FP32 points with 3 features,
written to a full 30000 x 30000 FP32 matrix (only j <= i), launched through
g(lambda) with the autotuned coarsened tile.  Inputs live in HBM before the
timed region; the output buffer is allocated once.

Printed (one JSON line on stdout): pairs/s of that step, the roofline of the
EDM kernel (algorithmic bytes = 4 B per cell written), the same step with
the bounding-box grid (I = t_BB / t_LTM), the paper-style launches of all
five strategies at rho = 8, 16, 32 with their launch statistics, the other
workloads' rows (each timed figure with its p10 / p90 spread, autotuning
costs apart), a reduced form of the paper's N x d grid, and the CPU oracle
leg: the oracle timed on a bounded sample, and the Gram form's error against
the FP64 oracle on a sample of the 100000-point workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--skip-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "EDM pairs/sec + % HBM roofline, g(λ) vs BB on 1 MI355X; fwd+bwd pairs/sec"
HBM_PEAK_GBS = 8000.0
BF16_PEAK_FLOPS = 2.5e15
WORKLOAD = "edm_n30000_d3_full"
STRATS = ("ltm", "bb", "utm", "rb", "rec")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """Hash of the code the EDM kernel is built from (line comments and
    whitespace removed, so editing a comment keeps it); a stored HBM traffic
    figure is only reported while it matches."""
    import re
    h = hashlib.sha256()
    for f in ("device.h", "tiled.hip"):
        with open(os.path.join(ROOT, "paper_1308_1419_amd", "csrc", f)) as fh:
            code = re.sub(r"//[^\n]*", "", fh.read())
        h.update("".join(code.split()).encode())
    return h.hexdigest()[:16]


def stored_traffic():
    path = os.path.join(ROOT, "profiles", "traffic_edm_band_n30000_d3_full.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec


def time_calls(fn, reps: int, warmup: int = 2, batch: int = 1):
    """Per-call times (ms) from HIP events on torch's current stream, which
    is the stream every call launches on.  With batch > 1 each sample is the
    mean over `batch` back-to-back calls between the two events, so the
    host's time to issue a call (binding, launch) overlaps the previous
    call's kernels instead of leaving the GPU idle after the first event."""
    import torch
    for _ in range(warmup):
        fn()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    out = []
    for _ in range(reps):
        s.record()
        for _ in range(batch):
            fn()
        e.record()
        e.synchronize()
        out.append(s.elapsed_time(e) / batch)
    return out


def _med_ms(fn, reps=10, warmup=2, spread=None, key=None, batch=1):
    """Median per-call time in ms; with `spread` (a dict) and `key`, also
    stores [p10, p90] in microseconds under spread[key]."""
    t = np.asarray(time_calls(fn, reps, warmup, batch))
    if spread is not None and key is not None:
        spread[key] = [round(float(np.percentile(t, 10)) * 1e3, 2),
                       round(float(np.percentile(t, 90)) * 1e3, 2)]
    return float(np.median(t))


def _tuning_ms(fn):
    """Wall time of a call that runs the autotuner (its first call for a
    configuration), in ms, synchronised on both sides."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3


# ---------------------------------------------------------------------------
# the oracle leg (the only place bench.py runs the oracle)
# ---------------------------------------------------------------------------

def cpu_baseline(X: np.ndarray, target_s: float = 10.0):
    """The C oracle (FP64 loops, OpenMP over rows) on a seeded sample of
    rows of the same workload, sized to about target_s seconds."""
    from oracle import native
    from paper_1308_1419_amd import synth
    N = X.shape[0]
    native.load()
    probe = synth.sample_rows(N, 64, seed=1)
    t0 = time.perf_counter()
    native.edm_rows(X, probe)
    dt = time.perf_counter() - t0
    rate = sum(i + 1 for i in probe) / max(dt, 1e-9)
    want_pairs = rate * target_s
    mean_row = (N + 1) / 2
    count = int(min(N, max(64, want_pairs / mean_row)))
    rows = synth.sample_rows(N, count, seed=2)
    pairs = sum(i + 1 for i in rows)
    t0 = time.perf_counter()
    native.edm_rows(X, rows)
    dt = time.perf_counter() - t0
    what = (f"all {N} rows (the whole N={N}, d=3 triangle)" if len(set(rows)) == N
            else f"{len(rows)} seeded rows of the N={N}, d=3 triangle")
    return {"value": pairs / dt, "unit": "pairs/s", "cores": native.threads(),
            "kind": "oracle",
            "sample": f"{what}: {pairs} pairs in {dt:.2f} s, FP64 C loops, OpenMP over rows"}


def gram_error_report(torch, tdmap, synth, nrows: int = 2048):
    """Error of both Gram precisions against the FP64 C oracle on the
    100000-point, d = 64 workload, outside any timed region: 2048 seeded rows
    plus the rows of every planted near-duplicate pair, whole, and the whole
    diagonal.  Per pair: |D_gpu - D_64|; relative error over pairs with
    D_64 > 0; pairs past the stated bound of a pair that was not recomputed
    (and not within the FP32 rule either) are counted."""
    from oracle import edm as oedm
    from oracle import native
    N, d = 100000, 64
    X, pairs = synth.gaussian_with_near_duplicates(N, d, seed=synth.workload_seed(3))
    Xd = torch.from_numpy(X).cuda()
    rows = set(synth.sample_rows(N, nrows, seed=11))
    rows.update(int(max(c, s)) for c, s in pairs)
    rows = sorted(rows)
    ref_rows = native.edm_rows(X, rows)
    norms = np.linalg.norm(X.astype(np.float64), axis=1)
    rel_tol = oedm.fp32_rel_tol()
    idx = np.concatenate([np.arange(oedm.tri(i), oedm.tri(i) + i + 1) for i in rows])
    idx_d = torch.from_numpy(idx).cuda()
    diag = torch.arange(N, device="cuda", dtype=torch.int64)
    diag = diag * (diag + 1) // 2 + diag
    out = {}
    D = torch.empty(N * (N + 1) // 2, dtype=torch.float32, device="cuda")
    for prec in ("bf16_gram", "bf16x3_gram"):
        tdmap.edm(Xd, layout="packed", strategy="ltm", rho=0, precision=prec, out=D)
        got_all = D.index_select(0, idx_d).cpu().numpy().astype(np.float64)
        diag_nonzero = int(torch.count_nonzero(D.index_select(0, diag)).item())
        n = 0
        max_abs = max_rel = sq = 0.0
        past_bound = fp32_rule = 0
        off = 0
        for i, ref in zip(rows, ref_rows):
            got = got_all[off: off + i + 1]
            off += i + 1
            err = np.abs(got - ref)
            bound = oedm.gram_bound(norms[i], norms[: i + 1], ref, d,
                                    split=prec == "bf16x3_gram")
            within_rule = err <= rel_tol * ref
            past_bound += int(np.sum(~((err <= bound) | within_rule)))
            fp32_rule += int(np.sum(within_rule))
            nz = ref > 0
            rel = err[nz] / ref[nz]
            max_abs = max(max_abs, float(err.max()))
            if rel.size:
                max_rel = max(max_rel, float(rel.max()))
                sq += float(np.dot(rel, rel))
            n += err.size
        out[prec] = {"pairs_checked": n, "rows": len(rows), "max_abs_err": max_abs,
                     "max_rel_err": max_rel, "rms_rel_err": (sq / max(n, 1)) ** 0.5,
                     "pairs_within_fp32_rule": fp32_rule, "pairs_past_stated_bound": past_bound,
                     "diagonal_nonzero": diag_nonzero}
        log(f"gram {prec} error: {out[prec]}")
    del D
    out["sample"] = (f"{nrows} seeded rows + the rows of all {len(pairs)} planted pairs "
                     f"({len(rows)} rows, whole) and the whole diagonal, "
                     "against the FP64 C oracle")
    return out


# ---------------------------------------------------------------------------
# workload rows
# ---------------------------------------------------------------------------

def row_small(torch, tdmap, synth):
    """1024 points, d = 3, full 1024 x 1024 output, 16 x 16 blocks: LTM vs BB
    (cache-resident, launch-latency bound) plus g(lambda) for all
    lambda < 2^16."""
    N = 1024
    X = torch.from_numpy(synth.uniform_points(N, 3, seed=synth.workload_seed(1))).cuda()
    D = torch.empty((N, N), dtype=torch.float32, device="cuda")
    sp = {}
    t_ltm = _med_ms(lambda: tdmap.edm(X, layout="full", strategy="ltm", rho=16, out=D), 200, 10,
                    sp, "ltm_us")
    t_bb = _med_ms(lambda: tdmap.edm(X, layout="full", strategy="bb", rho=16, out=D), 200, 10,
                   sp, "bb_us")
    ij = torch.empty((1 << 16, 2), dtype=torch.int32, device="cuda")
    t_map = _med_ms(lambda: tdmap.map_blocks(0, 1 << 16, out=ij), 200, 10, sp,
                    "map_blocks_2_16_us")
    return {"ltm_us": t_ltm * 1e3, "bb_us": t_bb * 1e3, "I": t_bb / t_ltm,
            "map_blocks_2_16_us": t_map * 1e3, "p10_p90_us": sp,
            "note": "launch-latency bound (output is cache resident)"}


def row_stress(torch, tdmap, synth):
    """Stress workload: 20000 points, d = 3, packed D, L = sum (D - delta)^2,
    hand-written backward.  fwd+bwd pairs/s counts the two library kernels;
    the torch loss ops are reported beside them.  Library calls are timed in
    batches of five back-to-back calls (per-call mean), as a training loop
    issues them."""
    N = 20000
    X, Xp = synth.stress_inputs(N, 3, seed=synth.workload_seed(4))
    Xd = torch.from_numpy(X).cuda()
    delta = tdmap.edm(torch.from_numpy(Xp).cuda(), layout="packed", rho=0)
    D = torch.empty(N * (N + 1) // 2, dtype=torch.float32, device="cuda")
    dX = torch.empty((N, 3), dtype=torch.float32, device="cuda")
    ws = torch.empty(tdmap.tdmap_workspace_size(tdmap.OP_BACKWARD, N, 3, 0, 0, 1),
                     dtype=torch.uint8, device="cuda")
    tdmap.edm(Xd, layout="packed", rho=0, out=D)
    dD = 2.0 * (D - delta)
    tune = {"bwd_det_ms": _tuning_ms(lambda: tdmap.edm_backward(
                Xd, dD, rho=0, deterministic=True, out=dX, workspace=ws)),
            "bwd_atomic_ms": _tuning_ms(lambda: tdmap.edm_backward(
                Xd, dD, rho=0, deterministic=False, out=dX))}
    pairs = N * (N + 1) // 2
    sp = {}
    t_f = _med_ms(lambda: tdmap.edm(Xd, layout="packed", rho=0, out=D), 20, 2, sp, "fwd_us",
                 batch=5)
    t_b = _med_ms(lambda: tdmap.edm_backward(Xd, dD, rho=0, deterministic=True, out=dX,
                                             workspace=ws), 20, 2, sp, "bwd_det_us", batch=5)
    t_ba = _med_ms(lambda: tdmap.edm_backward(Xd, dD, rho=0, deterministic=False, out=dX),
                   20, 2, sp, "bwd_atomic_us", batch=5)

    def full_step():
        tdmap.edm(Xd, layout="packed", rho=0, out=D)
        r = D - delta
        _ = (r * r).sum()
        tdmap.edm_backward(Xd, 2.0 * r, rho=0, deterministic=True, out=dX, workspace=ws)
    t_step = _med_ms(full_step, 20, 2, sp, "step_with_torch_loss_us")
    # fused: loss and gradient in one pass over delta (D never stored)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    ws_s = torch.empty(tdmap.tdmap_workspace_size(tdmap.OP_STRESS, N, 3, 0, 0, 1),
                       dtype=torch.uint8, device="cuda")
    tune["fused_det_ms"] = _tuning_ms(lambda: tdmap.stress_backward(
        Xd, delta, rho=0, out=dX, loss=loss, workspace=ws_s))
    tune["fused_atomic_ms"] = _tuning_ms(lambda: tdmap.stress_backward(
        Xd, delta, rho=0, deterministic=False, out=dX, loss=loss))
    t_sd = _med_ms(lambda: tdmap.stress_backward(Xd, delta, rho=0, out=dX, loss=loss,
                                                 workspace=ws_s), 20, 2, sp, "fused_stress_det_us",
                   batch=5)
    t_sa = _med_ms(lambda: tdmap.stress_backward(Xd, delta, rho=0, deterministic=False,
                                                 out=dX, loss=loss), 20, 2, sp,
                   "fused_stress_atomic_us", batch=5)
    bwd_bytes = 4 * pairs
    return {"N": N, "pairs": pairs, "fwd_us": t_f * 1e3, "bwd_det_us": t_b * 1e3,
            "bwd_atomic_us": t_ba * 1e3, "fwd_bwd_pairs_per_s": pairs / ((t_f + t_b) * 1e-3),
            "step_with_torch_loss_us": t_step * 1e3,
            "fused_stress_det_us": t_sd * 1e3, "fused_stress_atomic_us": t_sa * 1e3,
            "fused_stress_hbm_frac": 4 * pairs / (t_sd * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "fused_rho": tdmap.tdmap_tuned_rho(tdmap.OP_STRESS, 0, 0, 3, N),
            "fwd_hbm_frac": 4 * pairs / (t_f * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "bwd_hbm_frac": bwd_bytes / (t_b * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "fwd_rho": tdmap.tdmap_tuned_rho(tdmap.OP_EDM, tdmap.LTM, tdmap.PACKED, 3, N),
            "bwd_rho": tdmap.tdmap_tuned_rho(tdmap.OP_BACKWARD, 0, 0, 3, N),
            "autotune_ms": tune, "p10_p90_us": sp}


def row_strict(torch, tdmap, synth):
    """30000 points, d = 3, the problem without the diagonal (Eq. (10)):
    strictly lower packed output, linear sweep (positions mapped by the
    no-diagonal g) and 256-cell tiles, beside the packed layout with the
    diagonal."""
    N = 30000
    X = torch.from_numpy(synth.uniform_points(N, 3, seed=synth.workload_seed(2))).cuda()
    S = torch.empty(N * (N - 1) // 2, dtype=torch.float32, device="cuda")
    out = {"N": N, "pairs": S.numel()}
    sp = {}
    for rho in (1, 64, 128, 256):
        t = _med_ms(lambda rho=rho: tdmap.edm(X, layout="strict", rho=rho, out=S), 20, 2, sp,
                    f"strict_rho{rho}_us")
        out[f"strict_rho{rho}_us"] = t * 1e3
        out[f"strict_rho{rho}_hbm_frac"] = 4 * S.numel() / (t * 1e-3) / 1e9 / HBM_PEAK_GBS
    del S
    P = torch.empty(N * (N + 1) // 2, dtype=torch.float32, device="cuda")
    for rho in (1, 256):
        t = _med_ms(lambda rho=rho: tdmap.edm(X, layout="packed", rho=rho, out=P), 20, 2, sp,
                    f"packed_rho{rho}_us")
        out[f"packed_rho{rho}_us"] = t * 1e3
        out[f"packed_rho{rho}_hbm_frac"] = 4 * P.numel() / (t * 1e-3) / 1e9 / HBM_PEAK_GBS
    del P
    out["p10_p90_us"] = sp
    return out


def _paper_grid(torch, tdmap, synth, Ns, ds_by_N, reps):
    """I = t_BB / t_strategy of the paper's launches (one thread per cell,
    16 x 16 blocks, full N x N output) for the dummy kernel and the EDM with
    the feature counts ds_by_N, at each N in Ns."""
    Nmax = max(Ns)
    buf = torch.empty(Nmax * Nmax, dtype=torch.float32, device="cuda")
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    pts = {d: torch.from_numpy(synth.uniform_points(Nmax, d, seed=synth.workload_seed(2) + d)).cuda()
           for d in (1, 2, 3, 4)}

    def edm_us(s, N, d):
        X = pts[d][:N]
        D = buf[: N * N].view(N, N)
        return _med_ms(lambda: tdmap.edm(X, layout="full", strategy=s, rho=16, out=D), reps, 1) * 1e3

    grid = {"N": [], "dummy_I": {s: [] for s in STRATS}, "dummy_bb_us": []}
    ds = sorted({d for v in ds_by_N for d in v})
    for d in ds:
        grid[f"edm_d{d}_I"] = {s: [] for s in STRATS}
        grid[f"edm_d{d}_bb_us"] = []
    for N, dl in zip(Ns, ds_by_N):
        grid["N"].append(N)
        t = {s: _med_ms(lambda s=s: tdmap.dummy(s, N, 16, sink=sink), reps, 1) * 1e3 for s in STRATS}
        for s in STRATS:
            grid["dummy_I"][s].append(round(t["bb"] / t[s], 4))
        grid["dummy_bb_us"].append(round(t["bb"], 2))
        for d in ds:
            if d not in dl:
                continue
            e = {s: edm_us(s, N, d) for s in STRATS}
            for s in STRATS:
                grid[f"edm_d{d}_I"][s].append(round(e["bb"] / e[s], 4))
            grid[f"edm_d{d}_bb_us"].append(round(e["bb"], 2))
        log(f"grid N={N}: dummy I(ltm) {grid['dummy_I']['ltm'][-1]}")
    del buf
    return grid


def row_paper_grid(torch, tdmap, synth):
    """The paper's full measurement grid: N = 1024 .. 30720 in steps of 1024,
    every strategy with 16 x 16 blocks, the dummy kernel and the EDM with
    d = 1 and d = 4, as I = t_BB / t_strategy; plus I as a function of
    d = 1..4 at N = 30720.  Not part of the default run (about a minute)."""
    Ns = list(range(1024, 30720 + 1, 1024))
    grid = _paper_grid(torch, tdmap, synth, Ns, [(1, 4)] * len(Ns), 5)
    by_d = _paper_grid(torch, tdmap, synth, [30720], [(1, 2, 3, 4)], 5)
    grid["I_by_d_N30720"] = {f"d{d}": {s: by_d[f"edm_d{d}_I"][s][0] for s in STRATS}
                             for d in (1, 2, 3, 4)}
    mean = lambda v: round(sum(v) / len(v), 4)
    grid["mean_I"] = {k: {s: mean(grid[k][s]) for s in STRATS}
                      for k in ("dummy_I", "edm_d1_I", "edm_d4_I")}
    return grid


def row_paper_grid_reduced(torch, tdmap, synth):
    """A reduced form of the paper's grid for the default run: N in {1024,
    8192, 15360, 30720}, every strategy at 16 x 16, the dummy kernel and the
    EDM with d = 1 and d = 4 (full output), and I against d = 1..4 at
    N = 30720."""
    Ns = [1024, 8192, 15360, 30720]
    dl = [(1, 4), (1, 4), (1, 4), (1, 2, 3, 4)]
    grid = _paper_grid(torch, tdmap, synth, Ns, dl, 5)
    grid["I_by_d_N30720"] = {f"d{d}": {s: grid[f"edm_d{d}_I"][s][-1] for s in STRATS}
                             for d in (1, 2, 3, 4)}
    for d in (2, 3):  # only at N = 30720: kept in I_by_d_N30720
        grid.pop(f"edm_d{d}_I")
        grid.pop(f"edm_d{d}_bb_us")
    return grid


def row_gram(torch, tdmap, synth):
    """100000 points, d = 64, BF16 Gram form on MFMA, packed output; beside
    it the split form (hi + lo, three MFMA products).  Both kernels (rho 128:
    eight-wave tiles; rho 256: 32-row strips) are timed; the autotuned call is
    the row's figure.  The recompute count comes from the instrumented launch
    (never timed)."""
    N, d = 100000, 64
    X, pairs_planted = synth.gaussian_with_near_duplicates(N, d, seed=synth.workload_seed(3))
    Xd = torch.from_numpy(X).cuda()
    D = torch.empty(N * (N + 1) // 2, dtype=torch.float32, device="cuda")
    ws = torch.empty(tdmap.tdmap_workspace_size(tdmap.OP_EDM, N, d, 0, 0, tdmap.BF16X3_GRAM),
                     dtype=torch.uint8, device="cuda")
    pairs = N * (N + 1) // 2
    res = {"N": N, "d": d, "pairs": pairs, "planted_pairs": len(pairs_planted)}
    sp = {}
    tune = {}
    for prec, key in (("bf16_gram", ""), ("bf16x3_gram", "split_")):
        fn = lambda rho=0: tdmap.edm(Xd, layout="packed", rho=rho, precision=prec, out=D,
                                     workspace=ws)
        tune[key + "ms"] = _tuning_ms(fn)
        t = _med_ms(fn, 10, 2, sp, key + "us")
        flops = (2.0 if not key else 6.0) * d * pairs
        res.update({key + "us": t * 1e3, key + "pairs_per_s": pairs / (t * 1e-3),
                    key + "hbm_frac": 4 * pairs / (t * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    key + "mfma_frac_bf16": flops / (t * 1e-3) / BF16_PEAK_FLOPS,
                    key + "rho": tdmap.tdmap_tuned_rho(tdmap.OP_EDM, tdmap.LTM,
                                                       256 + tdmap.PRECISIONS[prec], d, N)})
        for rho in (128, 256):
            t = _med_ms(lambda rho=rho: fn(rho), 10, 2, sp, f"{key}rho{rho}_us")
            res[f"{key}rho{rho}_us"] = t * 1e3
        _, cnt = tdmap.gram_recompute_count(Xd, prec, rho=0, out=D, workspace=ws)
        res[key + "recomputed_pairs"] = int(cnt.item())
    res["autotune_ms"] = tune
    res["p10_p90_us"] = sp
    del D
    return res


def row_batched(torch, tdmap, synth):
    """4096 sets, n uniform in [64, 4096], d = 3, one persistent launch."""
    data = synth.batched_sets(4096, 64, 4096, 3, seed=synth.workload_seed(5))
    Xd = torch.from_numpy(data["X"]).cuda()
    po = torch.from_numpy(data["point_off"]).cuda()
    oo = torch.from_numpy(data["out_off"]).cuda()
    total = int(data["out_off"][-1])
    mean_n = int(data["point_off"][-1]) // 4096
    D = torch.empty(total, dtype=torch.float32, device="cuda")
    ws = torch.empty(tdmap.tdmap_workspace_size(tdmap.OP_BATCHED, 0, 3, 4096, 0, 0),
                     dtype=torch.uint8, device="cuda")
    fn = lambda: tdmap.edm_batched(Xd, po, oo, rho=0, out=D, workspace=ws)
    tune_ms = _tuning_ms(fn)
    sp = {}
    t = _med_ms(fn, 10, 2, sp, "us")
    per_rho = {}
    for rho in (1, 64, 128):
        per_rho[f"rho{rho}_us"] = _med_ms(
            lambda rho=rho: tdmap.edm_batched(Xd, po, oo, rho=rho, out=D, workspace=ws), 5, 2,
            sp, f"rho{rho}_us") * 1e3
    del D
    return {"sets": 4096, "pairs": total, "us": t * 1e3, "pairs_per_s": total / (t * 1e-3),
            "hbm_frac": 4 * total / (t * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "rho": tdmap.tdmap_tuned_rho(tdmap.OP_BATCHED, 0, mean_n, 3, 4096),
            "autotune_ms": tune_ms, **per_rho, "p10_p90_us": sp}


def first_map_failure(torch, tdmap, variant, chunk=1 << 27):
    """Smallest lambda < 2^32 where the map under `variant` breaks the
    row-major succession (0,0), (1,0), (1,1), (2,0), ... or None.  Uses no
    oracle: the succession from lambda = 0 defines the numbering."""
    out = torch.empty((chunk, 2), dtype=torch.int32, device="cuda")
    prev = None
    for lam0 in range(0, 1 << 32, chunk):
        tdmap.map_blocks_variant(lam0, chunk, variant, out=out)
        i = out[:, 0].to(torch.int64) & 0xFFFFFFFF
        j = out[:, 1].to(torch.int64) & 0xFFFFFFFF
        if prev is None:
            if int(i[0]) != 0 or int(j[0]) != 0:
                return 0
        else:
            pi, pj = prev
            ok0 = (int(i[0]) == pi and int(j[0]) == pj + 1 <= pi) or \
                  (int(i[0]) == pi + 1 and int(j[0]) == 0 and pj == pi)
            if not ok0:
                return lam0
        # the next cell of the row (still on or below the diagonal), or the
        # first cell of the next row
        ok = ((i[1:] == i[:-1]) & (j[1:] == j[:-1] + 1) & (j[1:] <= i[1:])) | \
             ((i[1:] == i[:-1] + 1) & (j[1:] == 0) & (j[:-1] == i[:-1]))
        bad = torch.nonzero(~ok)
        if bad.numel():
            return lam0 + int(bad[0, 0]) + 1
        prev = (int(i[-1]), int(j[-1]))
    return None


def row_mapcost(torch, tdmap, synth):
    """The paper's dummy kernel (map + filter, no EDM) for every strategy at
    N = 30000 and rho = 8, 16, 32, the LTM row variants at rho = 16, and where
    the uncorrected variants first name a wrong cell."""
    N = 30000
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    res = {}
    sp = {}
    for rho in (8, 16, 32):
        row = {}
        for s in STRATS:
            row[s] = _med_ms(lambda s=s: tdmap.dummy(s, N, rho, sink=sink), 10, 2, sp,
                             f"rho{rho}_{s}_us") * 1e3
        res[f"rho{rho}"] = {s: {"us": t, "I_vs_bb": row["bb"] / t} for s, t in row.items()}
    var = {}
    t_bb = res["rho16"]["bb"]["us"]
    for v, name in ((0, "ltm_fixup"), (1, "ltm_x_sqrtf"), (2, "ltm_r_rsq_eps")):
        t = _med_ms(lambda v=v: tdmap.dummy("ltm", N, 16, variant=v, sink=sink), 10, 2, sp,
                    f"{name}_us") * 1e3
        I = t_bb / t
        var[name] = {"us": t, "I_vs_bb": I, "k": 2.0 / I,
                     "first_wrong_lambda": first_map_failure(torch, tdmap, v) if v else None}
    res["ltm_variants_rho16"] = var
    res["p10_p90_us"] = sp
    return res


def row_paper_style(torch, tdmap, synth):
    """The paper's one-cell-per-thread launches of all five strategies on the
    30000-point, d = 3 full-layout EDM at rho = 8, 16, 32 (the launches the
    main step's comparison times), for profiler runs of these kernels."""
    N, d = 30000, 3
    X = synth.uniform_points(N, d, seed=synth.workload_seed(2))
    Xd = torch.from_numpy(X).cuda()
    D = torch.empty((N, N), dtype=torch.float32, device="cuda")
    bytes_alg = 4 * N * (N + 1) // 2
    out = {}
    for rho in (8, 16, 32):
        row = {}
        for s in STRATS:
            t = _med_ms(lambda s=s: tdmap.edm(Xd, layout="full", strategy=s, rho=rho, out=D),
                        10, 2)
            row[s] = {"us": t * 1e3, "hbm_frac": bytes_alg / (t * 1e-3) / 1e9 / HBM_PEAK_GBS}
        for s in row:
            row[s]["I_vs_bb"] = row["bb"]["us"] / row[s]["us"]
        out[f"rho{rho}"] = row
    return out


ROWS = {"edm_n1024_d3_full": row_small, "stress_n20000_d3": row_stress,
        "mapcost_n30000": row_mapcost, "strict_n30000_d3": row_strict,
        "paper_grid_rho16": row_paper_grid,
        "paper_grid_rho16_reduced": row_paper_grid_reduced,
        "gram_n100000_d64_packed": row_gram,
        "batched_s4096_n64_4096_d3": row_batched,
        "paper_style_n30000_d3": row_paper_style}
DEFAULT_ROWS = ("edm_n1024_d3_full", "mapcost_n30000", "strict_n30000_d3", "stress_n20000_d3",
                "gram_n100000_d64_packed", "batched_s4096_n64_4096_d3",
                "paper_grid_rho16_reduced")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--only-main", action="store_true",
                    help="time only the main step (for profiler runs)")
    ap.add_argument("--row", default=None,
                    help="run only one named workload row (for profiler runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy three times (scales the "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.zeros(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied 3 x 2^30 bytes")
        return
    if args.row:
        import torch
        from paper_1308_1419_amd import synth, tdmap
        print(json.dumps({args.row: ROWS[args.row](torch, tdmap, synth)}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported "
              "(the EDM path runs on a single device)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1308_1419_amd import synth, tdmap
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    N, d = 30000, 3
    X = synth.uniform_points(N, d, seed=synth.workload_seed(2))
    Xd = torch.from_numpy(X).cuda()
    D = torch.empty((N, N), dtype=torch.float32, device="cuda")
    pairs = N * (N + 1) // 2
    bytes_alg = 4 * pairs

    # tile choice (untimed): the autotuner runs once per configuration
    tune_ms = {"ltm": _tuning_ms(lambda: tdmap.edm(Xd, layout="full", strategy="ltm", rho=0,
                                                   out=D)),
               "bb": _tuning_ms(lambda: tdmap.edm(Xd, layout="full", strategy="bb", rho=0,
                                                  out=D))}
    ts_ltm = tdmap.tdmap_tuned_rho(tdmap.OP_EDM, tdmap.LTM, tdmap.FULL, d, N)
    ts_bb = tdmap.tdmap_tuned_rho(tdmap.OP_EDM, tdmap.BB, tdmap.FULL, d, N)
    log(f"tuned tiles: ltm {ts_ltm}, bb {ts_bb}")

    def step():
        tdmap.edm(Xd, layout="full", strategy="ltm", rho=ts_ltm, out=D)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = ev0.elapsed_time(ev1) / args.steps
    value = pairs * args.steps / wall
    log(f"ltm tile {ts_ltm}: {kern_ms * 1e3:.1f} us/step (events), "
        f"{wall / args.steps * 1e6:.1f} us/step (wall)")

    achieved = bytes_alg / (kern_ms * 1e-3) / 1e9
    # the same number of bytes as one plain linear stream of 16-byte
    # non-temporal stores: the store rate this device reaches at best
    del D
    torch.cuda.empty_cache()
    S = torch.empty(pairs, dtype=torch.float32, device="cuda")
    t_stream = float(np.median(time_calls(lambda: tdmap.stream_fill(S, 1.0), 20, 3)))
    del S
    torch.cuda.empty_cache()
    D = torch.empty((N, N), dtype=torch.float32, device="cuda")
    stream_gbs = bytes_alg / (t_stream * 1e-3) / 1e9
    traffic = stored_traffic()
    # the kernel's template arguments: feature count, layout (0 = full), BB
    # grid, dense 16-byte aligned points
    kname = (f"edm_band_kernel<{d}, 0, false, true>" if ts_ltm == 256
             else f"edm_tile_kernel<{ts_ltm}, {d}, 0, true, false>")
    if traffic and not traffic["kernel"].startswith(kname):
        traffic = None  # the counters were taken on another tile kernel
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic["bytes_per_launch"] if traffic else None,
                "kernel": kname + " (LTM, full layout)",
                "algorithmic_bytes_per_launch": bytes_alg,
                "stream_peak": round(stream_gbs, 1),
                "frac_of_stream": round(achieved / stream_gbs, 4)}

    result = {
        "metric": METRIC, "value": value, "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD, "N": N, "d": d, "layout": "full",
                   "strategy": "ltm", "rho": ts_ltm, "pairs": pairs},
        "roofline": roofline,
    }

    if not args.only_main:
        comp = {"autotune_ms": tune_ms}
        sp = {}
        # the same tile body on the bounding-box grid
        t_ltm = _med_ms(step, 20, 2, sp, "ltm_us")
        t_bb = _med_ms(lambda: tdmap.edm(Xd, layout="full", strategy="bb", rho=ts_bb, out=D),
                       20, 2, sp, "bb_us")
        comp["tiled"] = {"ltm_us": t_ltm * 1e3, "bb_us": t_bb * 1e3, "ltm_rho": ts_ltm,
                         "bb_rho": ts_bb, "I": t_bb / t_ltm,
                         "ltm_hbm_frac": bytes_alg / (t_ltm * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "p10_p90_us": sp}
        # the paper's launches: rho x rho threads, one cell each
        paper = {}
        for rho in (8, 16, 32):
            row = {}
            sp = {}
            for s in STRATS:
                t = _med_ms(lambda s=s: tdmap.edm(Xd, layout="full", strategy=s, rho=rho, out=D),
                            10, 2, sp, s)
                blocks, idle, idle_lanes = tdmap.waste_counts(s, N, rho)
                row[s] = {"us": t * 1e3, "blocks": blocks, "idle_blocks": idle,
                          "idle_threads": idle_lanes,
                          "hbm_frac": bytes_alg / (t * 1e-3) / 1e9 / HBM_PEAK_GBS,
                          "p10_p90_us": sp[s]}
            for s in row:
                row[s]["I_vs_bb"] = row["bb"]["us"] / row[s]["us"]
            paper[f"rho{rho}"] = row
            log(f"rho {rho}: " + ", ".join(f"{s} {row[s]['us']:.0f}us" for s in row))
        comp["paper_style"] = paper
        result["comparison"] = comp
        del D
        torch.cuda.empty_cache()
        rows = {}
        for name in DEFAULT_ROWS:
            log(f"row {name} ...")
            rows[name] = ROWS[name](torch, tdmap, synth)
            torch.cuda.empty_cache()
            log(f"row {name}: {rows[name]}")
        result["rows"] = rows
        result["fwd_bwd_pairs_per_s"] = rows["stress_n20000_d3"]["fwd_bwd_pairs_per_s"]

    if not args.skip_cpu:
        log("timing the CPU oracle on a sample ...")
        result["cpu_baseline"] = cpu_baseline(X)
        if "rows" in result:
            log("Gram error against the FP64 oracle on a sample ...")
            result["rows"]["gram_n100000_d64_packed"]["error_vs_fp64_oracle"] = \
                gram_error_report(torch, tdmap, synth)
            torch.cuda.empty_cache()

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
