"""Python binding of the tdmap C ABI (include/tdmap.h).

Two layers, both argument marshalling only -- every step of the work runs
in the HIP library:

* ``tdmap_*`` functions with the C names and signatures (integers for
  pointers and streams); a non-zero status raises ``TdmapError``.
* torch conveniences (``edm``, ``edm_backward``, ``edm_batched``,
  ``map_blocks``, ``EDM``) that take device tensors, allocate outputs with
  torch and pass torch's current stream.

The library is loaded on first use from ``libtdmap.so`` next to this file.
If it is missing, every call raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtdmap.so")

# enums (include/tdmap.h)
OK, ERR_INVALID, ERR_UNSUPPORTED, ERR_WORKSPACE, ERR_HIP = range(5)
LTM, BB, UTM, RB, REC = range(5)
FULL, PACKED, PACKED_STRICT = 0, 1, 2
FP32, BF16_GRAM, BF16X3_GRAM = 0, 1, 2
OP_EDM, OP_BACKWARD, OP_BATCHED, OP_STRESS = 0, 1, 2, 3

STRATEGIES = {"ltm": LTM, "bb": BB, "utm": UTM, "rb": RB, "rec": REC}
LAYOUTS = {"full": FULL, "packed": PACKED, "strict": PACKED_STRICT}
PRECISIONS = {"fp32": FP32, "bf16_gram": BF16_GRAM, "bf16x3_gram": BF16X3_GRAM}


class TdmapError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = _load()
        msg = lib.tdmap_status_string(status).decode()
        if status == ERR_HIP:
            msg += ": " + lib.tdmap_last_error().decode()
        super().__init__(f"{where}: {msg} (status {status})")
        self.status = status


_lib: Optional[ctypes.CDLL] = None


def _load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"tdmap HIP library not built: {LIB_PATH} is missing "
            "(run python -m paper_1308_1419_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64, u64, vp, sz = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                             ctypes.c_void_p, ctypes.c_size_t)
    sig = {
        "tdmap_map_blocks": ([u64, u64, vp, vp], ctypes.c_int),
        "tdmap_map_blocks_nodiag": ([u64, u64, vp, vp], ctypes.c_int),
        "tdmap_stream_fill": ([vp, u64, ctypes.c_float, vp], ctypes.c_int),
        "tdmap_edm": ([vp, i64, i32, i64, vp, i64, i32, i32, i32, i32, vp, sz, vp],
                      ctypes.c_int),
        "tdmap_edm_backward": ([vp, i64, i32, i64, vp, i64, i32, vp, i32, i32, vp, sz, vp],
                               ctypes.c_int),
        "tdmap_stress_backward": ([vp, i64, i32, i64, vp, i64, i32, vp, vp, i32, i32, vp, sz,
                                   vp], ctypes.c_int),
        "tdmap_edm_batched": ([vp, i32, i32, vp, vp, vp, i32, vp, sz, vp], ctypes.c_int),
        "tdmap_gram_recompute_count": ([vp, i64, i32, i64, vp, i32, i32, vp, sz, vp, vp],
                                       ctypes.c_int),
        "tdmap_edm_gram_noalloc": ([vp, i64, i32, i64, vp, i32, i32, vp], ctypes.c_int),
        "tdmap_edm_shard": ([vp, i64, i32, i64, vp, i64, i32, i32, i32, i32, vp, sz, i32, i32, vp],
                            ctypes.c_int),
        "tdmap_workspace_size": ([i32, i64, i32, i32, i32, i32], sz),
        "tdmap_waste_counts": ([i32, i64, i32, vp], ctypes.c_int),
        "tdmap_count_waste": ([i32, i64, i32, vp, vp], ctypes.c_int),
        "tdmap_map_blocks_variant": ([u64, u64, i32, vp, vp], ctypes.c_int),
        "tdmap_dummy": ([i32, i32, i64, i32, ctypes.c_uint32, vp, vp], ctypes.c_int),
        "tdmap_tuned_rho": ([i32, i32, i32, i32, i64], i32),
        "tdmap_autotune_reset": ([], None),
        "tdmap_status_string": ([i32], ctypes.c_char_p),
        "tdmap_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


EXPORTED = (
    "tdmap_map_blocks", "tdmap_map_blocks_nodiag", "tdmap_edm", "tdmap_edm_backward",
    "tdmap_stress_backward", "tdmap_edm_batched", "tdmap_gram_recompute_count",
    "tdmap_edm_gram_noalloc", "tdmap_edm_shard",
    "tdmap_workspace_size", "tdmap_waste_counts", "tdmap_count_waste",
    "tdmap_map_blocks_variant", "tdmap_dummy", "tdmap_stream_fill",
    "tdmap_tuned_rho", "tdmap_autotune_reset", "tdmap_status_string",
    "tdmap_last_error",
)


def _check(status: int, where: str) -> None:
    if status != OK:
        raise TdmapError(status, where)


# ---------------------------------------------------------------------------
# C-named entry points
# ---------------------------------------------------------------------------

def tdmap_map_blocks(lambda0: int, count: int, ij: int, stream: int) -> None:
    _check(_load().tdmap_map_blocks(lambda0, count, ij, stream), "tdmap_map_blocks")


def tdmap_map_blocks_nodiag(lambda0: int, count: int, ij: int, stream: int) -> None:
    _check(_load().tdmap_map_blocks_nodiag(lambda0, count, ij, stream),
           "tdmap_map_blocks_nodiag")


def tdmap_stream_fill(buf: int, n: int, value: float, stream: int) -> None:
    _check(_load().tdmap_stream_fill(buf, n, value, stream), "tdmap_stream_fill")


def stream_fill(buf, value: float = 0.0):
    """Write-stream reference: buf (a 16-byte aligned float32 CUDA tensor) := value."""
    tdmap_stream_fill(buf.data_ptr() if buf.numel() else 0, buf.numel(), value, _stream())
    return buf


def tdmap_edm(X: int, N: int, d: int, ldx: int, D: int, ldd: int, layout: int,
              strategy: int, rho: int, precision: int, workspace: int,
              ws_bytes: int, stream: int) -> None:
    _check(_load().tdmap_edm(X, N, d, ldx, D, ldd, layout, strategy, rho, precision,
                             workspace, ws_bytes, stream), "tdmap_edm")


def tdmap_edm_backward(X: int, N: int, d: int, ldx: int, dD: int, ldd: int,
                       layout: int, dX: int, rho: int, deterministic: int,
                       workspace: int, ws_bytes: int, stream: int) -> None:
    _check(_load().tdmap_edm_backward(X, N, d, ldx, dD, ldd, layout, dX, rho,
                                      deterministic, workspace, ws_bytes, stream),
           "tdmap_edm_backward")


def tdmap_stress_backward(X: int, N: int, d: int, ldx: int, delta: int, ldd: int,
                          layout: int, dX: int, loss: int, rho: int, deterministic: int,
                          workspace: int, ws_bytes: int, stream: int) -> None:
    _check(_load().tdmap_stress_backward(X, N, d, ldx, delta, ldd, layout, dX, loss, rho,
                                         deterministic, workspace, ws_bytes, stream),
           "tdmap_stress_backward")


def tdmap_edm_batched(X_cat: int, d: int, num_sets: int, point_off: int, out_off: int,
                      D_cat: int, rho: int, workspace: int, ws_bytes: int,
                      stream: int) -> None:
    _check(_load().tdmap_edm_batched(X_cat, d, num_sets, point_off, out_off, D_cat, rho,
                                     workspace, ws_bytes, stream), "tdmap_edm_batched")


def tdmap_gram_recompute_count(X: int, N: int, d: int, ldx: int, D: int, precision: int,
                               rho: int, workspace: int, ws_bytes: int, count: int,
                               stream: int) -> None:
    _check(_load().tdmap_gram_recompute_count(X, N, d, ldx, D, precision, rho, workspace,
                                              ws_bytes, count, stream),
           "tdmap_gram_recompute_count")


def tdmap_workspace_size(op: int, N: int, d: int, num_sets: int, rho: int, flags: int) -> int:
    return int(_load().tdmap_workspace_size(op, N, d, num_sets, rho, flags))


def tdmap_waste_counts(strategy: int, N: int, rho: int) -> tuple:
    out = (ctypes.c_int64 * 3)()
    _check(_load().tdmap_waste_counts(strategy, N, rho, ctypes.addressof(out)),
           "tdmap_waste_counts")
    return tuple(int(v) for v in out)


def tdmap_count_waste(strategy: int, N: int, rho: int, counts: int, stream: int) -> None:
    _check(_load().tdmap_count_waste(strategy, N, rho, counts, stream), "tdmap_count_waste")


def tdmap_map_blocks_variant(lambda0: int, count: int, variant: int, ij: int, stream: int) -> None:
    _check(_load().tdmap_map_blocks_variant(lambda0, count, variant, ij, stream),
           "tdmap_map_blocks_variant")


def tdmap_dummy(strategy: int, variant: int, N: int, rho: int, never: int, sink: int,
                stream: int) -> None:
    _check(_load().tdmap_dummy(strategy, variant, N, rho, never, sink, stream), "tdmap_dummy")


def tdmap_tuned_rho(op: int, strategy: int, layout: int, d: int, size: int) -> int:
    return int(_load().tdmap_tuned_rho(op, strategy, layout, d, size))


def tdmap_autotune_reset() -> None:
    _load().tdmap_autotune_reset()


def tdmap_status_string(status: int) -> str:
    return _load().tdmap_status_string(status).decode()


def tdmap_last_error() -> str:
    return _load().tdmap_last_error().decode()


# ---------------------------------------------------------------------------
# torch conveniences
# ---------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _stream() -> int:
    return _torch().cuda.current_stream().cuda_stream


def _points(X):
    torch = _torch()
    if not (isinstance(X, torch.Tensor) and X.is_cuda and X.dtype == torch.float32
            and X.dim() == 2):
        raise TypeError("X must be a 2D float32 CUDA tensor")
    if X.stride(1) != 1:
        raise ValueError("X must have unit stride along features")
    return X


def _device_tensor(t, name: str, dtype, device, min_numel: int = 0,
                   numel: Optional[int] = None):
    """Host-side checks of a tensor argument that needs no synchronisation:
    type, dtype, device, contiguity and size.  A wrong dtype or a short
    buffer would otherwise make a kernel read or write out of bounds."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda or t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must hold {numel} elements, got {t.numel()}")
    if t.numel() < min_numel:
        raise ValueError(f"{name} must hold at least {min_numel} elements, got {t.numel()}")
    return t


def _triangle_cells(N: int, layout: int) -> int:
    """Elements a packed or strict output of N points holds."""
    return strict_size(N) if layout == PACKED_STRICT else packed_size(N)


def _check_full_buffer(t, name: str, N: int, ldd: int, device):
    """A full-layout buffer: float32 on the device with room for N rows of
    pitch ldd (the last row needs N cells)."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32:
        raise TypeError(f"{name} must be a float32 tensor")
    if not t.is_cuda or t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if ldd < N:
        raise ValueError(f"{name}: row pitch {ldd} is below N = {N}")
    need = (N - 1) * ldd + N if N > 0 else 0
    if t.dim() == 2:
        if t.stride(1) != 1 or t.stride(0) != ldd or t.shape[0] < N or t.shape[1] < N:
            raise ValueError(f"{name}: expected at least {N} x {N} with row pitch {ldd}")
    elif not (t.is_contiguous() and t.numel() >= need):
        raise ValueError(f"{name} must be contiguous with at least {need} elements")


def packed_size(N: int) -> int:
    return N * (N + 1) // 2


def strict_size(N: int) -> int:
    return N * (N - 1) // 2 if N > 0 else 0


def map_blocks(lambda0: int, count: int, out=None):
    """g(lambda) for lambda0 .. lambda0+count-1 as a (count, 2) int32 tensor
    holding the uint32 (i, j) bits."""
    torch = _torch()
    if out is None:
        out = torch.empty((count, 2), dtype=torch.int32, device="cuda")
    tdmap_map_blocks(lambda0, count, out.data_ptr() if count else 0, _stream())
    return out


def map_blocks_nodiag(lambda0: int, count: int, out=None):
    """The map without the diagonal for lambda0 .. lambda0+count-1."""
    torch = _torch()
    if out is None:
        out = torch.empty((count, 2), dtype=torch.int32, device="cuda")
    tdmap_map_blocks_nodiag(lambda0, count, out.data_ptr() if count else 0, _stream())
    return out


def map_blocks_variant(lambda0: int, count: int, variant: int, out=None):
    """g(lambda) under a row variant (0 exact, 1 LTM-X, 2 LTM-R + eps)."""
    torch = _torch()
    if out is None:
        out = torch.empty((count, 2), dtype=torch.int32, device="cuda")
    tdmap_map_blocks_variant(lambda0, count, variant, out.data_ptr() if count else 0, _stream())
    return out


def dummy(strategy: str, N: int, rho: int, variant: int = 0, sink=None):
    """The mapping-cost (dummy) kernel of a strategy; returns the sink."""
    torch = _torch()
    if sink is None:
        sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    tdmap_dummy(STRATEGIES[strategy], variant, N, rho, 0xFFFFFFFF, sink.data_ptr(), _stream())
    return sink


def tdmap_edm_shard(X: int, N: int, d: int, ldx: int, D: int, ldd: int, layout: int,
                    strategy: int, rho: int, precision: int, workspace: int, ws_bytes: int,
                    shard: int, num_shards: int, stream: int) -> None:
    _check(_load().tdmap_edm_shard(X, N, d, ldx, D, ldd, layout, strategy, rho, precision,
                                   workspace, ws_bytes, shard, num_shards, stream),
           "tdmap_edm_shard")


def tdmap_edm_gram_noalloc(X: int, N: int, d: int, ldx: int, D: int, precision: int,
                           rho: int, stream: int) -> None:
    _check(_load().tdmap_edm_gram_noalloc(X, N, d, ldx, D, precision, rho, stream),
           "tdmap_edm_gram_noalloc")


def edm(X, layout: str = "full", strategy: str = "ltm", rho: int = 0,
        precision: str = "fp32", out=None, ldd: Optional[int] = None, workspace=None):
    """Lower-triangular EDM of the rows of X (see tdmap_edm)."""
    torch = _torch()
    X = _points(X)
    N, d = X.shape
    lay = LAYOUTS[layout]
    prec = PRECISIONS[precision]
    if out is None:
        if lay == FULL:
            out = torch.empty((N, N), dtype=torch.float32, device=X.device)
        elif lay == PACKED_STRICT:
            out = torch.empty(strict_size(N), dtype=torch.float32, device=X.device)
        else:
            out = torch.empty(packed_size(N), dtype=torch.float32, device=X.device)
    if ldd is None:
        ldd = out.stride(0) if lay == FULL else 0
    if lay == FULL:
        _check_full_buffer(out, "out", N, ldd, X.device)
    else:
        _device_tensor(out, "out", torch.float32, X.device,
                       min_numel=_triangle_cells(N, lay))
    ws_bytes = tdmap_workspace_size(OP_EDM, N, d, 0, rho, prec)
    if ws_bytes and workspace is None:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=X.device)
    ws_ptr = workspace.data_ptr() if workspace is not None else 0
    ws_len = workspace.numel() * workspace.element_size() if workspace is not None else 0
    tdmap_edm(X.data_ptr(), N, d, X.stride(0), out.data_ptr(), ldd, lay,
              STRATEGIES[strategy], rho, prec, ws_ptr, ws_len, _stream())
    return out


def edm_shard(X, shard: int, num_shards: int, layout: str = "full", rho: int = 256,
              precision: str = "fp32", out=None, ldd: Optional[int] = None, workspace=None):
    """Shard `shard` of `num_shards` of the LTM EDM of X (see tdmap_edm_shard):
    only that shard's cells of `out` are written (a new output is allocated
    uninitialised if none is given)."""
    torch = _torch()
    X = _points(X)
    N, d = X.shape
    lay = LAYOUTS[layout]
    prec = PRECISIONS[precision]
    if out is None:
        if lay == FULL:
            out = torch.empty((N, N), dtype=torch.float32, device=X.device)
        elif lay == PACKED_STRICT:
            out = torch.empty(strict_size(N), dtype=torch.float32, device=X.device)
        else:
            out = torch.empty(packed_size(N), dtype=torch.float32, device=X.device)
    if ldd is None:
        ldd = out.stride(0) if lay == FULL else 0
    if lay == FULL:
        _check_full_buffer(out, "out", N, ldd, X.device)
    else:
        _device_tensor(out, "out", torch.float32, X.device,
                       min_numel=_triangle_cells(N, lay))
    ws_bytes = tdmap_workspace_size(OP_EDM, N, d, 0, rho, prec)
    if ws_bytes and workspace is None:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=X.device)
    ws_ptr = workspace.data_ptr() if workspace is not None else 0
    ws_len = workspace.numel() * workspace.element_size() if workspace is not None else 0
    tdmap_edm_shard(X.data_ptr(), N, d, X.stride(0), out.data_ptr(), ldd, lay, LTM, rho, prec,
                    ws_ptr, ws_len, shard, num_shards, _stream())
    return out


def gram_recompute_count(X, precision: str = "bf16_gram", rho: int = 0, out=None,
                         workspace=None):
    """(D, count): the packed Gram-form EDM of X and the number of pairs
    j <= i that took the FP32 recompute (see tdmap_gram_recompute_count);
    ``count`` is a one-element int64 CUDA tensor holding the uint64 bits."""
    torch = _torch()
    X = _points(X)
    N, d = X.shape
    prec = PRECISIONS[precision]
    if out is None:
        out = torch.empty(packed_size(N), dtype=torch.float32, device=X.device)
    _device_tensor(out, "out", torch.float32, X.device, min_numel=packed_size(N))
    ws_bytes = tdmap_workspace_size(OP_EDM, N, d, 0, rho, prec)
    if ws_bytes and workspace is None:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=X.device)
    ws_ptr = workspace.data_ptr() if workspace is not None else 0
    ws_len = workspace.numel() * workspace.element_size() if workspace is not None else 0
    count = torch.empty(1, dtype=torch.int64, device=X.device)
    tdmap_gram_recompute_count(X.data_ptr(), N, d, X.stride(0), out.data_ptr(), prec, rho,
                               ws_ptr, ws_len, count.data_ptr(), _stream())
    return out, count


def edm_backward(X, dD, layout: str = "packed", rho: int = 0, deterministic: bool = True,
                 ldd: Optional[int] = None, out=None, workspace=None):
    """dL/dX from dL/dD over the triangle (see tdmap_edm_backward)."""
    torch = _torch()
    X = _points(X)
    N, d = X.shape
    lay = LAYOUTS[layout]
    if out is None:
        out = torch.empty((N, d), dtype=torch.float32, device=X.device)
    _device_tensor(out, "out", torch.float32, X.device, numel=N * d)
    if ldd is None:
        ldd = dD.stride(0) if lay == FULL else 0
    if lay == FULL:
        _check_full_buffer(dD, "dD", N, ldd, X.device)
    else:
        _device_tensor(dD, "dD", torch.float32, X.device, min_numel=_triangle_cells(N, lay))
    det = 1 if deterministic else 0
    ws_bytes = tdmap_workspace_size(OP_BACKWARD, N, d, 0, rho, det)
    if ws_bytes and workspace is None:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=X.device)
    ws_ptr = workspace.data_ptr() if workspace is not None else 0
    ws_len = workspace.numel() * workspace.element_size() if workspace is not None else 0
    tdmap_edm_backward(X.data_ptr(), N, d, X.stride(0), dD.data_ptr(), ldd, lay,
                       out.data_ptr(), rho, det, ws_ptr, ws_len, _stream())
    return out


def stress_backward(X, delta, layout: str = "packed", rho: int = 0,
                    deterministic: bool = True, ldd: Optional[int] = None, out=None,
                    loss=None, workspace=None):
    """(loss, dX) of L = sum_{j<i} (D_ij - delta_ij)^2 in one pass (see
    tdmap_stress_backward); ``loss`` is a one-element CUDA tensor."""
    torch = _torch()
    X = _points(X)
    N, d = X.shape
    lay = LAYOUTS[layout]
    if out is None:
        out = torch.empty((N, d), dtype=torch.float32, device=X.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
    _device_tensor(out, "out", torch.float32, X.device, numel=N * d)
    _device_tensor(loss, "loss", torch.float32, X.device, min_numel=1)
    if ldd is None:
        ldd = delta.stride(0) if lay == FULL else 0
    if lay == FULL:
        _check_full_buffer(delta, "delta", N, ldd, X.device)
    else:
        _device_tensor(delta, "delta", torch.float32, X.device,
                       min_numel=_triangle_cells(N, lay))
    det = 1 if deterministic else 0
    ws_bytes = tdmap_workspace_size(OP_STRESS, N, d, 0, rho, det)
    if ws_bytes and workspace is None:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=X.device)
    ws_ptr = workspace.data_ptr() if workspace is not None else 0
    ws_len = workspace.numel() * workspace.element_size() if workspace is not None else 0
    delta_ptr = delta.data_ptr() if delta.numel() else 0
    tdmap_stress_backward(X.data_ptr(), N, d, X.stride(0), delta_ptr, ldd, lay,
                          out.data_ptr(), loss.data_ptr(), rho, det, ws_ptr, ws_len,
                          _stream())
    return loss, out


def edm_batched(X_cat, point_off, out_off, rho: int = 0, out=None, workspace=None):
    """Packed EDMs of many point sets in one launch (see tdmap_edm_batched).
    ``point_off`` / ``out_off`` are int64 CUDA tensors of length S+1; the
    total output size is read from ``out_off`` only when ``out`` is None."""
    torch = _torch()
    X_cat = _points(X_cat)
    d = X_cat.shape[1]
    if X_cat.stride(0) != d:
        raise ValueError("X_cat must be contiguous")
    S = point_off.numel() - 1
    if S < 0:
        raise ValueError("point_off must hold S+1 offsets")
    _device_tensor(point_off, "point_off", torch.int64, X_cat.device)
    _device_tensor(out_off, "out_off", torch.int64, X_cat.device, numel=S + 1)
    if out is None:
        total = int(out_off[-1].item())
        out = torch.empty(total, dtype=torch.float32, device=X_cat.device)
    # the size of out against out_off[S] would need a synchronising read of
    # the device offsets: only its type, device and contiguity are checked
    _device_tensor(out, "out", torch.float32, X_cat.device)
    ws_bytes = tdmap_workspace_size(OP_BATCHED, 0, d, S, rho, 0)
    if ws_bytes and workspace is None:
        workspace = torch.empty(ws_bytes, dtype=torch.uint8, device=X_cat.device)
    ws_ptr = workspace.data_ptr() if workspace is not None else 0
    ws_len = workspace.numel() * workspace.element_size() if workspace is not None else 0
    tdmap_edm_batched(X_cat.data_ptr(), d, S, point_off.data_ptr(), out_off.data_ptr(),
                      out.data_ptr(), rho, ws_ptr, ws_len, _stream())
    return out


def count_waste(strategy: str, N: int, rho: int):
    """(blocks, fully idle blocks, idle threads) counted on the device."""
    torch = _torch()
    counts = torch.empty(3, dtype=torch.int64, device="cuda")
    tdmap_count_waste(STRATEGIES[strategy], N, rho, counts.data_ptr(), _stream())
    return tuple(int(v) for v in counts.cpu().tolist())


def waste_counts(strategy: str, N: int, rho: int):
    """(blocks, fully idle blocks, idle threads) in closed form (host)."""
    return tdmap_waste_counts(STRATEGIES[strategy], N, rho)


def _make_autograd():
    torch = _torch()

    class EDM(torch.autograd.Function):
        """Packed lower-triangular EDM with the hand-written backward."""

        @staticmethod
        def forward(ctx, X, rho: int = 0, deterministic: bool = True):
            if rho not in FORWARD_RHOS:
                raise ValueError(f"rho must be one of {FORWARD_RHOS}, got {rho}")
            ctx.save_for_backward(X)
            # the backward tiles are 64, 128 or 256 cells wide; a forward
            # block size it has no tile for (the one-cell sweep, the paper's
            # 8 / 16 / 32 blocks) leaves the backward to the autotuner
            ctx.rho = rho if rho in BACKWARD_RHOS else 0
            ctx.deterministic = deterministic
            return edm(X.contiguous(), layout="packed", strategy="ltm", rho=rho)

        @staticmethod
        def backward(ctx, dD):
            (X,) = ctx.saved_tensors
            dX = edm_backward(X.contiguous(), dD.contiguous(), layout="packed",
                              rho=ctx.rho, deterministic=ctx.deterministic)
            return dX, None, None

    return EDM


# block sizes of the packed forward and of the backward (tdmap.h)
FORWARD_RHOS = (0, 1, 8, 16, 32, 64, 128, 256)
BACKWARD_RHOS = (0, 64, 128, 256)

_EDM = None


def EDM():
    """The torch.autograd.Function class (built on first use)."""
    global _EDM
    if _EDM is None:
        _EDM = _make_autograd()
    return _EDM
