"""The C ABI library on the CPU: it loads, exports every symbol the header
declares, and its host-only logic (validation, workspace sizes, closed-form
launch statistics) behaves as documented.  No call here reaches the GPU:
each one returns before any HIP call."""
import ctypes
import os
import re

import pytest

from oracle import maps
from paper_1308_1419_amd import tdmap

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tdmap.h")


def _header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tdmap_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(tdmap.LIB_PATH):
        pytest.fail("libtdmap.so is not built (run __graft_entry__.build())")
    return tdmap._load()


def test_library_exports_every_header_symbol(lib):
    names = _header_functions()
    assert len(names) >= 11
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(tdmap.EXPORTED)


def test_status_strings(lib):
    for s in range(5):
        assert tdmap.tdmap_status_string(s)
    assert tdmap.tdmap_status_string(99) == "unknown status"
    assert tdmap.tdmap_last_error() == ""


def test_validation_rejects_before_launch(lib):
    L = tdmap._load()
    # NULL X / D with N > 0
    assert L.tdmap_edm(None, 10, 3, 3, None, 10, 0, 0, 16, 0, None, 0, None) == tdmap.ERR_INVALID
    # N < 0, d < 1, ldx < d
    assert L.tdmap_edm(8, -1, 3, 3, 8, 10, 0, 0, 16, 0, None, 0, None) == tdmap.ERR_INVALID
    assert L.tdmap_edm(8, 10, 0, 3, 8, 10, 0, 0, 16, 0, None, 0, None) == tdmap.ERR_INVALID
    assert L.tdmap_edm(8, 10, 3, 2, 8, 10, 0, 0, 16, 0, None, 0, None) == tdmap.ERR_INVALID
    # ldd < N for the full layout; unknown layout / strategy / rho
    assert L.tdmap_edm(8, 10, 3, 3, 8, 9, 0, 0, 16, 0, None, 0, None) == tdmap.ERR_INVALID
    assert L.tdmap_edm(8, 10, 3, 3, 8, 10, 7, 0, 16, 0, None, 0, None) == tdmap.ERR_INVALID
    assert L.tdmap_edm(8, 10, 3, 3, 8, 10, 0, 9, 16, 0, None, 0, None) == tdmap.ERR_INVALID
    assert L.tdmap_edm(8, 10, 3, 3, 8, 10, 0, 0, 12, 0, None, 0, None) == tdmap.ERR_INVALID
    # tiled rho only for LTM / BB, d <= 4
    assert L.tdmap_edm(8, 10, 3, 3, 8, 10, 0, tdmap.RB, 128, 0, None, 0, None) == tdmap.ERR_UNSUPPORTED
    assert L.tdmap_edm(8, 10, 5, 5, 8, 10, 0, 0, 128, 0, None, 0, None) == tdmap.ERR_UNSUPPORTED
    # N = 0 is a no-op even with NULL buffers
    assert L.tdmap_edm(None, 0, 3, 3, None, 0, 0, 0, 16, 0, None, 0, None) == tdmap.OK
    # the map: NULL output, and a range past 2^32
    assert L.tdmap_map_blocks(0, 10, None, None) == tdmap.ERR_INVALID
    assert L.tdmap_map_blocks((1 << 32) - 5, 6, 8, None) == tdmap.ERR_UNSUPPORTED
    assert L.tdmap_map_blocks(5, 0, None, None) == tdmap.OK
    # UTM's thread index is 32-bit: N(N+1)/2 must stay below 2^32
    assert L.tdmap_edm(8, 100000, 3, 3, 8, 100000, 0, tdmap.UTM, 16, 0, None, 0, None) \
        == tdmap.ERR_UNSUPPORTED
    # map variants and the dummy kernel validate before launching
    assert L.tdmap_map_blocks_variant(0, 10, 3, 8, None) == tdmap.ERR_INVALID
    assert L.tdmap_map_blocks_variant(0, 10, 1, None, None) == tdmap.ERR_INVALID
    assert L.tdmap_dummy(tdmap.BB, 1, 100, 16, 0, 8, None) == tdmap.ERR_INVALID
    assert L.tdmap_dummy(0, 0, 100, 64, 0, 8, None) == tdmap.ERR_UNSUPPORTED
    assert L.tdmap_dummy(0, 0, 100, 16, 0, None, None) == tdmap.ERR_INVALID
    # the layout without the diagonal: FP32 tiles or the sweep, LTM / BB only
    S = tdmap.PACKED_STRICT
    for strat, rho in [(tdmap.LTM, 16), (tdmap.UTM, 16), (tdmap.RB, 8), (tdmap.REC, 32),
                       (tdmap.BB, 1), (tdmap.UTM, 64)]:
        assert L.tdmap_edm(8, 10, 3, 3, 16, 0, S, strat, rho, 0, None, 0, None) \
            == tdmap.ERR_UNSUPPORTED, (strat, rho)
    assert L.tdmap_edm(8, 10, 3, 3, 16, 0, S, 0, 0, tdmap.BF16_GRAM, 8, 1 << 20, None) \
        == tdmap.ERR_UNSUPPORTED
    # the sweep needs a 16-byte aligned output
    assert L.tdmap_edm(8, 10, 3, 3, 20, 0, S, 0, 1, 0, None, 0, None) == tdmap.ERR_UNSUPPORTED
    # NULL output: invalid unless N = 1 (no cell); a layout past the last one
    assert L.tdmap_edm(8, 10, 3, 3, None, 0, S, 0, 64, 0, None, 0, None) == tdmap.ERR_INVALID
    assert L.tdmap_edm(8, 10, 3, 3, 16, 0, 3, 0, 64, 0, None, 0, None) == tdmap.ERR_INVALID
    assert L.tdmap_edm_backward(8, 10, 3, 3, None, 0, S, 8, 64, 0, None, 0, None) \
        == tdmap.ERR_INVALID
    # the no-diagonal map validates like the map
    assert L.tdmap_map_blocks_nodiag(0, 10, None, None) == tdmap.ERR_INVALID
    assert L.tdmap_map_blocks_nodiag((1 << 32) - 5, 6, 8, None) == tdmap.ERR_UNSUPPORTED
    assert L.tdmap_map_blocks_nodiag(5, 0, None, None) == tdmap.OK
    # the write-stream fill wants a 16-byte aligned buffer
    assert L.tdmap_stream_fill(None, 16, ctypes.c_float(1.0), None) == tdmap.ERR_INVALID
    assert L.tdmap_stream_fill(8, 16, ctypes.c_float(1.0), None) == tdmap.ERR_INVALID
    assert L.tdmap_stream_fill(None, 0, ctypes.c_float(1.0), None) == tdmap.OK
    # the instrumented count needs a paper-style rho
    assert L.tdmap_count_waste(0, 100, 64, 8, None) == tdmap.ERR_UNSUPPORTED
    assert L.tdmap_count_waste(0, 100, 16, None, None) == tdmap.ERR_INVALID


def test_gram_workspace_sizes(lib):
    # BF16 copy (padded to 128 points x a multiple of 16 features) and the
    # norms; the split form holds a second BF16 array for the low parts
    N, d = 1000, 50
    Npad, KP = 1024, 64
    assert tdmap.tdmap_workspace_size(tdmap.OP_EDM, N, d, 0, 0, tdmap.BF16_GRAM) == \
        Npad * KP * 2 + Npad * 4
    assert tdmap.tdmap_workspace_size(tdmap.OP_EDM, N, d, 0, 0, tdmap.BF16X3_GRAM) == \
        2 * Npad * KP * 2 + Npad * 4
    L = tdmap._load()
    # the split form is validated like the BF16 form: packed LTM only, and a
    # workspace of the size above
    assert L.tdmap_edm(8, N, d, d, 16, N, tdmap.FULL, 0, 0, tdmap.BF16X3_GRAM, 8, 1 << 30,
                       None) == tdmap.ERR_UNSUPPORTED
    assert L.tdmap_edm(8, N, d, d, 16, 0, tdmap.PACKED, 0, 0, tdmap.BF16X3_GRAM, 8,
                       Npad * KP * 2 + Npad * 4, None) == tdmap.ERR_WORKSPACE
    assert L.tdmap_edm(8, N, d, d, 16, 0, tdmap.PACKED, 0, 0, 3, 8, 1 << 30, None) \
        == tdmap.ERR_INVALID
    # the BF16 copies are 16-byte chunks: a workspace off a 16-byte boundary
    # is refused before any launch, in both precisions and at every tile edge
    for prec in (tdmap.BF16_GRAM, tdmap.BF16X3_GRAM):
        for rho in (0, 128, 256):
            assert L.tdmap_edm(16, N, d, d, 16, 0, tdmap.PACKED, 0, rho, prec, 8, 1 << 30,
                               None) == tdmap.ERR_INVALID


def test_stress_validation_and_workspace(lib):
    L = tdmap._load()
    N, d = 1000, 3
    # per tile: 2 ts d gradient partials and one loss partial
    for ts in (64, 128, 256):
        nb = -(-N // ts)
        T = nb * (nb + 1) // 2
        assert tdmap.tdmap_workspace_size(tdmap.OP_STRESS, N, d, 0, ts, 1) == \
            T * (2 * ts * d + 1) * 4
    assert tdmap.tdmap_workspace_size(tdmap.OP_STRESS, N, d, 0, 0, 1) == max(
        tdmap.tdmap_workspace_size(tdmap.OP_STRESS, N, d, 0, ts, 1) for ts in (64, 128, 256))
    assert tdmap.tdmap_workspace_size(tdmap.OP_STRESS, N, d, 0, 64, 0) == 0
    assert tdmap.tdmap_workspace_size(tdmap.OP_STRESS, N, d, 0, 512, 1) == 0
    assert tdmap.tdmap_workspace_size(tdmap.OP_STRESS, N, 5, 0, 64, 1) == 0
    P = tdmap.PACKED
    # NULL loss / dX / delta, bad rho, d > 4, a workspace too small
    assert L.tdmap_stress_backward(8, N, d, d, 16, 0, P, 8, None, 64, 0, None, 0, None) \
        == tdmap.ERR_INVALID
    assert L.tdmap_stress_backward(8, N, d, d, 16, 0, P, None, 8, 64, 0, None, 0, None) \
        == tdmap.ERR_INVALID
    assert L.tdmap_stress_backward(8, N, d, d, None, 0, P, 8, 8, 64, 0, None, 0, None) \
        == tdmap.ERR_INVALID
    assert L.tdmap_stress_backward(8, N, d, d, 16, 0, P, 8, 8, 512, 0, None, 0, None) \
        == tdmap.ERR_INVALID
    assert L.tdmap_stress_backward(8, N, 5, 5, 16, 0, P, 8, 8, 64, 0, None, 0, None) \
        == tdmap.ERR_UNSUPPORTED
    need = tdmap.tdmap_workspace_size(tdmap.OP_STRESS, N, d, 0, 64, 1)
    assert L.tdmap_stress_backward(8, N, d, d, 16, 0, P, 8, 8, 64, 1, 16, need - 1, None) \
        == tdmap.ERR_WORKSPACE
    need0 = tdmap.tdmap_workspace_size(tdmap.OP_STRESS, N, d, 0, 0, 1)
    assert L.tdmap_stress_backward(8, N, d, d, 16, 0, P, 8, 8, 0, 1, 16, need0 - 1, None) \
        == tdmap.ERR_WORKSPACE  # rho = 0 needs room for either tile edge
    assert L.tdmap_stress_backward(8, N, d, d, 16, N - 1, tdmap.FULL, 8, 8, 64, 0, None, 0,
                                   None) == tdmap.ERR_INVALID


def test_fp32_needs_no_workspace(lib):
    for rho in (0, 8, 16, 32, 64, 128, 256):
        assert tdmap.tdmap_workspace_size(tdmap.OP_EDM, 30000, 3, 0, rho, tdmap.FP32) == 0


@pytest.mark.parametrize("strategy", ["ltm", "bb", "utm", "rb", "rec"])
def test_closed_form_waste_matches_oracle_enumeration(lib, strategy):
    for N in [1, 2, 5, 16, 17, 31, 64, 65, 100, 129]:
        for rho in [1, 2, 3, 8, 16]:
            e = maps.enumerate_waste(strategy, N, rho)
            got = tdmap.waste_counts(strategy, N, rho)
            assert got == (e["blocks"], e["idle_blocks"], e["idle_lanes"]), (N, rho)


@pytest.mark.parametrize("strategy", ["ltm", "bb", "utm", "rb", "rec"])
def test_closed_form_waste_matches_oracle_at_benchmark_sizes(lib, strategy):
    for N in [1024, 30000, 30720]:
        for rho in [8, 16, 32]:
            c = maps.waste_closed_form(strategy, N, rho)
            got = tdmap.waste_counts(strategy, N, rho)
            assert got == (c["blocks"], c["idle_blocks"], c["idle_lanes"]), (N, rho)


def test_waste_counts_invalid(lib):
    out = (ctypes.c_int64 * 3)()
    L = tdmap._load()
    assert L.tdmap_waste_counts(9, 10, 16, ctypes.addressof(out)) == tdmap.ERR_INVALID
    assert L.tdmap_waste_counts(0, 10, 0, ctypes.addressof(out)) == tdmap.ERR_INVALID
    assert L.tdmap_waste_counts(0, 10, 16, None) == tdmap.ERR_INVALID


def test_product_path_never_imports_oracle():
    # the binding and the HIP sources must not import, load or include
    # anything from oracle/
    pkg = os.path.join(ROOT, "paper_1308_1419_amd")
    pat = re.compile(r"(^\s*(from|import)\s+oracle\b)|liboracle|oracle/|#include.*oracle",
                     re.M)
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert not pat.search(text), f


def test_gram_kernel_choice_validates(lib):
    L = tdmap._load()
    G = tdmap.BF16_GRAM
    # Gram: rho 0, 128 or 256 only; packed LTM only
    assert L.tdmap_edm(8, 10, 64, 64, 8, 0, tdmap.PACKED, 0, 64, G, 8, 1 << 20, None) \
        == tdmap.ERR_UNSUPPORTED
    assert L.tdmap_edm(8, 10, 64, 64, 8, 0, tdmap.PACKED, 0, 256, G, None, 0, None) \
        == tdmap.ERR_WORKSPACE
    assert L.tdmap_gram_recompute_count(8, 10, 64, 64, 8, G, 256, 8, 1 << 20, None, None) \
        == tdmap.ERR_INVALID
    assert L.tdmap_gram_recompute_count(8, 10, 64, 64, 8, tdmap.FP32, 256, 8, 1 << 20, 8,
                                        None) == tdmap.ERR_INVALID
