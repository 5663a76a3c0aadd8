"""Pins for the oracle's exact-integer maps (CPU only).

Each test checks the oracle against something other than itself: the worked
example of the block numbering printed in the paper (Sec. II-A, Eq. (1)),
brute-force enumeration of the triangle, closed forms, and the inequalities
of the improvement model (Sec. II-B).
"""
import math
import os

import pytest

from oracle import maps


def _load_numbering(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "block_numbering.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            n, lam, i, j = (int(t) for t in line.split())
            rows.append((n, lam, i, j))
    return rows


def test_g_worked_example(golden_dir):
    rows = _load_numbering(golden_dir)
    assert len(rows) >= 10
    for n, lam, i, j in rows:
        assert maps.g_oracle(lam) == (i, j), (n, lam)
        if n:
            # the last row of an n-block triangle is row n-1
            assert i == n - 1


def test_g_matches_enumeration_below_2_16():
    count = 1 << 16
    ref = maps.g_enumerate(count)
    for lam in range(count):
        assert maps.g_oracle(lam) == ref[lam]


def test_g_row_boundaries_to_2_32():
    # every row start T_i below 2^32 and its neighbours: the definition
    # puts T_i at (i, 0), T_i - 1 at the end of row i-1 and T_i + 1 at (i, 1)
    i = 1
    while maps.tri(i) + 1 < (1 << 32):
        t = maps.tri(i)
        assert maps.g_oracle(t) == (i, 0)
        assert maps.g_oracle(t - 1) == (i - 1, i - 1)
        assert maps.g_oracle(t + 1) == (i, 1)
        i += 1
    assert i - 1 == 92681  # the last row that starts below 2^32 - 1
    assert maps.g_oracle((1 << 32) - 1) == (92681, (1 << 32) - 1 - maps.tri(92681))


def test_g_inverse_of_row_major_index():
    # lambda = i(i+1)/2 + j for 0 <= j <= i, i.e. g inverts Eq. (9)
    for i in list(range(0, 300)) + [46340, 65535, 92680]:
        for j in sorted({0, 1, i // 2, max(i - 1, 0), i}):
            if j <= i:
                assert maps.g_oracle(maps.tri(i) + j) == (i, j)


def test_g_nodiag_matches_enumeration():
    ref = [(i, j) for i in range(1, 400) for j in range(i)]
    for lam, cell in enumerate(ref):
        assert maps.g_oracle_nodiag(lam) == cell


def test_g_nodiag_printed_column_is_negative():
    # the column as printed in Eq. (10), lambda - i(i+1)/2, is negative for
    # every lambda; the oracle uses lambda - i(i-1)/2 instead
    for lam in range(2000):
        i, _ = maps.g_oracle_nodiag(lam)
        assert lam - maps.tri(i) < 0


def test_utm_formula_matches_enumeration():
    for n in range(2, 80):
        ref = maps.utm_enumerate(n)
        for k, cell in enumerate(ref):
            assert maps.utm_formula(n, k) == cell, (n, k)


@pytest.mark.parametrize("strategy", sorted(maps.STRATEGIES))
@pytest.mark.parametrize("rho", [1, 2, 3, 8, 16])
def test_strategy_covers_triangle_exactly_once(strategy, rho):
    Ns = list(range(1, 41)) + [63, 64, 65, 100, 127]
    for N in Ns:
        stats = maps.enumerate_waste(strategy, N, rho)
        assert stats["exact_cover"], (strategy, N, rho)


@pytest.mark.parametrize("strategy", sorted(maps.STRATEGIES))
def test_waste_closed_forms_match_enumeration(strategy):
    for N in [1, 2, 7, 16, 17, 50, 96, 129, 200]:
        for rho in [1, 2, 3, 4, 8, 16]:
            e = maps.enumerate_waste(strategy, N, rho)
            c = maps.waste_closed_form(strategy, N, rho)
            for key in ("blocks", "idle_blocks", "idle_lanes"):
                assert e[key] == c[key], (strategy, N, rho, key)


def test_bb_waste_is_quadratic_ltm_linear():
    # Sec. II-A: BB discards n(n-1)/2 blocks; LTM discards none on a 1D grid
    # and only the upper halves of its n diagonal blocks, ~n/2 block
    # equivalents, when rho divides N
    for N, rho in [(1024, 16), (30000, 8), (30000, 16), (30720, 16)]:
        n = maps.ceil_div(N, rho)
        bb = maps.waste_closed_form("bb", N, rho)
        ltm = maps.waste_closed_form("ltm", N, rho)
        assert bb["idle_blocks"] == n * (n - 1) // 2
        assert ltm["idle_blocks"] == 0
        assert ltm["blocks"] == n * (n + 1) // 2
        if N % rho == 0:
            assert ltm["idle_lanes"] == n * rho * (rho - 1) // 2
            equiv = ltm["idle_lanes"] / (rho * rho)
            assert abs(equiv - n / 2) <= n / (2 * rho) + 1e-9


def test_balanced_grid_idle_blocks_are_few():
    # the paper's n' x n' grid leaves n'^2 - T(n) < 2 n' + 1 blocks idle
    for n in [1, 2, 3, 10, 64, 1875, 3750]:
        side = maps.ltm_balanced_side(n)
        assert (side - 1) ** 2 < maps.tri(n) <= side ** 2
        assert side * side - maps.tri(n) < 2 * side + 1


def test_block_ratio_below_two():
    # Sec. II-B, Eq. (11) with k = 1: |G_BB| / |G_LTM| = 2n/(n+1) < 2
    for n in [1, 2, 3, 64, 1875, 10 ** 6]:
        r = maps.block_ratio(n)
        assert r < 2.0
        assert math.isclose(r, (n * n) / maps.tri(n), rel_tol=1e-15)
    assert math.isclose(maps.block_ratio(1875), 1.998934, rel_tol=1e-6)


def test_improvement_model_bounds():
    # Eqs. (12)-(15): I ~ 2/k for large n, 0 < I < 2, and the paper's
    # hypothesis k in [1.5, 2) gives 1.00 < I <= 1.33
    n = 10 ** 7
    for k in [1.0, 1.25, 1.5, 1.75, 1.999, 2.0, 3.0]:
        I = maps.improvement_model(n, k)
        assert 0 < I < 2
        assert math.isclose(I, 2.0 / k, rel_tol=1e-6)
    for k in [1.5, 1.6, 1.9, 1.99]:
        I = maps.improvement_model(n, k)
        assert 1.0 < I <= 1.34
    assert maps.improvement_model(n, 2.0) < 1.0


def test_rb_rectangle_holds_triangle():
    for N in range(1, 200):
        rows, cols = maps.rb_rectangle(N)
        assert rows * cols == maps.tri(N)


def test_rec_shape_matches_paper_sizes():
    # N = m 2^k with m a multiple of rho (Sec. III-B); the paper's largest
    # size 30720 = 15 * 2^7 * 16 is of that form at rho = 16
    assert maps.rec_shape(30720 // 16) == (15, 7)
    m, k = maps.rec_shape(1875)
    assert m * 2 ** k == 1920
    for nb in range(1, 3000):
        m, k = maps.rec_shape(nb)
        assert 1 <= m <= 16 and m * 2 ** k >= nb
        # no smaller admissible side exists
        for mm in range(1, 17):
            kk = 0
            while mm << kk < nb:
                kk += 1
            assert (mm << kk) >= m << k


def test_rec_exact_power_has_only_base_waste():
    N, rho = 30720, 16
    n = N // rho
    m, k = maps.rec_shape(n)
    c = maps.waste_closed_form("rec", N, rho)
    assert c["idle_blocks"] == (1 << k) * m * (m - 1) // 2
    assert c["blocks"] == (1 << k) * m * m + sum(
        (1 << (k - 1 - lev)) * (m << lev) ** 2 for lev in range(k))
