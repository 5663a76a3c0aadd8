"""Exact-integer block maps, strategy coverage and waste counts (oracle).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

Everything here works on Python integers (arbitrary precision), so nothing is
subject to floating-point rounding.  The functions are deliberately plain:
loops and ``math.isqrt``; no blocking, no vectorisation.

Notation follows Sec. II-A of the paper: ``N`` is the problem size (number of
points, the td-problem has N(N+1)/2 cells), ``rho`` the dimensional block size
in threads, ``n = ceil(N / rho)`` the number of blocks per dimension and
``T(n) = n(n+1)/2`` the number of lower-triangular blocks.
"""
from __future__ import annotations

import math
from typing import Iterator, List, Optional, Tuple

Cell = Tuple[int, int]


def tri(i: int) -> int:
    """T(i) = i(i+1)/2: the index of the first block of row i in the
    row-major numbering of the lower triangle (Sec. II-A, Eq. (1))."""
    return i * (i + 1) // 2


def ceil_div(a: int, b: int) -> int:
    return -(-a // b)


# ---------------------------------------------------------------------------
# g(lambda): the lower-triangular map
# ---------------------------------------------------------------------------

def g_enumerate(count: int) -> List[Cell]:
    """The plain definition of the block numbering of Sec. II-A, Eq. (1):
    walk the lower triangle (diagonal included) row by row, left to right,
    and hand out consecutive indices.  Returns the first ``count`` cells."""
    out: List[Cell] = []
    i = 0
    while len(out) < count:
        for j in range(i + 1):
            out.append((i, j))
            if len(out) == count:
                break
        i += 1
    return out


def g_oracle(lam: int) -> Cell:
    """g(lambda) = (i, j) of Sec. II-A, Eq. (2), evaluated exactly.

    The proof (Eqs. (3)-(9)) writes lambda = x(x+1)/2, takes the positive
    root x = (sqrt(1 + 8 lambda) - 1)/2 (Eq. (7)), sets i = floor(x) (Eq. (8))
    and j = lambda - i(i+1)/2 (Eq. (9)).  With the integer square root,
    floor((sqrt(8 lambda + 1) - 1)/2) = (isqrt(8 lambda + 1) - 1) // 2 holds
    exactly: both sides are the largest i with i(i+1)/2 <= lambda.
    """
    if lam < 0:
        raise ValueError("lambda must be non-negative")
    i = (math.isqrt(8 * lam + 1) - 1) // 2
    return i, lam - tri(i)


def g_oracle_nodiag(lam: int) -> Cell:
    """Map without the diagonal (Sec. II-A, Eq. (10)): lambda enumerates the
    strictly lower triangle {(i, j): 0 <= j < i} row-major.

    Eq. (10) gives i = floor(sqrt(1/4 + 2 lambda) + 1/2), i.e. the largest i
    with i(i-1)/2 <= lambda.  The printed column, lambda - i(i+1)/2, is
    negative for every lambda (it subtracts the start of the *next* row);
    the reading used here is j = lambda - i(i-1)/2, the offset of lambda from
    the start of row i in the strictly lower numbering.
    """
    if lam < 0:
        raise ValueError("lambda must be non-negative")
    # largest i >= 1 with i(i-1)/2 <= lam  <=>  (2i-1)^2 <= 8 lam + 1
    i = (math.isqrt(8 * lam + 1) + 1) // 2
    return i, lam - i * (i - 1) // 2


# ---------------------------------------------------------------------------
# Strategy coverage by enumeration (Sec. II-A and Sec. III-B)
#
# Each ``cover_*`` generator yields one entry per launched block, in launch
# order: (lanes, cells) where ``lanes`` is the number of threads in the block
# and ``cells`` the (i, j) cells those threads write (idle lanes write none).
# A strategy is correct when the cells of all blocks, taken together, are
# every (i, j) with 0 <= j <= i < N exactly once.
# ---------------------------------------------------------------------------

BlockCover = Tuple[int, List[Cell]]


def _square_block(N: int, rho: int, bi: int, bj: int) -> List[Cell]:
    """Cells written by a rho x rho block placed at block row ``bi`` and block
    column ``bj``: a lane keeps (i, j) when i < N and j <= i (the thread-level
    diagonal filter, Sec. II-A after Fig. 2 and Sec. III-B on BB)."""
    cells = []
    for ty in range(rho):
        i = bi * rho + ty
        if i >= N:
            continue
        for tx in range(rho):
            j = bj * rho + tx
            if j <= i:
                cells.append((i, j))
    return cells


def cover_bb(N: int, rho: int) -> Iterator[BlockCover]:
    """Bounding box, Sec. II-A and Sec. III-B: an n x n grid; a block whose
    column index exceeds its row index returns at once, the others filter
    their lanes against the diagonal and the edge."""
    n = ceil_div(N, rho)
    for by in range(n):
        for bx in range(n):
            if bx > by:
                yield rho * rho, []
            else:
                yield rho * rho, _square_block(N, rho, by, bx)


def cover_ltm(N: int, rho: int) -> Iterator[BlockCover]:
    """LTM on a 1D grid of exactly T(n) blocks: block lambda goes to block
    (i, j) = g(lambda) (Sec. II-A, Eq. (2))."""
    n = ceil_div(N, rho)
    for lam in range(tri(n)):
        bi, bj = g_oracle(lam)
        yield rho * rho, _square_block(N, rho, bi, bj)


def ltm_balanced_side(n: int) -> int:
    """n' = ceil(sqrt(n(n+1)/2)), the side of the paper's balanced 2D grid
    (Sec. II-A)."""
    t = tri(n)
    s = math.isqrt(t)
    return s if s * s == t else s + 1


def cover_ltm_balanced(N: int, rho: int) -> Iterator[BlockCover]:
    """LTM as the paper launches it: an n' x n' grid, lambda = x + y n'
    (Sec. II-A, Lemma); blocks with lambda >= T(n) do nothing."""
    n = ceil_div(N, rho)
    side = ltm_balanced_side(n)
    for y in range(side):
        for x in range(side):
            lam = x + y * side
            if lam >= tri(n):
                yield rho * rho, []
            else:
                bi, bj = g_oracle(lam)
                yield rho * rho, _square_block(N, rho, bi, bj)


def rb_rectangle(N: int) -> Tuple[int, int]:
    """(rows, cols) of the rectangular-box grid in threads (Sec. III-B).

    Even N: the sub-triangle with column > N/2 is turned over above the
    diagonal; the result has N+1 rows and N/2 columns.  Odd N: cut at
    floor(N/2); N rows and floor(N/2)+1 columns.  Both hold N(N+1)/2 cells.
    """
    if N % 2 == 0:
        return N + 1, N // 2
    return N, N // 2 + 1


def rb_cell(N: int, ty: int, tx: int) -> Cell:
    """Rectangular-box thread (ty, tx) -> cell (Sec. III-B).

    The printed rule (below the diagonal i = ty - 1 with j unchanged; on or
    above it i = N - ty - 1) leaves the column of the turned-over part
    garbled.  Reading used: the turned-over thread takes the column mirrored
    about the last one, j = N - 1 - tx for even N and j = N - tx for odd N,
    which makes the map a bijection onto the triangle (checked by
    enumeration in the tests).
    """
    if N % 2 == 0:
        if ty > tx:
            return ty - 1, tx
        return N - 1 - ty, N - 1 - tx
    if ty >= tx:
        return ty, tx
    return N - 1 - ty, N - tx


def cover_rb(N: int, rho: int) -> Iterator[BlockCover]:
    """Rectangular box tiled by rho x rho blocks; lanes outside the rectangle
    are idle."""
    rows, cols = rb_rectangle(N)
    for by in range(ceil_div(rows, rho)):
        for bx in range(ceil_div(cols, rho)):
            cells = []
            for ly in range(rho):
                ty = by * rho + ly
                for lx in range(rho):
                    tx = bx * rho + lx
                    if ty < rows and tx < cols:
                        cells.append(rb_cell(N, ty, tx))
            yield rho * rho, cells


def rec_shape(nb: int, max_base: int = 16) -> Tuple[int, int]:
    """(m, k) for the recursive partition in block units (Sec. III-B): the
    problem side is m 2^k blocks with m <= ``max_base``.  For a side that is
    not of that form the smallest m 2^k >= nb is taken (ties: the largest m,
    i.e. the fewest levels); the blocks past nb are idle."""
    if nb <= 0:
        raise ValueError("nb must be positive")
    best: Optional[Tuple[int, int, int]] = None
    for m in range(max_base, 0, -1):
        k = 0
        while m << k < nb:
            k += 1
        side = m << k
        if best is None or side < best[0]:
            best = (side, m, k)
    assert best is not None
    return best[1], best[2]


def rec_launches(N: int, rho: int) -> List[List[Tuple[int, int]]]:
    """The launches of the recursive partition, each a list of the
    (block row, block column) its blocks are placed at, in launch order.

    Launch 0 is the extra diagonal pass (Sec. III-B): 2^k base squares of
    m x m blocks along the diagonal, each run as a small bounding box (blocks
    above its diagonal return at once; they are listed with column > row).
    Launch l+1 (l = 0..k-1) is level l of the bottom-up recursion: 2^(k-1-l)
    squares of (m 2^l) x (m 2^l) blocks; square q sits at block rows
    [(2q+1) m 2^l, (2q+2) m 2^l) and block columns [2q m 2^l, (2q+1) m 2^l),
    i.e. directly below the pair of triangles it joins.
    """
    nb = ceil_div(N, rho)
    m, k = rec_shape(nb)
    launches: List[List[Tuple[int, int]]] = []
    diag = []
    for q in range(1 << k):
        for by in range(m):
            for bx in range(m):
                diag.append((q * m + by, q * m + bx))
    launches.append(diag)
    for lev in range(k):
        s = m << lev
        blocks = []
        for q in range(1 << (k - 1 - lev)):
            for by in range(s):
                for bx in range(s):
                    blocks.append(((2 * q + 1) * s + by, 2 * q * s + bx))
        launches.append(blocks)
    return launches


def cover_rec(N: int, rho: int) -> Iterator[BlockCover]:
    nb = ceil_div(N, rho)
    for launch in rec_launches(N, rho):
        for bi, bj in launch:
            if bj > bi or bi >= nb:
                yield rho * rho, []
            else:
                yield rho * rho, _square_block(N, rho, bi, bj)


def utm_enumerate(n: int) -> List[Cell]:
    """Plain definition behind the upper-triangular mapping of Sec. III-B: the
    strictly upper triangle {(a, b): 1 <= a < b <= n} of an n x n matrix,
    1-indexed, walked row by row; thread k takes the k-th pair."""
    return [(a, b) for a in range(1, n) for b in range(a + 1, n + 1)]


def utm_formula(n: int, k: int) -> Cell:
    """The printed UTM formula (Sec. III-B),
        a = floor((-(2n+1) + sqrt(4n^2 - 4n - 8k + 1)) / -2),
        b = (a+1) + k - (a-1)(2n-a)/2,
    evaluated exactly: with s = isqrt(D), floor((2n+1 - sqrt D)/2) equals
    (2n+1-s)//2 when D is a perfect square and (2n-s)//2 otherwise."""
    D = 4 * n * n - 4 * n - 8 * k + 1
    s = math.isqrt(D)
    a = (2 * n + 1 - s) // 2 if s * s == D else (2 * n - s) // 2
    b = (a + 1) + k - (a - 1) * (2 * n - a) // 2
    return a, b


def utm_cell(N: int, k: int) -> Cell:
    """UTM thread k -> cell of the lower triangle with diagonal.

    The map of Sec. III-B covers the strictly upper triangle of an n x n
    matrix; with n = N + 1 it has N(N+1)/2 pairs, one per cell of our
    triangle.  A half-turn, (i, j) = (N - a, N + 1 - b), sends it onto
    {0 <= j <= i < N} (the paper notes that upper and lower domains are
    interchangeable by transposition; the half-turn keeps consecutive k on
    one output row)."""
    a, b = utm_formula(N + 1, k)
    return N - a, N + 1 - b


def cover_utm(N: int, rho: int) -> Iterator[BlockCover]:
    """UTM maps threads, not blocks: a 1D grid of ceil(P / rho^2) blocks of
    rho^2 threads, P = N(N+1)/2; threads with k >= P are idle."""
    P = tri(N)
    lanes = rho * rho
    for blk in range(ceil_div(P, lanes)):
        cells = []
        for t in range(lanes):
            k = blk * lanes + t
            if k < P:
                cells.append(utm_cell(N, k))
        yield lanes, cells


STRATEGIES = {
    "ltm": cover_ltm,
    "ltm_balanced": cover_ltm_balanced,
    "bb": cover_bb,
    "rb": cover_rb,
    "rec": cover_rec,
    "utm": cover_utm,
}


def enumerate_waste(strategy: str, N: int, rho: int) -> dict:
    """Launch statistics of a strategy by enumeration: blocks launched, fully
    idle blocks (blocks that write nothing), idle lanes, and whether the
    written cells are exactly the triangle, each once."""
    seen = set()
    blocks = idle_blocks = idle_lanes = dup = 0
    for lanes, cells in STRATEGIES[strategy](N, rho):
        blocks += 1
        if not cells:
            idle_blocks += 1
        idle_lanes += lanes - len(cells)
        for c in cells:
            if c in seen:
                dup += 1
            seen.add(c)
    exact = dup == 0 and len(seen) == tri(N) and all(
        0 <= j <= i < N for i, j in seen)
    return {"blocks": blocks, "idle_blocks": idle_blocks,
            "idle_lanes": idle_lanes, "exact_cover": exact}


# ---------------------------------------------------------------------------
# Closed forms (Sec. II-A: BB wastes n(n-1)/2 blocks, LTM O(n))
# ---------------------------------------------------------------------------

def waste_closed_form(strategy: str, N: int, rho: int) -> dict:
    """Blocks launched, fully idle blocks and idle lanes in closed form.

    BB launches n^2 blocks of which the n(n-1)/2 above the diagonal are idle;
    LTM on a 1D grid launches T(n) blocks, none idle; its only idle lanes are
    the upper halves of the n diagonal blocks (rho(rho-1)/2 each, about n/2
    block equivalents, the paper's O(n)) plus the edge when rho does not
    divide N.  RB and UTM tile a region of exactly P = N(N+1)/2 cells, so
    only their last row/column of blocks carries idle lanes.  REC is summed
    over its launches.
    """
    n = ceil_div(N, rho)
    P = tri(N)
    lanes = rho * rho
    if strategy == "bb":
        blocks, idle = n * n, n * (n - 1) // 2
    elif strategy == "ltm":
        blocks, idle = tri(n), 0
    elif strategy == "ltm_balanced":
        side = ltm_balanced_side(n)
        blocks, idle = side * side, side * side - tri(n)
    elif strategy == "rb":
        rows, cols = rb_rectangle(N)
        blocks, idle = ceil_div(rows, rho) * ceil_div(cols, rho), 0
    elif strategy == "utm":
        blocks, idle = ceil_div(P, lanes), 0
    elif strategy == "rec":
        m, k = rec_shape(n)
        side = m << k
        # diagonal pass: 2^k squares of m^2 blocks; the m(m-1)/2 above each
        # base diagonal are idle, and so is every base block row >= n.
        blocks = (1 << k) * m * m
        idle = (1 << k) * (m * (m - 1) // 2)
        # base block rows >= n that are on or below their base diagonal
        for q in range(1 << k):
            for by in range(m):
                if q * m + by >= n:
                    idle += by + 1
        for lev in range(k):
            s = m << lev
            for q in range(1 << (k - 1 - lev)):
                blocks += s * s
                r0 = (2 * q + 1) * s
                idle += s * max(0, min(s, r0 + s - n))
        del side
    else:
        raise ValueError(strategy)
    return {"blocks": blocks, "idle_blocks": idle,
            "idle_lanes": blocks * lanes - P}


# ---------------------------------------------------------------------------
# Improvement model (Sec. II-B)
# ---------------------------------------------------------------------------

def block_ratio(n: int) -> float:
    """|G_BB| / |G_LTM| = n^2 / (n(n+1)/2) = 2n/(n+1), the factor in Eq. (11)
    when the per-block costs are equal (k = 1)."""
    return 2.0 * n / (n + 1)


def improvement_model(n: int, k: float) -> float:
    """I = beta |G_BB| rho^2 / (tau |G_LTM| rho^2) with tau = k beta
    (Sec. II-B, Eq. (11)) = 2 n^2 / (k (n^2 + n))."""
    return 2.0 * n * n / (k * (n * n + n))
