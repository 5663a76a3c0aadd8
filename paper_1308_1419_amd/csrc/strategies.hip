// The five space-of-computation strategies as the paper launches them
// (Sec. II-A, Sec. III-B): rho x rho threads per block, one cell per
// thread, the same per-pair function everywhere (so every strategy writes
// bit-identical values).  The maps are arithmetic only: no lookup tables,
// no auxiliary global memory (the restriction of Sec. III-B).
//
// Each kernel has two twins that evaluate the same map and filters: one
// counts blocks / fully idle blocks / idle threads instead of storing, the
// other is the paper's dummy kernel (Sec. III-A, Sec. IV), which measures
// the cost of the map alone.
#include "device.h"
#include "kernels.h"

namespace tdmap {

enum { kLTM = 0, kBB = 1, kUTM = 2, kRB = 3, kREC = 4 };
enum { kModeStore = 0, kModeCount = 1, kModeDummy = 2 };

template <int D, int LAYOUT, int MODE>
__device__ __forceinline__ void finish_cell(const EdmArgs &a, bool live, int64_t i, int64_t j,
                                            unsigned long long *counts) {
  if constexpr (MODE == kModeCount) {
    count_block(counts, live ? 1 : 0, (int)(blockDim.x * blockDim.y));
  } else if constexpr (MODE == kModeDummy) {
    // the mapping-cost kernel: the cell's i + j is "written" only when it
    // equals a run-time value no cell has, which keeps every step of the map
    // live without a store per thread to one address
    if (live && (uint32_t)(i + j) == a.never) a.sink[0] = (uint32_t)(i + j);
  } else {
    if (live) a.D[out_index<LAYOUT>(i, j, a.ldd)] = cell_dist<D>(a.X, a.ldx, a.d, i, j);
  }
}

// LTM: a 1D grid of exactly n(n+1)/2 blocks; block lambda covers block row
// and column g(lambda) (Sec. II-A, Eq. (2)).  Only the n diagonal blocks
// (and the edge when rho does not divide N) filter threads.
template <int D, int LAYOUT, int MODE>
__global__ void ltm_cell_kernel(EdmArgs a, uint32_t lam0, unsigned long long *counts) {
  uint32_t bi, bj;
  if constexpr (MODE == kModeDummy)
    g_lambda_variant(lam0 + blockIdx.x, a.variant, bi, bj);
  else
    g_lambda(lam0 + blockIdx.x, bi, bj);
  const int64_t i = (int64_t)bi * blockDim.y + threadIdx.y;
  const int64_t j = (int64_t)bj * blockDim.x + threadIdx.x;
  finish_cell<D, LAYOUT, MODE>(a, i < a.N && j <= i, i, j, counts);
}

// BB: an n x n grid (x = block column, y = block row).  A block above the
// diagonal returns before computing any thread coordinate; the others keep
// cells with j <= i < N (Sec. III-B).
template <int D, int LAYOUT, int MODE>
__global__ void bb_cell_kernel(EdmArgs a, unsigned long long *counts) {
  const uint32_t bx = blockIdx.x, by = blockIdx.y;
  // the timed kernels (EDM and dummy) discard the block at once; the
  // counting variant keeps every thread for the block-wide count
  if constexpr (MODE != kModeCount) {
    if (bx > by) return;
  }
  const int64_t i = (int64_t)by * blockDim.y + threadIdx.y;
  const int64_t j = (int64_t)bx * blockDim.x + threadIdx.x;
  finish_cell<D, LAYOUT, MODE>(a, bx <= by && i < a.N && j <= i, i, j, counts);
}

// UTM (Avril et al., Sec. III-B): thread k of a 1D grid takes the k-th pair
// (a, b), 1 <= a < b <= n, of the strictly upper triangle of an n x n
// matrix, with n = N + 1 so that there are exactly N(N+1)/2 pairs:
//   a = floor(((2n+1) - sqrt((2n-1)^2 - 8k)) / 2),
//   b = (a+1) + k - (a-1)(2n-a)/2.
// The square root is single precision; two integer conditionals repair a
// row that is off by one.  The pair is half-turned onto the lower triangle
// with the diagonal: (i, j) = (N - a, N + 1 - b), which keeps consecutive
// threads on one output row.
template <int D, int LAYOUT, int MODE>
__global__ void utm_cell_kernel(EdmArgs a, uint64_t k0, unsigned long long *counts) {
  const uint32_t lanes = blockDim.x * blockDim.y;
  const uint64_t k = k0 + (uint64_t)blockIdx.x * lanes + threadIdx.y * blockDim.x + threadIdx.x;
  const int64_t N = a.N;
  const uint64_t P = (uint64_t)N * (uint64_t)(N + 1) / 2;
  bool live = k < P;
  int64_t i = 0, j = 0;
  if (live) {
    const int64_t n = N + 1;
    const int64_t disc = (2 * n - 1) * (2 * n - 1) - 8 * (int64_t)k;
    const float sq = __builtin_amdgcn_sqrtf((float)disc);
    int64_t r = (int64_t)__builtin_floorf(((float)(2 * n + 1) - sq) * 0.5f);
    // start(a) = (a-1)(2n-a)/2 is the index of the first pair of row a
    const int64_t kk = (int64_t)k;
    if ((r - 1) * (2 * n - r) / 2 > kk) {
      --r;
    } else if (r * (2 * n - r - 1) / 2 <= kk) {
      ++r;
    }
    const int64_t b = (r + 1) + kk - (r - 1) * (2 * n - r) / 2;
    i = N - r;
    j = N + 1 - b;
    // a guess more than one row off would land outside the triangle: such
    // a thread stores nothing (the coverage tests would then fail)
    live = i >= 0 && i < N && j >= 0 && j <= i;
  }
  finish_cell<D, LAYOUT, MODE>(a, live, i, j, counts);
}

// RB (Jung et al., Sec. III-B): the threads form a rectangle; for even N
// it has N+1 rows and N/2 columns, the part above its diagonal being the
// turned-over sub-triangle of columns >= N/2.  Below the diagonal
// (ty > tx): (i, j) = (ty - 1, tx); on or above: (N - 1 - ty, N - 1 - tx).
// Odd N cuts at floor(N/2): N rows, floor(N/2)+1 columns, (ty, tx) when
// ty >= tx, else (N - 1 - ty, N - tx).
template <int D, int LAYOUT, int MODE>
__global__ void rb_cell_kernel(EdmArgs a, unsigned long long *counts) {
  const int64_t N = a.N;
  const int64_t ty = (int64_t)blockIdx.y * blockDim.y + threadIdx.y;
  const int64_t tx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool even = (N & 1) == 0;
  const int64_t rows = even ? N + 1 : N;
  const int64_t cols = even ? N / 2 : N / 2 + 1;
  const bool live = ty < rows && tx < cols;
  int64_t i, j;
  if (even) {
    if (ty > tx) {
      i = ty - 1;
      j = tx;
    } else {
      i = N - 1 - ty;
      j = N - 1 - tx;
    }
  } else {
    if (ty >= tx) {
      i = ty;
      j = tx;
    } else {
      i = N - 1 - ty;
      j = N - tx;
    }
  }
  finish_cell<D, LAYOUT, MODE>(a, live, i, j, counts);
}

// REC (Ries et al., Sec. III-B), in block units: the side is padded to
// m 2^k blocks (m <= 16).  mode 0 is the diagonal pass: 2^k base squares of
// m x m blocks, each a small bounding box (grid m x (m 2^k)).  mode 1 is one
// level of the bottom-up recursion with squares of side s = m 2^l: square q
// sits at block rows [(2q+1)s, (2q+2)s) and block columns [2qs, (2q+1)s)
// (grid s x (s * 2^(k-1-l))).  Block coordinates are computed at run time,
// not looked up.  Blocks past the real side nb are idle.
template <int D, int LAYOUT, int MODE>
__global__ void rec_cell_kernel(EdmArgs a, int mode, uint32_t side, uint32_t nb,
                                unsigned long long *counts) {
  const uint32_t q = blockIdx.y / side;
  const uint32_t lby = blockIdx.y - q * side;
  uint32_t R, C;
  bool blk_live;
  if (mode == 0) {
    R = q * side + lby;
    C = q * side + blockIdx.x;
    blk_live = blockIdx.x <= lby;
  } else {
    R = (2 * q + 1) * side + lby;
    C = 2 * q * side + blockIdx.x;
    blk_live = true;
  }
  blk_live = blk_live && R < nb;
  if constexpr (MODE != kModeCount) {
    if (!blk_live) return;
  }
  const int64_t i = (int64_t)R * blockDim.y + threadIdx.y;
  const int64_t j = (int64_t)C * blockDim.x + threadIdx.x;
  finish_cell<D, LAYOUT, MODE>(a, blk_live && i < a.N && j <= i, i, j, counts);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

static void rec_shape(uint32_t nb, uint32_t &m, uint32_t &k) {
  uint64_t best = 0;
  for (uint32_t mm = 16; mm >= 1; --mm) {
    uint32_t kk = 0;
    while (((uint64_t)mm << kk) < nb) ++kk;
    const uint64_t side = (uint64_t)mm << kk;
    if (best == 0 || side < best) {
      best = side;
      m = mm;
      k = kk;
    }
  }
}

template <int D, int LAYOUT, int MODE>
static hipError_t launch_cell_t(int strategy, int rho, const EdmArgs &a,
                                unsigned long long *counts) {
  const dim3 blk(rho, rho);
  const uint64_t lanes = (uint64_t)rho * rho;
  const uint64_t nb = (uint64_t)((a.N + rho - 1) / rho);
  // keep every launch below 2^32 work-items
  const uint64_t max_blocks = (((uint64_t)1 << 32) - 1) / lanes;
  hipError_t e = hipSuccess;
  switch (strategy) {
    case kLTM: {
      const uint64_t T = nb * (nb + 1) / 2;
      for (uint64_t l0 = 0; l0 < T; l0 += max_blocks) {
        const uint64_t c = T - l0 < max_blocks ? T - l0 : max_blocks;
        hipLaunchKernelGGL((ltm_cell_kernel<D, LAYOUT, MODE>), dim3((uint32_t)c), blk, 0,
                           a.stream, a, (uint32_t)l0, counts);
        if ((e = hipGetLastError()) != hipSuccess) return e;
      }
      return e;
    }
    case kBB:
      hipLaunchKernelGGL((bb_cell_kernel<D, LAYOUT, MODE>), dim3((uint32_t)nb, (uint32_t)nb),
                         blk, 0, a.stream, a, counts);
      return hipGetLastError();
    case kUTM: {
      const uint64_t P = (uint64_t)a.N * (uint64_t)(a.N + 1) / 2;
      const uint64_t blocks = (P + lanes - 1) / lanes;
      for (uint64_t b0 = 0; b0 < blocks; b0 += max_blocks) {
        const uint64_t c = blocks - b0 < max_blocks ? blocks - b0 : max_blocks;
        hipLaunchKernelGGL((utm_cell_kernel<D, LAYOUT, MODE>), dim3((uint32_t)c), blk, 0,
                           a.stream, a, b0 * lanes, counts);
        if ((e = hipGetLastError()) != hipSuccess) return e;
      }
      return e;
    }
    case kRB: {
      const int64_t rows = (a.N % 2 == 0) ? a.N + 1 : a.N;
      const int64_t cols = (a.N % 2 == 0) ? a.N / 2 : a.N / 2 + 1;
      const uint32_t gx = (uint32_t)((cols + rho - 1) / rho);
      const uint32_t gy = (uint32_t)((rows + rho - 1) / rho);
      if (gx == 0 || gy == 0) return hipSuccess;
      hipLaunchKernelGGL((rb_cell_kernel<D, LAYOUT, MODE>), dim3(gx, gy), blk, 0, a.stream, a,
                         counts);
      return hipGetLastError();
    }
    case kREC: {
      uint32_t m = 1, k = 0;
      rec_shape((uint32_t)nb, m, k);
      hipLaunchKernelGGL((rec_cell_kernel<D, LAYOUT, MODE>), dim3(m, m << k), blk, 0, a.stream,
                         a, 0, m, (uint32_t)nb, counts);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      for (uint32_t lev = 0; lev < k; ++lev) {
        const uint32_t s = m << lev;
        const uint32_t squares = 1u << (k - 1 - lev);
        hipLaunchKernelGGL((rec_cell_kernel<D, LAYOUT, MODE>), dim3(s, s * squares), blk, 0,
                           a.stream, a, 1, s, (uint32_t)nb, counts);
        if ((e = hipGetLastError()) != hipSuccess) return e;
      }
      return e;
    }
    default:
      return hipErrorInvalidValue;
  }
}

template <int LAYOUT>
static hipError_t launch_cell_layout(int strategy, int rho, const EdmArgs &a) {
  switch (a.d) {
    case 1: return launch_cell_t<1, LAYOUT, kModeStore>(strategy, rho, a, nullptr);
    case 2: return launch_cell_t<2, LAYOUT, kModeStore>(strategy, rho, a, nullptr);
    case 3: return launch_cell_t<3, LAYOUT, kModeStore>(strategy, rho, a, nullptr);
    case 4: return launch_cell_t<4, LAYOUT, kModeStore>(strategy, rho, a, nullptr);
    default: return launch_cell_t<0, LAYOUT, kModeStore>(strategy, rho, a, nullptr);
  }
}

hipError_t launch_cell(int strategy, int rho, const EdmArgs &a, unsigned long long *counts) {
  if (a.N == 0) return hipSuccess;
  if (counts) return launch_cell_t<1, kLayoutPacked, kModeCount>(strategy, rho, a, counts);
  return a.layout == kLayoutFull ? launch_cell_layout<kLayoutFull>(strategy, rho, a)
                                 : launch_cell_layout<kLayoutPacked>(strategy, rho, a);
}

hipError_t launch_dummy(int strategy, int rho, const EdmArgs &a) {
  if (a.N == 0) return hipSuccess;
  return launch_cell_t<1, kLayoutPacked, kModeDummy>(strategy, rho, a, nullptr);
}

}  // namespace tdmap
