// Gram-form EDM on the MFMA units (gfx950), packed output.
//
//   D_ij^2 = ||x_i||^2 + ||x_j||^2 - 2 x_i . x_j
//
// A prologue rounds X to BF16 (round to nearest even), pads the features to
// a multiple of 16 with zeros and the points to a multiple of 128, and
// computes the squared norms of the rounded points in FP32.  The main
// kernel walks the triangle by g(lambda) (Sec. II-A, Eq. (2)) on 256 x 256
// tiles, a work-group taking one row half (two 128 x 128 tiles side by
// side); each wave owns 32 rows x 128 columns of one of them, computed by
// four v_mfma_f32_32x32x16_bf16 accumulators (BF16 products are exact in
// FP32, the sums accumulate in FP32).  The epilogue forms
// G = n_i + n_j - 2 acc and, when G <= theta (n_i + n_j) (theta = 1/4:
// the pair is close relative to its norms, where the Gram form cancels),
// recomputes the distance exactly in FP32 difference form from the FP32
// points; otherwise it stores sqrt(G).
//
// Split mode (precision BF16X3): each point is held as x = hi + lo with
// hi = bf16(x) and lo = bf16(x - hi) (x - hi is exact in FP32, and hi + lo
// is exact in FP32), the norms are those of hi + lo, and the dot product is
// hi.hi' + hi.lo' + lo.hi', three MFMA products into the same FP32
// accumulator; only lo.lo' (below 2^-16 of |x||y|) is dropped.
#include "device.h"
#include "kernels.h"

namespace tdmap {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kGramTile = 128;
constexpr float kGramTheta = 0.25f;

__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// One thread per padded point: BF16 copy (zero padded) and the squared norm
// of the represented point; with Xlo != nullptr also the low parts.
__global__ __launch_bounds__(256) void gram_prologue_kernel(const float *__restrict__ X, int64_t N, int d,
                                                            int64_t ldx, uint16_t *__restrict__ Xb,
                                                            uint16_t *__restrict__ Xlo,
                                                            float *__restrict__ nrm, int64_t Npad,
                                                            int KP) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= Npad) return;
  float s = 0.0f;
  for (int k = 0; k < KP; ++k) {
    const float v = (p < N && k < d) ? X[p * ldx + k] : 0.0f;
    const uint16_t b = bf16_rne(v);
    Xb[p * KP + k] = b;
    float r = bf16_to_f32(b);
    if (Xlo != nullptr) {
      const uint16_t c = bf16_rne(v - r);
      Xlo[p * KP + k] = c;
      r += bf16_to_f32(c);
    }
    s = __builtin_fmaf(r, r, s);
  }
  nrm[p] = s;
}

// FP32 difference form with eight interleaved partial sums combined as a
// tree, which keeps the rounding error of the squared distance near
// (d/8 + 6) units of roundoff.
__device__ __forceinline__ float exact_dist(const float *__restrict__ X, int64_t ldx, int d, int64_t i,
                                         int64_t j) {
  float s[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) s[u] = 0.0f;
  const float *xi = X + i * ldx;
  const float *xj = X + j * ldx;
  for (int k0 = 0; k0 < d; k0 += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (k0 + u < d) {
        const float t = xi[k0 + u] - xj[k0 + u];
        s[u] = __builtin_fmaf(t, t, s[u]);
      }
    }
  }
  const float q = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
  return __builtin_amdgcn_sqrtf(q);
}

typedef float f4 __attribute__((ext_vector_type(4)));

// Each wave owns 32 whole rows of the 128 x 128 tile: four 32 x 32
// v_mfma_f32_32x32x16_bf16 accumulators (one per 32-column block).  Its
// distances go, 16 rows at a time, through a wave-private LDS slice and are
// written as packed rows with 16-byte stores; no work-group barrier is
// needed, so the waves run independently.
//
// Store layout: a half-wave writes one 128-cell row segment.  Packed row i's
// segment [col0, col0 + 128) starts sh = (i(i+1)/2 + col0) mod 4 positions
// past a 16-byte boundary; lane h stores the aligned chunk at columns
// col0 - sh + 4h .. + 3, read from LDS at that shift.  The cells of the two
// partial chunks at the ends of each segment (the neighbouring tiles write
// the rest of those chunks) are gathered one row per lane and written with
// four instructions per 16 rows: single-lane stores per row would multiply
// the store instruction count several times over.  Diagonal and edge rows
// go cell by cell.
constexpr int kGramRows = 16;  // rows staged per step and wave

// (i(i+1)/2 + col0) mod 4 for the tile row rr of a 16-row step: the step's
// first row is a multiple of 16 and col0 a multiple of 128, and
// i(i+1)/2 mod 4 has period 8 in i.
__device__ __forceinline__ int row_shift(int rr) {
  const int m = rr & 7;
  return ((m * (m + 1)) >> 1) & 3;
}


// KPC: the padded feature count as a compile-time constant (16, 32, 64 or
// 128), which unrolls the MFMA loop so that the loads of every feature step
// are issued before the first product waits (measured: split form 9.5 ->
// 8.7 ms at N = 100000, d = 64); 0 for any other count.
template <bool SPLIT, int KPC>
__global__ __launch_bounds__(512, SPLIT ? 3 : 4) void gram_tile_kernel(GramArgs a, uint32_t lam0,
                                                                      uint32_t nblk) {
  // Eight waves: the two side-by-side 128 x 128 tiles (I, 2 J2) and
  // (I, 2 J2 + 1) that form one row half, I = 2 I2 + wg mod 2, of the
  // 256 x 256 tile (I2, J2) = g(wg / 2), so each row is written as a 1 KB
  // segment (measured 7.2 -> 7.0 ms, split 8.7 -> 8.4 ms, against one 128 x
  // 128 tile per work-group; four tiles side by side gave the gain back).
  // Each XCD takes one contiguous range of wg: neighbouring tiles share
  // the partial 16-byte chunks (and lines) at the ends of their row
  // segments, which then combine in one L2 (measured 9.6 -> 7.2 ms), and
  // they share their BF16 row block.
  const uint32_t wg = lam0 + xcd_contiguous(blockIdx.x, nblk);
  uint32_t I2, J2;
  g_lambda(wg >> 1, I2, J2);
  const int wl = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint32_t I = 2 * I2 + (wg & 1);
  uint32_t J = 2 * J2 + (wl >> 2);
  I = __builtin_amdgcn_readfirstlane(I);  // uniform: keep the tile origin scalar
  J = __builtin_amdgcn_readfirstlane(J);
  // the upper right tile of a diagonal 256 x 256 tile, or rows past N
  if (J > I || (int64_t)I * kGramTile >= a.N) return;
  const int w = wl & 3;  // the wave's 32-row block of its 128 x 128 tile
  const int l = threadIdx.x & 63;
  const int lr = l & 31;
  const int lk = (l >> 5) * 8;
  const int64_t N = a.N;
  const int64_t row0 = (int64_t)I * kGramTile;
  const int64_t col0 = (int64_t)J * kGramTile;
  const int64_t rw = row0 + 32 * w;  // this wave's first row
  const bool diag = I == J;
  // on a diagonal tile, column blocks right of this wave's rows are above
  // the diagonal
  const int nbj = diag ? w + 1 : 4;
  const int KP = KPC ? KPC : a.KP;
  const uint16_t *__restrict__ Xb = a.Xb;

  float nr[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) nr[v] = a.nrm[rw + (v >> 2) * 8 + (l >> 5) * 4 + (v & 3)];
  float nc[4];
#pragma unroll
  for (int bj = 0; bj < 4; ++bj) nc[bj] = a.nrm[col0 + bj * 32 + lr];

  f32x16 acc[4];
#pragma unroll
  for (int bj = 0; bj < 4; ++bj)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[bj][v] = 0.0f;
  // lane l supplies row (l % 32) of a 32-row block and the 8 features
  // [8 (l / 32), 8 (l / 32) + 8) of each 16-feature step; B uses the same
  // assignment for its points, so the product is x_i . x_j.
  const uint16_t *__restrict__ Xl = a.Xlo;
  auto kstep = [&](int k) {
    const int64_t ao = (rw + lr) * KP + k + lk;
    const bf16x8 av = *reinterpret_cast<const bf16x8 *>(Xb + ao);
    bf16x8 al;
    if constexpr (SPLIT) al = *reinterpret_cast<const bf16x8 *>(Xl + ao);
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
      if (bj < nbj) {
        const int64_t bo = (col0 + bj * 32 + lr) * KP + k + lk;
        const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(Xb + bo);
        if constexpr (SPLIT) {
          const bf16x8 bl = *reinterpret_cast<const bf16x8 *>(Xl + bo);
          acc[bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bv, acc[bj], 0, 0, 0);
          acc[bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bl, acc[bj], 0, 0, 0);
        }
        acc[bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[bj], 0, 0, 0);
      }
    }
  };
  if constexpr (KPC != 0) {
#pragma unroll
    for (int k = 0; k < KPC; k += 16) kstep(k);
  } else {
    for (int k = 0; k < KP; k += 16) kstep(k);
  }

  // stage row rr holds column c at position c + sh(rr), where sh(rr) is the
  // offset of the packed row past a 16-byte boundary; the stored chunks are
  // then aligned 16-byte LDS reads without bank conflicts
  __shared__ __align__(16) float stage[8][kGramRows][kGramTile + 4];
  float(*st)[kGramTile + 4] = stage[wl];
  float *__restrict__ out = a.D;
  const int h = l & 31;
  const bool full_rows = !diag && row0 + kGramTile <= N;
#pragma unroll
  for (int vh = 0; vh < 2; ++vh) {
    // accumulator v of a 32 x 32 block holds row (v/4)*8 + (l/32)*4 + v%4
    // and column l % 32; v in [8 vh, 8 vh + 8) are the rows 16 vh .. +15
    bool any = false;
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
#pragma unroll
      for (int v = 8 * vh; v < 8 * vh + 8; ++v) {
        const int rr = (v >> 2) * 8 + (l >> 5) * 4 + (v & 3) - 16 * vh;
        const float sn = nr[v] + nc[bj];
        const float G = __builtin_fmaf(-2.0f, acc[bj][v], sn);
        const bool rec = G <= kGramTheta * sn;
        any |= rec;
        // a pair below the threshold is marked -1 and filled in below
        st[rr][bj * 32 + lr + row_shift(rr)] = rec ? -1.0f : __builtin_amdgcn_sqrtf(G);
      }
    }
    if (any) {
      // rare: the diagonal and near-duplicate pairs, exact FP32 difference
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) {
#pragma unroll
        for (int v = 8 * vh; v < 8 * vh + 8; ++v) {
          const int rr = (v >> 2) * 8 + (l >> 5) * 4 + (v & 3) - 16 * vh;
          const int c = bj * 32 + lr + row_shift(rr);
          if (st[rr][c] < 0.0f) {
            const int64_t i = rw + 16 * vh + rr;
            const int64_t j = col0 + bj * 32 + lr;
            st[rr][c] = (i < N && j <= i) ? exact_dist(a.X, a.ldx, a.d, i, j) : 0.0f;
          }
        }
      }
    }
    // the wave reads back its own LDS writes: no barrier needed
    if (full_rows) {
      // Row rw + m (m < 32) starts at T(rw) + col0 + m rw + m(m+1)/2: a
      // uniform base and a 32-bit offset (m rw < 32 N < 2^30 under the
      // 32-bit tile index), with the row's shift row_shift(m) (rw is a
      // multiple of 32, so T(rw) and m rw add nothing mod 4).
      float *__restrict__ outw = out + tri64((uint64_t)rw) + (uint64_t)col0;
      const uint32_t rw32 = (uint32_t)rw;
      auto row_off = [&](uint32_t m) { return m * rw32 + ((m * (m + 1)) >> 1); };
      // cell offset -> address as a 32-bit byte offset from the uniform base
      auto at = [&](uint32_t e) {
        return reinterpret_cast<float *>(reinterpret_cast<char *>(outw) + e * 4u);
      };
      // whole aligned chunks, two rows per instruction
#pragma unroll 2
      for (int p = 0; p < kGramRows / 2; ++p) {
        const int r = 2 * p + (l >> 5);
        const uint32_t m = 16 * vh + r;
        const int sh = row_shift(r);
        if (h > 0 || sh == 0) {
          const f4 v4 = *reinterpret_cast<const f4 *>(&st[r][4 * h]);
          f4 *dst = reinterpret_cast<f4 *>(at(row_off(m) - sh + 4 * h));
          // BF16 form: plain stores (6.3 against 7.0 ms with non-temporal
          // ones); the split form keeps non-temporal stores (8.4 against
          // 9.3 ms with plain ones)
          if constexpr (SPLIT)
            __builtin_nontemporal_store(v4, dst);
          else
            *dst = v4;
        }
      }
      // the partial chunks at both ends of every row: the 4 - sh head cells
      // (columns 0 .. 3 - sh) and the sh tail cells (columns 128 - sh .. 127),
      // one row per lane, four instructions for all 16 rows
      if (l < kGramRows) {
        const uint32_t m = 16 * vh + l;
        const int sh = row_shift(l);
        if (sh != 0) {
          const uint32_t o0 = row_off(m);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int c = q < 4 - sh ? q : kGramTile - 4 + q;
            // plain (cached) store: the neighbouring tile writes the rest
            // of this 16-byte chunk, and the two halves then meet in L2
            // instead of reaching HBM as two partial line writes
            *at(o0 + c) = st[l][c + sh];
          }
        }
      }
    } else {
      for (int p = 0; p < kGramRows / 2; ++p) {
        const int r = 2 * p + (l >> 5);
        const int64_t i = rw + 16 * vh + r;
        if (i >= N) continue;
        const uint64_t first = tri64((uint64_t)i) + (uint64_t)col0;
        const int sh = (int)(first & 3);
        const int64_t jmax = (diag ? i : N - 1) - col0;
        for (int c = h; c < kGramTile; c += 32)
          if (c <= jmax) __builtin_nontemporal_store(st[r][c + sh], out + first + c);
      }
    }
  }
}

template <bool SPLIT>
static void launch_gram_tiles(int KP, dim3 grid, hipStream_t stream, const GramArgs &a, uint32_t l0) {
  const dim3 block(512);
  switch (KP) {
    case 16:
      hipLaunchKernelGGL((gram_tile_kernel<SPLIT, 16>), grid, block, 0, stream, a, l0, grid.x);
      break;
    case 32:
      hipLaunchKernelGGL((gram_tile_kernel<SPLIT, 32>), grid, block, 0, stream, a, l0, grid.x);
      break;
    case 64:
      hipLaunchKernelGGL((gram_tile_kernel<SPLIT, 64>), grid, block, 0, stream, a, l0, grid.x);
      break;
    case 128:
      hipLaunchKernelGGL((gram_tile_kernel<SPLIT, 128>), grid, block, 0, stream, a, l0, grid.x);
      break;
    default:
      hipLaunchKernelGGL((gram_tile_kernel<SPLIT, 0>), grid, block, 0, stream, a, l0, grid.x);
  }
}

size_t gram_workspace_bytes(int64_t N, int d, bool split) {
  const int64_t Npad = (N + kGramTile - 1) / kGramTile * kGramTile;
  const int64_t KP = (d + 15) / 16 * 16;
  return (size_t)Npad * (size_t)KP * 2 * (split ? 2 : 1) + (size_t)Npad * 4;
}

hipError_t launch_gram(const float *X, int64_t N, int d, int64_t ldx, float *D, void *ws, bool split,
                       hipStream_t stream) {
  if (N == 0) return hipSuccess;
  const int64_t Npad = (N + kGramTile - 1) / kGramTile * kGramTile;
  const int KP = (d + 15) / 16 * 16;
  // workspace: hi parts, [lo parts,] norms
  uint16_t *Xb = reinterpret_cast<uint16_t *>(ws);
  uint16_t *Xlo = split ? Xb + (size_t)Npad * KP : nullptr;
  float *nrm = reinterpret_cast<float *>(reinterpret_cast<char *>(ws) +
                                         (size_t)Npad * KP * 2 * (split ? 2 : 1));
  hipLaunchKernelGGL(gram_prologue_kernel, dim3((uint32_t)((Npad + 255) / 256)), dim3(256), 0, stream,
                     X, N, d, ldx, Xb, Xlo, nrm, Npad, KP);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  GramArgs a{X, N, d, ldx, Xb, Xlo, nrm, KP, D};
  const uint64_t nb = (uint64_t)(Npad / kGramTile);
  const uint64_t nb2 = (nb + 1) / 2;
  const uint64_t T = nb2 * (nb2 + 1);  // two work-groups per 256 x 256 tile
  const uint64_t max_blocks = (((uint64_t)1 << 32) - 1) / 512;
  for (uint64_t l0 = 0; l0 < T; l0 += max_blocks) {
    const uint64_t c = T - l0 < max_blocks ? T - l0 : max_blocks;
    if (split)
      launch_gram_tiles<true>(KP, dim3((uint32_t)c), stream, a, (uint32_t)l0);
    else
      launch_gram_tiles<false>(KP, dim3((uint32_t)c), stream, a, (uint32_t)l0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace tdmap
