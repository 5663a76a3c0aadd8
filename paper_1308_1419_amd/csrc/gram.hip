// Gram-form EDM on the MFMA units (gfx950), packed output.
//
//   D_ij^2 = ||x_i||^2 + ||x_j||^2 - 2 x_i . x_j
//
// A prologue rounds X to BF16 (round to nearest even), pads the features to
// a multiple of 16 with zeros and the points to a multiple of 128, and
// computes the squared norms of the rounded points in FP32.  The main
// kernel walks the 128 x 128 tiles of the triangle by g(lambda) (Sec. II-A,
// Eq. (2)); four waves each own a 64 x 64 quadrant computed by 2 x 2
// v_mfma_f32_32x32x16_bf16 accumulators (BF16 products are exact in FP32,
// the sums accumulate in FP32).  The epilogue forms
// G = n_i + n_j - 2 acc and, when G <= theta (n_i + n_j) (theta = 1/4:
// the pair is close relative to its norms, where the Gram form cancels),
// recomputes the distance exactly in FP32 difference form from the FP32
// points; otherwise it stores sqrt(G).
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

// One thread per padded point: BF16 copy (zero padded) and its squared norm.
__global__ __launch_bounds__(256) void gram_prologue_kernel(const float *__restrict__ X, int64_t N, int d,
                                                            int64_t ldx, uint16_t *__restrict__ Xb,
                                                            float *__restrict__ nrm, int64_t Npad,
                                                            int KP) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= Npad) return;
  float s = 0.0f;
  for (int k = 0; k < KP; ++k) {
    const float v = (p < N && k < d) ? X[p * ldx + k] : 0.0f;
    const uint16_t b = bf16_rne(v);
    Xb[p * KP + k] = b;
    const float r = bf16_to_f32(b);
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

// Writes the 128 x 128 tile held in LDS to the packed output.  Each wave
// owns 32 tile rows and writes two per instruction (one per half-wave).
// Packed row i's segment [col0, col0 + 128) starts sh = (i(i+1)/2 + col0)
// mod 4 positions past a 16-byte boundary; half-wave lane h stores the
// aligned chunk at columns col0 - sh + 4h .. + 3, read back from LDS at that
// shift.  Lane 0 of each half-wave writes the 4 - sh head cells and the sh
// tail cells one by one (the neighbouring tiles write the rest of those two
// chunks).  Diagonal and edge rows go cell by cell.
__device__ __forceinline__ void store_tile_rows(const float (*tileD)[kGramTile + 4], int64_t row0,
                                                int64_t col0, int64_t N, bool diag,
                                                float *__restrict__ out) {
  const int w = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  const int h = l & 31;
  const bool full_rows = !diag && row0 + kGramTile <= N;
  for (int p = 0; p < 16; ++p) {
    const int r = w * 32 + 2 * p + (l >> 5);
    const int64_t i = row0 + r;
    if (i >= N) continue;
    const uint64_t first = tri64((uint64_t)i) + (uint64_t)col0;
    if (full_rows) {
      const int sh = (int)(first & 3);
      const uint64_t A0 = first - (uint64_t)sh;
      if (h > 0 || sh == 0) {
        const int c = 4 * h - sh;
        f4 v = {tileD[r][c], tileD[r][c + 1], tileD[r][c + 2], tileD[r][c + 3]};
        __builtin_nontemporal_store(v, reinterpret_cast<f4 *>(out + A0 + 4 * h));
      } else {
        for (int q = sh; q < 4; ++q) __builtin_nontemporal_store(tileD[r][q - sh], out + A0 + q);
        for (int q = 0; q < sh; ++q)
          __builtin_nontemporal_store(tileD[r][kGramTile - sh + q], out + A0 + kGramTile + q);
      }
    } else {
      // last valid column of this row inside the tile
      const int64_t jmax = (diag ? i : N - 1) - col0;
      for (int c = h; c < kGramTile; c += 32)
        if (c <= jmax) __builtin_nontemporal_store(tileD[r][c], out + first + c);
    }
  }
}

__global__ __launch_bounds__(256) void gram_tile_kernel(GramArgs a, uint32_t lam0) {
  uint32_t I, J;
  g_lambda(lam0 + blockIdx.x, I, J);
  const int t = threadIdx.x;
  const int w = t >> 6;
  const int l = t & 63;
  const int wr = w >> 1;
  const int wc = w & 1;
  const int64_t r0 = (int64_t)I * kGramTile + wr * 64;
  const int64_t c0 = (int64_t)J * kGramTile + wc * 64;
  const int KP = a.KP;
  const uint16_t *__restrict__ Xb = a.Xb;
  // the upper-right quadrant of a diagonal tile lies above the diagonal:
  // its wave skips the products but still stores its share of the rows
  const bool above = I == J && wr < wc;

  f32x16 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[bi][bj][v] = 0.0f;

  // lane l supplies row (l % 32) of each 32-row block and the 8 features
  // [8 (l / 32), 8 (l / 32) + 8) of each 16-feature step; B uses the same
  // assignment for its points, so the product is x_i . x_j.
  const int lr = l & 31;
  const int lk = (l >> 5) * 8;
  for (int k = 0; k < (above ? 0 : KP); k += 16) {
    bf16x8 av[2], bv[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      av[b] = *reinterpret_cast<const bf16x8 *>(Xb + (r0 + b * 32 + lr) * KP + k + lk);
      bv[b] = *reinterpret_cast<const bf16x8 *>(Xb + (c0 + b * 32 + lr) * KP + k + lk);
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj)
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[bi], bv[bj], acc[bi][bj], 0, 0, 0);
  }

  // accumulator v of a 32 x 32 block holds row (v/4)*8 + (l/32)*4 + v%4 and
  // column l % 32.  The norms of every row and column this lane touches are
  // loaded up front (the padded norm array covers every tile row).
  const int64_t N = a.N;
  float nr[2][16];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int v = 0; v < 16; ++v)
      nr[bi][v] = a.nrm[r0 + bi * 32 + (v >> 2) * 8 + (l >> 5) * 4 + (v & 3)];
  float nc[2];
#pragma unroll
  for (int bj = 0; bj < 2; ++bj) nc[bj] = a.nrm[c0 + bj * 32 + lr];

  // distances go to an LDS copy of the tile first: sqrt(G) for every pair
  // above the recompute threshold, then (rare: the diagonal and
  // near-duplicate pairs) the exact FP32 difference form for the others
  __shared__ float tileD[kGramTile][kGramTile + 4];
  const int tr0 = wr * 64;
  const int tc0 = wc * 64;
  uint64_t need = 0;
#pragma unroll
  for (int bj = 0; bj < 2; ++bj) {
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
#pragma unroll
      for (int v = 0; v < 16 && !above; ++v) {
        const int rr = bi * 32 + (v >> 2) * 8 + (l >> 5) * 4 + (v & 3);
        const float sn = nr[bi][v] + nc[bj];
        const float G = __builtin_fmaf(-2.0f, acc[bi][bj][v], sn);
        if (G <= kGramTheta * sn) need |= (uint64_t)1 << ((bj * 2 + bi) * 16 + v);
        tileD[tr0 + rr][tc0 + bj * 32 + lr] = __builtin_amdgcn_sqrtf(__builtin_fmaxf(G, 0.0f));
      }
    }
  }
  while (need) {
    const int b = __builtin_ctzll(need);
    need &= need - 1;
    const int bj = b >> 5;
    const int bi = (b >> 4) & 1;
    const int v = b & 15;
    const int rr = bi * 32 + (v >> 2) * 8 + (l >> 5) * 4 + (v & 3);
    const int64_t i = r0 + rr;
    const int64_t j = c0 + bj * 32 + lr;
    if (i < N && j <= i) tileD[tr0 + rr][tc0 + bj * 32 + lr] = exact_dist(a.X, a.ldx, a.d, i, j);
  }
  __syncthreads();
  store_tile_rows(tileD, (int64_t)I * kGramTile, (int64_t)J * kGramTile, N, I == J, a.D);
}

size_t gram_workspace_bytes(int64_t N, int d) {
  const int64_t Npad = (N + kGramTile - 1) / kGramTile * kGramTile;
  const int64_t KP = (d + 15) / 16 * 16;
  return (size_t)Npad * (size_t)KP * 2 + (size_t)Npad * 4;
}

hipError_t launch_gram(const float *X, int64_t N, int d, int64_t ldx, float *D, void *ws,
                       hipStream_t stream) {
  if (N == 0) return hipSuccess;
  const int64_t Npad = (N + kGramTile - 1) / kGramTile * kGramTile;
  const int KP = (d + 15) / 16 * 16;
  uint16_t *Xb = reinterpret_cast<uint16_t *>(ws);
  float *nrm = reinterpret_cast<float *>(reinterpret_cast<char *>(ws) + (size_t)Npad * KP * 2);
  hipLaunchKernelGGL(gram_prologue_kernel, dim3((uint32_t)((Npad + 255) / 256)), dim3(256), 0, stream,
                     X, N, d, ldx, Xb, nrm, Npad, KP);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  GramArgs a{X, N, d, ldx, Xb, nrm, KP, D};
  const uint64_t nb = (uint64_t)(Npad / kGramTile);
  const uint64_t T = nb * (nb + 1) / 2;
  const uint64_t max_blocks = (((uint64_t)1 << 32) - 1) / 256;
  for (uint64_t l0 = 0; l0 < T; l0 += max_blocks) {
    const uint64_t c = T - l0 < max_blocks ? T - l0 : max_blocks;
    hipLaunchKernelGGL(gram_tile_kernel, dim3((uint32_t)c), dim3(256), 0, stream, a, (uint32_t)l0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace tdmap
