// Gram-form EDM on the MFMA units (gfx950), packed output.
//
//   D_ij^2 = ||x_i||^2 + ||x_j||^2 - 2 x_i . x_j
//
// A prologue rounds X to BF16 (round to nearest even), pads the features to
// a multiple of 16 with zeros and the points to a multiple of 256, and
// computes the squared norms of the rounded points in FP32.  The products
// are taken by v_mfma_f32_32x32x16_bf16 on 32 x 32 output blocks (BF16
// products are exact in FP32, the sums accumulate in FP32).  The epilogue
// forms G = n_i + n_j - 2 acc and, when G <= theta (n_i + n_j) (theta =
// 1/4: the pair is close relative to its norms, where the Gram form
// cancels), recomputes the distance exactly in FP32 difference form from the
// FP32 points; otherwise it stores sqrt(G).
//
// Two kernels walk the triangle by g(lambda) (Sec. II-A, Eq. (2)) and
// compute every 32 x 32 block with the same instructions in the same order,
// so their outputs are equal bit for bit:
//   - gram_tile_kernel: a work-group of eight waves owns one row half (two
//     128 x 128 tiles side by side) of a 256 x 256 tile;
//   - gram_strip_kernel: a work-group of four waves owns a 32-row strip of
//     a 256 x 256 tile, the strips of a tile row taken strip by strip across
//     the row (the order of the FP32 strips), so that the writes in flight
//     stay in a compact window of the packed output.
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
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kGramTile = 128;  // tile kernel: 128 x 128 per eight waves
constexpr int kGramPad = 256;   // operand rows are padded to this
constexpr float kGramTheta = 0.25f;

__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// The BF16 copy (zero padded) and the squared norms of the represented
// points; with Xlo != nullptr also the low parts.  A thread converts one
// 8-feature chunk of one point and writes it as one 16-byte store, so
// consecutive threads write consecutive chunks.  A work-group takes
// ppb = 256 / cpp whole points (cpp = KP / 8 chunks per point; a point with
// more than 256 chunks takes a work-group alone, its threads stepping by
// 256 chunks); the chunk partial sums of a point are then added in chunk
// order by its first thread.
__global__ __launch_bounds__(256) void gram_prologue_kernel(const float *__restrict__ X, int64_t N, int d,
                                                            int64_t ldx, uint16_t *__restrict__ Xb,
                                                            uint16_t *__restrict__ Xlo,
                                                            float *__restrict__ nrm, int64_t Npad,
                                                            int KP) {
  typedef uint32_t u4 __attribute__((ext_vector_type(4)));
  __shared__ float part[256];
  const int cpp = KP >> 3;
  const int ppb = cpp <= 256 ? 256 / cpp : 1;
  const int t = threadIdx.x;
  const int pl = cpp <= 256 ? t / cpp : 0;  // the thread's point within the work-group
  const int64_t p = (int64_t)blockIdx.x * ppb + pl;
  const bool live = pl < ppb && p < Npad;
  float s = 0.0f;
  if (live) {
    for (int c = cpp <= 256 ? t - pl * cpp : t; c < cpp; c += 256) {
      uint16_t hb[8], lb[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = 8 * c + u;
        const float v = (p < N && k < d) ? X[p * ldx + k] : 0.0f;
        hb[u] = bf16_rne(v);
        float r = bf16_to_f32(hb[u]);
        if (Xlo != nullptr) {
          lb[u] = bf16_rne(v - r);
          r += bf16_to_f32(lb[u]);
        }
        s = __builtin_fmaf(r, r, s);
      }
      u4 h, lo;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        h[e] = (uint32_t)hb[2 * e] | ((uint32_t)hb[2 * e + 1] << 16);
        lo[e] = (uint32_t)lb[2 * e] | ((uint32_t)lb[2 * e + 1] << 16);
      }
      *reinterpret_cast<u4 *>(Xb + p * KP + 8 * c) = h;
      if (Xlo != nullptr) *reinterpret_cast<u4 *>(Xlo + p * KP + 8 * c) = lo;
    }
  }
  part[t] = s;
  __syncthreads();
  if (live && (cpp > 256 ? t == 0 : t == pl * cpp)) {
    float n = 0.0f;
    const int m = cpp < 256 ? cpp : 256;
    for (int c = 0; c < m; ++c) n += part[t + c];
    nrm[p] = n;
  }
}

// FP32 difference form with eight interleaved partial sums combined as a
// tree, which keeps the rounding error of the squared distance near
// (d/8 + 6) units of roundoff.
__device__ __forceinline__ float exact_dist(const float *__restrict__ X, int64_t ldx, int d, int64_t i,
                                         int64_t j) {
  // a point's distance to itself is exactly 0: the diagonal, most of the
  // recomputed cells, needs no loads
  if (i == j) return 0.0f;
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

// The products of NB 32 x 32 blocks sharing one 32-row block of A: block b
// takes the 32 points starting at col[b].  Lane l supplies row (l % 32) of
// a 32-row block and the 8 features [8 (l / 32), 8 (l / 32) + 8) of each
// 16-feature step; B uses the same assignment for its points, so the
// product is x_i . x_j.  Blocks with live[b] false are left at zero.  The
// steps run in increasing feature order and, in split mode, each step adds
// lo.hi', hi.lo', hi.hi' in that order: every kernel that calls this gets
// the same bits for the same block.
template <bool SPLIT, int KPC, int NB>
__device__ __forceinline__ void gram_products(const GramArgs &a, int KP, int64_t row, const int64_t (&col)[NB],
                                              const bool (&live)[NB], f32x16 (&acc)[NB]) {
  const int l = threadIdx.x & 63;
  const int lr = l & 31;
  const int lk = (l >> 5) * 8;
  const uint16_t *__restrict__ Xb = a.Xb;
  const uint16_t *__restrict__ Xl = a.Xlo;
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[b][v] = 0.0f;
  auto kstep = [&](int k) {
    const int64_t ao = (row + lr) * KP + k + lk;
    const bf16x8 av = *reinterpret_cast<const bf16x8 *>(Xb + ao);
    bf16x8 al;
    if constexpr (SPLIT) al = *reinterpret_cast<const bf16x8 *>(Xl + ao);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (live[b]) {
        const int64_t bo = (col[b] + lr) * KP + k + lk;
        const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(Xb + bo);
        if constexpr (SPLIT) {
          const bf16x8 bl = *reinterpret_cast<const bf16x8 *>(Xl + bo);
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bv, acc[b], 0, 0, 0);
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bl, acc[b], 0, 0, 0);
        }
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc[b], 0, 0, 0);
      }
    }
  };
  if constexpr (KPC != 0) {
#pragma unroll
    for (int k = 0; k < KPC; k += 16) kstep(k);
  } else {
    for (int k = 0; k < KP; k += 16) kstep(k);
  }
}

// Accumulator v of a 32 x 32 block holds row (v/4)*8 + (l/32)*4 + v%4 of
// the block and column l % 32.
__device__ __forceinline__ int acc_row(int v, int l) { return (v >> 2) * 8 + (l >> 5) * 4 + (v & 3); }

// The epilogue value of one pair from its accumulator and the two squared
// norms: sqrt(G), or -1 for a pair below the threshold (filled in by the
// exact recompute).
__device__ __forceinline__ float gram_value(float acc, float ni, float nj) {
  const float sn = ni + nj;
  const float G = __builtin_fmaf(-2.0f, acc, sn);
  return G <= kGramTheta * sn ? -1.0f : __builtin_amdgcn_sqrtf(G);
}

// (i(i+1)/2 + c) mod 4 for a row i that is a multiple of 32 plus rr and a
// column c that is a multiple of 128: i(i+1)/2 mod 4 has period 8 in i.
__device__ __forceinline__ int row_shift(int rr) {
  const int m = rr & 7;
  return ((m * (m + 1)) >> 1) & 3;
}

// ---------------------------------------------------------------------------
// tile kernel: eight waves, two 128 x 128 tiles side by side
// ---------------------------------------------------------------------------

// Each wave owns 32 whole rows of the 128 x 128 tile: four 32 x 32
// accumulators (one per 32-column block).  Its distances go, 16 rows at a
// time, through a wave-private LDS slice and are written as packed rows with
// 16-byte stores; no work-group barrier is needed, so the waves run
// independently.
//
// Store layout: a half-wave writes one 128-cell row segment.  Packed row i's
// segment [col0, col0 + 128) starts sh = (D / 4 + i(i+1)/2 + col0) mod 4
// positions past a 16-byte boundary (D / 4: the output's own offset in
// floats); lane h stores the aligned chunk at columns col0 - sh + 4h .. + 3,
// read from LDS at that shift.  The cells of the two partial chunks at the
// ends of each segment (the neighbouring tiles write the rest of those
// chunks) are gathered one row per lane and written with four instructions
// per 16 rows: single-lane stores per row would multiply the store
// instruction count several times over.  Diagonal and edge rows go cell by
// cell.
constexpr int kGramRows = 16;  // rows staged per step and wave

template <bool SPLIT, int KPC, bool COUNT>
__global__ __launch_bounds__(512, SPLIT ? 3 : 4) void gram_tile_kernel(GramArgs a, uint32_t lam0,
                                                                      uint32_t nblk) {
  // Eight waves: the two side-by-side 128 x 128 tiles (I, 2 J2) and
  // (I, 2 J2 + 1) that form one row half, I = 2 I2 + wg mod 2, of the
  // 256 x 256 tile (I2, J2) = g(wg / 2), so each row is written as a 1 KB
  // segment.  Each XCD takes one contiguous range of wg: neighbouring tiles
  // share the partial 16-byte chunks (and lines) at the ends of their row
  // segments, which then combine in one L2, and they share their BF16 row
  // block.
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
  const int64_t N = a.N;
  const int64_t row0 = (int64_t)I * kGramTile;
  const int64_t col0 = (int64_t)J * kGramTile;
  const int64_t rw = row0 + 32 * w;  // this wave's first row
  const bool diag = I == J;
  const int KP = KPC ? KPC : a.KP;
  const int bsh = (int)((reinterpret_cast<uintptr_t>(a.D) >> 2) & 3);
  auto shift = [&](int rr) { return (row_shift(rr) + bsh) & 3; };

  float nr[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) nr[v] = a.nrm[rw + acc_row(v, l)];
  float nc[4];
#pragma unroll
  for (int bj = 0; bj < 4; ++bj) nc[bj] = a.nrm[col0 + bj * 32 + lr];

  // on a diagonal tile, column blocks right of this wave's rows are above
  // the diagonal
  int64_t cols[4];
  bool live[4];
#pragma unroll
  for (int bj = 0; bj < 4; ++bj) {
    cols[bj] = col0 + bj * 32;
    live[bj] = !diag || bj <= w;
  }
  f32x16 acc[4];
  gram_products<SPLIT, KPC, 4>(a, KP, rw, cols, live, acc);

  // stage row rr holds column c at position c + shift(rr); the stored
  // chunks are then aligned 16-byte LDS reads without bank conflicts
  __shared__ __align__(16) float stage[8][kGramRows][kGramTile + 4];
  float(*st)[kGramTile + 4] = stage[wl];
  float *__restrict__ out = a.D;
  const int h = l & 31;
  const bool full_rows = !diag && row0 + kGramTile <= N;
  uint32_t nrec = 0;
#pragma unroll
  for (int vh = 0; vh < 2; ++vh) {
    // v in [8 vh, 8 vh + 8) are the rows 16 vh .. +15
    bool any = false;
#pragma unroll
    for (int bj = 0; bj < 4; ++bj) {
#pragma unroll
      for (int v = 8 * vh; v < 8 * vh + 8; ++v) {
        const int rr = acc_row(v, l) - 16 * vh;
        const float g = gram_value(acc[bj][v], nr[v], nc[bj]);
        any |= g < 0.0f;
        st[rr][bj * 32 + lr + shift(rr)] = g;
      }
    }
    if (any) {
      // rare: the diagonal and near-duplicate pairs, exact FP32 difference
#pragma unroll
      for (int bj = 0; bj < 4; ++bj) {
#pragma unroll
        for (int v = 8 * vh; v < 8 * vh + 8; ++v) {
          const int rr = acc_row(v, l) - 16 * vh;
          const int c = bj * 32 + lr + shift(rr);
          if (st[rr][c] < 0.0f) {
            const int64_t i = rw + 16 * vh + rr;
            const int64_t j = col0 + bj * 32 + lr;
            const bool cell = i < N && j <= i;
            if (COUNT) nrec += cell;
            st[rr][c] = cell ? exact_dist(a.X, a.ldx, a.d, i, j) : 0.0f;
          }
        }
      }
    }
    // the wave reads back its own LDS writes: no barrier needed
    if (full_rows) {
      // Row rw + m (m < 32) starts at T(rw) + col0 + m rw + m(m+1)/2: a
      // uniform base and a 32-bit offset (m rw < 32 N < 2^30 under the
      // 32-bit tile index), with the row's shift shift(m) (rw is a multiple
      // of 32, so T(rw) and m rw add nothing mod 4).
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
        const int sh = shift(r);
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
        const int sh = shift(l);
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
        const int sh = shift(r);
        const int64_t jmax = (diag ? i : N - 1) - col0;
        for (int c = h; c < kGramTile; c += 32)
          if (c <= jmax) __builtin_nontemporal_store(st[r][c + sh], out + first + c);
      }
    }
  }
  if (COUNT && nrec) atomicAdd(a.rec_count, (unsigned long long)nrec);
}

// ---------------------------------------------------------------------------
// strip kernel: eight waves, one 32-row strip of a 256 x 256 tile
// ---------------------------------------------------------------------------

// Tile row I (256 rows) is cut into kStripsPerTile strips of 32 rows and a
// work-group computes one strip of one tile, 32 x 256 cells.  The strips of
// tile row I are numbered u = 0 .. 8 (I + 1) - 1 and taken in column groups
// of kStripGroup tiles: group outer, strip next, tile column inner, so the
// work-groups in flight write a few 32-row bands of the packed triangle (a
// compact window of addresses) while a group's BF16 column points stay in
// L2 across its 8 strips.
//
// Operands: the strip's 32 row points and 256 column points are staged in
// LDS, 128 bytes per point and pass (64 BF16 features, or 32 high and 32
// low parts in split mode; larger feature counts take several passes), by
// 16-byte loads straight into LDS when every pass is full, else by
// coalesced 16-byte loads through registers.  The 16-byte chunk c of staged row r sits at
// chunk c ^ ((r / 2) mod 8) of its row, so that both the coalesced writes
// and the MFMA operand reads (32 rows, one chunk each) hit every LDS bank
// once per 16 lanes.  Wave q computes the 32 x 32 block of columns
// [32 q, 32 q + 32) with the products of gram_products in the same order.
//
// Output: the distances of the strip are staged in LDS (over the operand
// area) and each wave writes whole packed rows q, q + 8, q + 16, q + 24:
// lane l owns columns l + 64 c and every 4-byte store instruction writes 256
// contiguous bytes.  The LDS footprint (37 KB) leaves four work-groups per
// CU.
constexpr int kStripRows = 32;
constexpr int kStripsPerTile = 256 / kStripRows;
constexpr int kStripWaves = 8;
constexpr int kStripOpRows = kStripRows + 256;  // staged operand rows
constexpr int kStripOpBytes = 128;              // bytes per staged row and pass
constexpr int kStripPitch = 260;                // floats per staged output row
constexpr uint32_t kStripGroup = 8;
static_assert(kStripRows * kStripPitch * 4 <= kStripOpRows * kStripOpBytes,
              "the staged output overlays the operand area");

__device__ __forceinline__ void strip_order(uint32_t w, uint32_t group, uint32_t &I, uint32_t &k,
                                            uint32_t &J) {
  uint32_t Jt;
  g_lambda(w / kStripsPerTile, I, Jt);
  // u: this work-group's place among the 8 (I + 1) strips of tile row I
  const uint32_t u = kStripsPerTile * Jt + w % kStripsPerTile;
  const uint32_t ntile = I + 1;
  const uint32_t gs = group < ntile ? group : ntile;
  const uint32_t nfull = ntile / gs;
  const uint32_t span = gs * kStripsPerTile;
  if (u < nfull * span) {
    const uint32_t g = u / span, r = u - g * span;
    k = r / gs;
    J = g * gs + (r - k * gs);
  } else {
    const uint32_t rem = ntile - nfull * gs;  // the last, narrower group
    const uint32_t r = u - nfull * span;
    k = r / rem;
    J = nfull * gs + (r - k * rem);
  }
}

// Byte offset of 16-byte chunk c of staged operand row r.
__device__ __forceinline__ int strip_chunk(int r, int c) {
  return r * kStripOpBytes + ((c ^ ((r >> 1) & 7)) << 4);
}

template <bool SPLIT, int KPC, bool COUNT>
__global__ __launch_bounds__(kStripWaves * 64) void gram_strip_kernel(GramArgs a, uint32_t w0,
                                                                      uint32_t nblk) {
  typedef uint32_t u4 __attribute__((ext_vector_type(4)));
  __shared__ __align__(16) unsigned char ops[kStripOpRows * kStripOpBytes];
  __shared__ float nrow[kStripRows];
  float *st = reinterpret_cast<float *>(ops);  // after the products
  const uint32_t w = w0 + xcd_contiguous(blockIdx.x, nblk);
  uint32_t I, k, J;
  strip_order(w, kStripGroup, I, k, J);
  const int64_t N = a.N;
  const int64_t r0 = (int64_t)I * 256 + (int64_t)k * kStripRows;
  if (r0 >= N) return;  // a strip past the last point (uniform)
  const int64_t c0 = (int64_t)J * 256;
  const bool diag = I == J;
  const int t = threadIdx.x;
  const int q = __builtin_amdgcn_readfirstlane(t >> 6);
  const int l = t & 63;
  const int lr = l & 31;
  const int hl = l >> 5;
  const int KP = KPC ? KPC : a.KP;
  if (t < kStripRows) nrow[t] = a.nrm[r0 + t];
  const float ncol = a.nrm[c0 + 32 * q + lr];

  f32x16 acc;
#pragma unroll
  for (int v = 0; v < 16; ++v) acc[v] = 0.0f;
  // features per pass: 64, or 32 high + 32 low parts
  constexpr int kFpp = SPLIT ? 32 : 64;
  constexpr int kMaxLoads = (kStripOpRows * kStripOpBytes / 16 + kStripWaves * 64 - 1) / (kStripWaves * 64);
  for (int k0 = 0; k0 < KP; k0 += kFpp) {
    const int nf = KP - k0 < kFpp ? KP - k0 : kFpp;  // a multiple of 16
    if constexpr (KPC != 0 && KPC % kFpp == 0) {
      // every pass full (8 chunks per staged row): one wave instruction
      // fills 8 staged rows, 1 KB of LDS, straight from global memory
      // (gfx950 global-to-LDS loads, no register round trip); lane l fills
      // slot l % 8 of row 8 b + l / 8 with the chunk the swizzle puts there
      const int lrow = l >> 3, slot = l & 7;
      for (int b = q; b < kStripOpRows / 8; b += kStripWaves) {
        const int row = 8 * b + lrow;
        const int cl = slot ^ ((row >> 1) & 7);
        const int part = SPLIT ? (cl >> 2) : 0;
        const int c = SPLIT ? (cl & 3) : cl;
        const int64_t g = row < kStripRows ? r0 + row : c0 + (row - kStripRows);
        const uint16_t *src = (SPLIT && part) ? a.Xlo : a.Xb;
        __builtin_amdgcn_global_load_lds(
            (const __attribute__((address_space(1))) void *)(src + g * KP + k0 + 8 * c),
            (__attribute__((address_space(3))) void *)(ops + b * 1024), 16, 0, 0);
      }
      __builtin_amdgcn_s_waitcnt(0);  // the wave's staged rows have landed
    } else {
      const int cpr = nf >> 3;  // chunks per row and part
      const int per_part = kStripOpRows * cpr;
      const int total = per_part * (SPLIT ? 2 : 1);
      u4 v[kMaxLoads];
#pragma unroll
      for (int m = 0; m < kMaxLoads; ++m) {
        const int e = t + kStripWaves * 64 * m;
        if (e < total) {
          const int part = SPLIT ? (e >= per_part) : 0;
          const int e2 = e - part * per_part;
          const int row = e2 / cpr, c = e2 - row * cpr;
          const int64_t g = row < kStripRows ? r0 + row : c0 + (row - kStripRows);
          const uint16_t *src = (SPLIT && part) ? a.Xlo : a.Xb;
          v[m] = *reinterpret_cast<const u4 *>(src + g * KP + k0 + 8 * c);
        }
      }
#pragma unroll
      for (int m = 0; m < kMaxLoads; ++m) {
        const int e = t + kStripWaves * 64 * m;
        if (e < total) {
          const int part = SPLIT ? (e >= per_part) : 0;
          const int e2 = e - part * per_part;
          const int row = e2 / cpr, c = e2 - row * cpr;
          *reinterpret_cast<u4 *>(ops + strip_chunk(row, c + 4 * part)) = v[m];
        }
      }
    }
    __syncthreads();
    // k-steps of 16 features: lane (lr, hl) reads chunk 2 ks + hl of its
    // row (split: the low parts are chunks 4 + 2 ks + hl)
    const int ra = lr, rb = kStripRows + 32 * q + lr;
    for (int ks = 0; ks < (nf >> 4); ++ks) {
      const bf16x8 av = *reinterpret_cast<const bf16x8 *>(ops + strip_chunk(ra, 2 * ks + hl));
      const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(ops + strip_chunk(rb, 2 * ks + hl));
      if constexpr (SPLIT) {
        const bf16x8 al = *reinterpret_cast<const bf16x8 *>(ops + strip_chunk(ra, 4 + 2 * ks + hl));
        const bf16x8 bl = *reinterpret_cast<const bf16x8 *>(ops + strip_chunk(rb, 4 + 2 * ks + hl));
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bv, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bl, acc, 0, 0, 0);
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
    }
    __syncthreads();  // the operands are read: the next pass or the output may overwrite them
  }

  // epilogue: the wave's 32 x 32 block into the staged output; pairs below
  // the threshold are marked and recomputed afterwards (rare: the diagonal,
  // which needs no loads, and near-duplicate pairs)
  const int col = 32 * q + lr;
  uint32_t rflag = 0;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int rr = acc_row(v, l);
    const float e = acc[v];  // (copied out: a bit cast of a vector element is avoided)
    const float g = gram_value(e, nrow[rr], ncol);
    rflag |= (uint32_t)(g < 0.0f) << v;
    st[rr * kStripPitch + col] = g < 0.0f ? 0.0f : g;
  }
  uint32_t nrec = 0;
  if (rflag != 0) {
#pragma unroll 1
    for (int v = 0; v < 16; ++v) {
      if ((rflag >> v) & 1u) {
        const int rr = acc_row(v, l);
        const int64_t i = r0 + rr;
        const int64_t j = c0 + col;
        const bool cell = i < N && j <= i;
        if (COUNT) nrec += cell;
        st[rr * kStripPitch + col] = cell ? exact_dist(a.X, a.ldx, a.d, i, j) : 0.0f;
      }
    }
  }
  if (COUNT && nrec) atomicAdd(a.rec_count, (unsigned long long)nrec);
  __syncthreads();

  // Strip row r starts at T(r0 + r) + c0 = T(r0) + c0 + r r0 + r(r+1)/2: a
  // uniform 64-bit base and a 32-bit offset (r r0 < 32 N).
  float *__restrict__ outb = a.D + tri64((uint64_t)r0) + (uint64_t)c0;
  const uint32_t r0u = (uint32_t)r0;
  auto row_off = [&](uint32_t r) { return r * r0u + ((r * (r + 1)) >> 1); };
  if (!diag && r0 + kStripRows <= N) {
#pragma unroll
    for (int m = 0; m < kStripRows / kStripWaves; ++m) {
      const int r = q + kStripWaves * m;
      float *o = outb + row_off(r);
#pragma unroll
      for (int c = 0; c < 4; ++c) o[l + 64 * c] = st[r * kStripPitch + l + 64 * c];
    }
  } else {
    // diagonal or edge strip: rows below N, cells with j <= i
    for (int m = 0; m < kStripRows / kStripWaves; ++m) {
      const int r = q + kStripWaves * m;
      const int64_t i = r0 + r;
      if (i >= N) break;
      const int64_t jmax = diag ? i - c0 : 255;
      float *o = outb + row_off(r);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int cc = l + 64 * c;
        if (cc <= jmax) o[cc] = st[r * kStripPitch + cc];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

template <bool SPLIT, bool COUNT>
static void launch_gram_tiles(int KP, dim3 grid, hipStream_t stream, const GramArgs &a, uint32_t l0) {
  const dim3 block(512);
  switch (KP) {
    case 16:
      hipLaunchKernelGGL((gram_tile_kernel<SPLIT, 16, COUNT>), grid, block, 0, stream, a, l0, grid.x);
      break;
    case 32:
      hipLaunchKernelGGL((gram_tile_kernel<SPLIT, 32, COUNT>), grid, block, 0, stream, a, l0, grid.x);
      break;
    case 64:
      hipLaunchKernelGGL((gram_tile_kernel<SPLIT, 64, COUNT>), grid, block, 0, stream, a, l0, grid.x);
      break;
    case 128:
      hipLaunchKernelGGL((gram_tile_kernel<SPLIT, 128, COUNT>), grid, block, 0, stream, a, l0, grid.x);
      break;
    default:
      hipLaunchKernelGGL((gram_tile_kernel<SPLIT, 0, COUNT>), grid, block, 0, stream, a, l0, grid.x);
  }
}

template <bool SPLIT, bool COUNT>
static void launch_gram_strips(int KP, dim3 grid, hipStream_t stream, const GramArgs &a, uint32_t w0) {
  const dim3 block(kStripWaves * 64);
  switch (KP) {
    case 16:
      hipLaunchKernelGGL((gram_strip_kernel<SPLIT, 16, COUNT>), grid, block, 0, stream, a, w0, grid.x);
      break;
    case 32:
      hipLaunchKernelGGL((gram_strip_kernel<SPLIT, 32, COUNT>), grid, block, 0, stream, a, w0, grid.x);
      break;
    case 64:
      hipLaunchKernelGGL((gram_strip_kernel<SPLIT, 64, COUNT>), grid, block, 0, stream, a, w0, grid.x);
      break;
    case 128:
      hipLaunchKernelGGL((gram_strip_kernel<SPLIT, 128, COUNT>), grid, block, 0, stream, a, w0, grid.x);
      break;
    default:
      hipLaunchKernelGGL((gram_strip_kernel<SPLIT, 0, COUNT>), grid, block, 0, stream, a, w0, grid.x);
  }
}

static int64_t gram_npad(int64_t N) { return (N + kGramPad - 1) / kGramPad * kGramPad; }

size_t gram_workspace_bytes(int64_t N, int d, bool split) {
  const int64_t KP = (d + 15) / 16 * 16;
  const int64_t Npad = gram_npad(N);
  return (size_t)Npad * (size_t)KP * 2 * (split ? 2 : 1) + (size_t)Npad * 4;
}

bool gram_supported(int64_t N, int ts) {
  if (ts == 128) {
    const uint64_t nb2 = (uint64_t)((N + 255) / 256);
    return nb2 * (nb2 + 1) <= 0xffffffffull;
  }
  if (ts == 256) {
    const uint64_t nb = (uint64_t)((N + 255) / 256);
    return (uint64_t)kStripsPerTile * (nb * (nb + 1) / 2) <= 0xffffffffull;
  }
  return false;
}

template <bool COUNT>
static hipError_t launch_gram_t(const float *X, int64_t N, int d, int64_t ldx, float *D, void *ws,
                                bool split, int ts, unsigned long long *count, hipStream_t stream,
                                uint32_t shard = 0, uint32_t nshards = 1) {
  if (N == 0) return hipSuccess;
  const int64_t Npad = gram_npad(N);
  const int KP = (d + 15) / 16 * 16;
  // workspace: hi parts, [lo parts,] norms
  uint16_t *Xb = reinterpret_cast<uint16_t *>(ws);
  uint16_t *Xlo = split ? Xb + (size_t)Npad * KP : nullptr;
  float *nrm = reinterpret_cast<float *>(reinterpret_cast<char *>(ws) +
                                         (size_t)Npad * KP * 2 * (split ? 2 : 1));
  const int cpp = KP / 8;
  const int64_t ppb = cpp <= 256 ? 256 / cpp : 1;
  hipLaunchKernelGGL(gram_prologue_kernel, dim3((uint32_t)((Npad + ppb - 1) / ppb)), dim3(256), 0, stream,
                     X, N, d, ldx, Xb, Xlo, nrm, Npad, KP);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  GramArgs a{X, N, d, ldx, Xb, Xlo, nrm, KP, D, count};
  if (ts == 256) {
    const uint64_t nb = (uint64_t)(Npad / 256);
    const uint64_t W = (uint64_t)kStripsPerTile * (nb * (nb + 1) / 2);
    uint64_t lo, hi;
    shard_range(W, shard, nshards, lo, hi);
    const uint64_t max_blocks = (((uint64_t)1 << 32) - 1) / (kStripWaves * 64);
    for (uint64_t w0 = lo; w0 < hi; w0 += max_blocks) {
      const uint64_t c = hi - w0 < max_blocks ? hi - w0 : max_blocks;
      if (split)
        launch_gram_strips<true, COUNT>(KP, dim3((uint32_t)c), stream, a, (uint32_t)w0);
      else
        launch_gram_strips<false, COUNT>(KP, dim3((uint32_t)c), stream, a, (uint32_t)w0);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
  }
  if (ts != 128) return hipErrorInvalidValue;
  const uint64_t nb2 = (uint64_t)(Npad / 256);
  const uint64_t T = nb2 * (nb2 + 1);  // two work-groups per 256 x 256 tile
  uint64_t lo, hi;
  shard_range(T, shard, nshards, lo, hi);
  const uint64_t max_blocks = (((uint64_t)1 << 32) - 1) / 512;
  for (uint64_t l0 = lo; l0 < hi; l0 += max_blocks) {
    const uint64_t c = hi - l0 < max_blocks ? hi - l0 : max_blocks;
    if (split)
      launch_gram_tiles<true, COUNT>(KP, dim3((uint32_t)c), stream, a, (uint32_t)l0);
    else
      launch_gram_tiles<false, COUNT>(KP, dim3((uint32_t)c), stream, a, (uint32_t)l0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_gram(const float *X, int64_t N, int d, int64_t ldx, float *D, void *ws, bool split,
                       int ts, hipStream_t stream, uint32_t shard, uint32_t nshards) {
  return launch_gram_t<false>(X, N, d, ldx, D, ws, split, ts, nullptr, stream, shard, nshards);
}

hipError_t launch_gram_count(const float *X, int64_t N, int d, int64_t ldx, float *D, void *ws,
                             bool split, int ts, unsigned long long *count, hipStream_t stream) {
  hipError_t e = launch_fill(reinterpret_cast<float *>(count), 2, 0.0f, stream);
  if (e != hipSuccess) return e;
  return launch_gram_t<true>(X, N, d, ldx, D, ws, split, ts, count, stream);
}

}  // namespace tdmap
