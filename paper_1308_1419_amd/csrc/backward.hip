// Gradient through the lower-triangular EDM, over the same g(lambda) tiles
// as the forward map.
//
// For a cell (i, j), j < i, with g = dL/dD_ij and diff = x_i - x_j:
//   c = g / ||diff|| = g * rsq(||diff||^2)   (0 when ||diff|| = 0)
//   dX_i += c * diff,   dX_j -= c * diff.
// A 256-thread work-group owns a TS x TS tile (I, J) = g(lambda).  Column
// sums stay in registers; row sums are reduced across lanes with DPP moves.
// Per-tile partial sums then either go to a workspace (deterministic: a
// second kernel adds them in a fixed order) or are added to dX with
// atomics.
//
// Stress mode (the fused loss and gradient): the tile reads the targets
// delta_ij instead of dL/dD_ij, forms D_ij itself and uses
// dL/dD_ij = 2 (D_ij - delta_ij), and also sums the loss
// sum_{j<i} (D_ij - delta_ij)^2 per tile (to the workspace, or atomically).
#include "device.h"
#include "kernels.h"

namespace tdmap {

typedef float f4 __attribute__((ext_vector_type(4)));

// Sum over the 64 lanes of a wave with DPP lane moves (plain VALU adds, no
// LDS crossbar traffic): swaps within quads, mirrors within 8 and 16 lanes
// leave every lane of a 16-lane row holding the row's sum; two row
// broadcasts then accumulate rows 0..3 into row 3.  The total is valid in
// lane 63 (kSumLane).
constexpr int kSumLane = 63;

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_move(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xF, false));
}

// A lane move inside 16-lane rows whose every source lane exists (quad
// permutes, the row mirrors): with bound control set, the move folds into
// the add that consumes it.
template <int CTRL>
__device__ __forceinline__ float dpp_row_move(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}

__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_move<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x141, 0xF>(v);  // row_half_mirror
  v += dpp_move<0x140, 0xF>(v);  // row_mirror
  v += dpp_move<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  return v;
}

constexpr uint32_t kBwdChunk = 4;  // consecutive tiles per XCD turn

// Lanes per row group in the tiles (16 measured faster than 8: 8 halves the
// reduction moves per cell but needed three waves per SIMD's worth of
// registers at TS = 128).
constexpr int kBwdLanesPerRow = 16;

// Sum over the LPR lanes of a row group (LPR = 8 or 16 consecutive lanes);
// every lane of the group receives the sum.
template <int LPR>
__device__ __forceinline__ float group_sum(float v) {
  v += dpp_row_move<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_row_move<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_row_move<0x141>(v);  // row_half_mirror
  if constexpr (LPR == 16) v += dpp_row_move<0x140>(v);  // row_mirror
  return v;
}

// Sum over the four 16-lane rows of a wave at each position in the row:
// every lane l receives the sum over lanes l mod 16 + 16 r, r < 4.  The
// gfx950 lane swaps pair row 0 with 1 and 2 with 3 (16), then the wave's
// halves (32), in registers (no LDS round trip as with a lane shuffle).
__device__ __forceinline__ float cross_row_sum(float v) {
  const uint32_t u = __builtin_bit_cast(uint32_t, v);
  const auto a = __builtin_amdgcn_permlane16_swap(u, u, false, false);
  const uint32_t a0 = a[0], a1 = a[1];  // copied out before the bit casts
  const float s = __builtin_bit_cast(float, a0) + __builtin_bit_cast(float, a1);
  const uint32_t w = __builtin_bit_cast(uint32_t, s);
  const auto b = __builtin_amdgcn_permlane32_swap(w, w, false, false);
  const uint32_t b0 = b[0], b1 = b[1];
  return __builtin_bit_cast(float, b0) + __builtin_bit_cast(float, b1);
}

// Element distance in dD from row i to row i + p (same column) in the
// layout's row-major order; p = SR gives the next step's first row.
template <int LAYOUT>
__device__ __forceinline__ uint64_t row_gap(uint64_t i, int p, int64_t ldd) {
  if constexpr (LAYOUT == kLayoutFull) return (uint64_t)p * (uint64_t)ldd;
  else if constexpr (LAYOUT == kLayoutPacked) return (uint64_t)p * i + (uint64_t)(p * (p + 1) / 2);
  else return (uint64_t)p * i + (uint64_t)(p * (p - 1) / 2);
}

// Lane layout of a wave's H x H tile quarter: LPR lanes per row group,
// RG = 64 / LPR row groups; lane l = LPR rg + cg owns columns cg + LPR q
// (q < Q = H / LPR) and, in step s of SR rows, rows rq0 + SR s + P rg + p
// (p < P = SR / RG).  SR = 8 for TS = 128 and 256 (a lane's 2 x Q block
// per step keeps TS = 256 at 150 VGPRs, three waves per SIMD; 16-row steps
// took 216, two waves, and were 4 % slower), 16 for TS = 64.
template <int TS, int LPR>
struct BwdLayout {
  static constexpr int H = TS / 2;
  static constexpr int RG = 64 / LPR;
  static constexpr int Q = H / LPR;
  static constexpr int SR = TS >= 128 ? 8 : 16;  // rows per step
  static constexpr int P = SR / RG;
  static constexpr int STEPS = H / SR;
};

// STRESS: the loaded values are the targets delta_ij rather than dL/dD_ij;
// each cell then takes e = D_ij - delta_ij, adds e^2 to lacc and uses
// dL/dD_ij = 2 e (cells outside the strict lower triangle contribute
// nothing to either).
// `stage` stores the tile's points (loaded into registers with coalesced
// loads) to LDS and, after the barrier, `read_cols` takes the lane's column
// points from there.  In the gradient passes (not STRESS) the first step's
// dD loads are issued before `stage`, so a tile's start waits for one round
// of loads instead of two; the fused pass, short of registers at TS = 256,
// loads each step after the barrier.
template <int TS, int LPR, int D, int LAYOUT, bool INTERIOR, bool STRESS, typename Stage,
          typename ReadCols>
__device__ __forceinline__ void bwd_quarter_steps(Stage stage, ReadCols read_cols,
    const BwdArgs &a, const float *xs, float *rowp, const float (&xj)[BwdLayout<TS, LPR>::Q][D],
    const bool (&jok)[BwdLayout<TS, LPR>::Q], float (&cacc)[BwdLayout<TS, LPR>::Q][D],
    int64_t row0, int64_t cbase, int rq0, int rg, int cg, bool diag, float &lacc) {
  using L = BwdLayout<TS, LPR>;
  constexpr int Q = L::Q;
  constexpr int P = L::P;
  const int64_t N = a.N;
  // row p = 0 of the current step and its element index in dD; the rows
  // below it follow by row_gap (no multiply by the row per load)
  int64_t ist = row0 + rq0 + P * rg;
  uint64_t bst = out_index<LAYOUT>((uint64_t)ist, (uint64_t)cbase, a.ldd);
  auto load_row = [&](int p, float (&g)[Q], bool (&okm)[Q]) {
    const int64_t i = ist + p;
    const float *rp = a.dD + bst + row_gap<LAYOUT>((uint64_t)ist, p, a.ldd);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if constexpr (INTERIOR) {
        g[q] = rp[LPR * q];
        okm[q] = true;
      } else {
        const int64_t j = cbase + LPR * q;
        const bool ok = i < N && jok[q] && (!diag || j < i);
        g[q] = ok ? rp[LPR * q] : 0.0f;
        okm[q] = ok;
      }
    }
  };
  constexpr bool EARLY = !STRESS;  // the first step's loads before the barrier
  float g[P][Q];
  bool okm[P][Q];
  if constexpr (EARLY) {
#pragma unroll
    for (int p = 0; p < P; ++p) load_row(p, g[p], okm[p]);
    bst += row_gap<LAYOUT>((uint64_t)ist, L::SR, a.ldd);
    ist += L::SR;
  }
  stage();
  __syncthreads();
  read_cols();
#pragma unroll 1
  for (int s = 0; s < L::STEPS; ++s) {
    if (!EARLY || s > 0) {
#pragma unroll
      for (int p = 0; p < P; ++p) load_row(p, g[p], okm[p]);
      bst += row_gap<LAYOUT>((uint64_t)ist, L::SR, a.ldd);
      ist += L::SR;
    }
    const int rl = rq0 + L::SR * s + P * rg;  // tile-local row of p = 0
#pragma unroll
    for (int p = 0; p < P; ++p) {
      float xi[D], rs[D];
#pragma unroll
      for (int k = 0; k < D; ++k) {
        xi[k] = xs[(rl + p) * D + k];
        rs[k] = 0.0f;
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        float diff[D];
        float s2 = 0.0f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
          diff[k] = xi[k] - xj[q][k];
          s2 = __builtin_fmaf(diff[k], diff[k], s2);
        }
        float cc;
        if constexpr (STRESS) {
          // D = s2 rsq(s2) (0 at coincident points, where the gradient
          // term is 0 as well)
          const float r = s2 > 0.0f ? __builtin_amdgcn_rsqf(s2) : 0.0f;
          const float e = s2 * r - g[p][q];
          const bool ok = INTERIOR || okm[p][q];
          lacc = ok ? __builtin_fmaf(e, e, lacc) : lacc;
          // the factor 2 of dL/dD = 2 e is applied to the sums (exact)
          cc = ok ? e * r : 0.0f;
        } else {
          // g is 0 for every cell outside the strict lower triangle; the
          // select is on the reciprocal (0 at coincident points), so the
          // load of g is not tied to a branch
          const float r = s2 > 0.0f ? __builtin_amdgcn_rsqf(s2) : 0.0f;
          cc = g[p][q] * r;
        }
#pragma unroll
        for (int k = 0; k < D; ++k) {
          rs[k] = __builtin_fmaf(cc, diff[k], rs[k]);
          cacc[q][k] = __builtin_fmaf(-cc, diff[k], cacc[q][k]);
        }
      }
#pragma unroll
      for (int k = 0; k < D; ++k) {
        rs[k] = group_sum<LPR>(rs[k]);
        // keep the last add beside its lane move (it folds into one DPP
        // add) rather than inside the one-lane store below
        asm volatile("" : "+v"(rs[k]));
      }
      if (cg == LPR - 1) {
#pragma unroll
        for (int k = 0; k < D; ++k) rowp[(rl + p) * D + k] = STRESS ? 2.0f * rs[k] : rs[k];
      }
    }
  }
}

// TS = 64, 128 or 256.  The four waves split the tile into 2 x 2 quarters
// of H = TS/2 rows and columns; wave w takes row half w >> 1 and column
// half w & 1.  Inside a wave, lane l = LPR rg + cg owns columns cg + LPR q
// (q < Q = H/LPR) of its column half, so one load instruction reads LPR
// consecutive cells of each of RG = 64/LPR rows, and rows P rg .. P rg + P - 1
// (P = SR/RG) of each step of SR rows.  A lane thus works on a P x Q block
// of cells per step: the row sums of its rows are reduced over only the LPR
// lanes of its row group (full-rate DPP moves, no broadcasts), and the
// column sums stay in registers for the whole tile and are reduced over the
// row groups once at the end.  A step's P x Q loads are issued together
// before its arithmetic; the next step's are not prefetched (prefetching,
// also into the registers each row frees, was slower: it costs waves per
// SIMD and the tiles are not waiting on HBM latency alone).
template <int TS, int D, int LAYOUT, bool DET, bool STRESS = false>
__global__ __launch_bounds__(256) void edm_bwd_tile(BwdArgs a, uint32_t lam0) {
  constexpr int LPR = kBwdLanesPerRow;
  using L = BwdLayout<TS, LPR>;
  constexpr int H = L::H;
  constexpr int Q = L::Q;
  // Tile order for reads: the hardware deals work-groups to the eight XCDs
  // in turn; chunks of kBwdChunk consecutive tiles per XCD, dealt in turn,
  // read faster than one contiguous range of tiles per XCD (which the
  // write-bound kernels use) or than plain order (at N = 20000, TS = 256:
  // 168, 173 and 171 us).  The ragged end keeps plain order.
  uint32_t lam;
  {
    const uint32_t b = blockIdx.x, full = gridDim.x / (8u * kBwdChunk) * (8u * kBwdChunk);
    const uint32_t r = b >> 3;
    lam = lam0 + (b < full ? ((r / kBwdChunk) * 8u + (b & 7u)) * kBwdChunk + r % kBwdChunk : b);
  }
  uint32_t I, J;
  g_lambda(lam, I, J);
  const int t = threadIdx.x;
  const int w = t >> 6;
  const int l = t & 63;
  const int ch = w & 1;
  const int rh = w >> 1;
  const int rg = l / LPR;
  const int cg = l % LPR;
  const int64_t N = a.N;
  const int64_t row0 = (int64_t)I * TS;
  const int64_t col0 = (int64_t)J * TS;
  const int64_t cbase = col0 + H * ch + cg;  // column of q = 0

  __shared__ float xs[TS * D];        // the tile's row points
  __shared__ float xc[TS * D];        // the tile's column points
  __shared__ float rowp[2][TS * D];  // by column half
  __shared__ float colp[2][TS * D];  // by row half
  // The tile's row and column points: coalesced loads into registers,
  // stored to LDS by `stage` (in the gradient passes after the first step's
  // dD loads are out), the lane's column points then read from LDS.
  constexpr int kXsPer = (TS * D + 255) / 256;
  float xsv[kXsPer], xcv[kXsPer];
#pragma unroll
  for (int m = 0; m < kXsPer; ++m) {
    const int e = t + 256 * m;
    const int r = e / D;
    const int k = e - r * D;
    const int64_t p = row0 + r;
    const int64_t pc = col0 + r;
    xsv[m] = (e < TS * D && p < N) ? a.X[p * a.ldx + k] : 0.0f;
    xcv[m] = (e < TS * D && pc < N) ? a.X[pc * a.ldx + k] : 0.0f;
  }
  auto stage = [&]() {
#pragma unroll
    for (int m = 0; m < kXsPer; ++m)
      if (t + 256 * m < TS * D) {
        xs[t + 256 * m] = xsv[m];
        xc[t + 256 * m] = xcv[m];
      }
  };
  float xj[Q][D];  // the lane's column points
  bool jok[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) jok[q] = cbase + LPR * q < N;
  const int cl0 = H * ch + cg;  // tile-local column of q = 0
  auto read_cols = [&]() {
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int k = 0; k < D; ++k) xj[q][k] = xc[(cl0 + LPR * q) * D + k];
  };
  float cacc[Q][D];
#pragma unroll
  for (int q = 0; q < Q; ++q)
#pragma unroll
    for (int k = 0; k < D; ++k) cacc[q][k] = 0.0f;

  const bool diag = I == J;
  float lacc = 0.0f;
  if ((J < I) && (row0 + TS <= N))
    bwd_quarter_steps<TS, LPR, D, LAYOUT, true, STRESS>(stage, read_cols, a, xs, rowp[ch], xj, jok, cacc, row0,
                                                         cbase, H * rh, rg, cg, false, lacc);
  else
    bwd_quarter_steps<TS, LPR, D, LAYOUT, false, STRESS>(stage, read_cols, a, xs, rowp[ch], xj, jok, cacc, row0,
                                                          cbase, H * rh, rg, cg, diag, lacc);
  __shared__ float lossp[4];
  if constexpr (STRESS) {
    lacc = wave_sum(lacc);
    if (l == kSumLane) lossp[w] = lacc;
  }
  // column sums over the row groups (lanes cg + LPR rg)
  static_assert(LPR == 16, "the row-group sum pairs 16-lane rows");
#pragma unroll
  for (int q = 0; q < Q; ++q)
#pragma unroll
    for (int k = 0; k < D; ++k) cacc[q][k] = cross_row_sum(cacc[q][k]);
  if (rg == 0) {
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int k = 0; k < D; ++k)
        colp[rh][(H * ch + cg + LPR * q) * D + k] = STRESS ? 2.0f * cacc[q][k] : cacc[q][k];
  }
  __syncthreads();

  for (int e = t; e < TS * D; e += 256) {
    const float rsum = rowp[0][e] + rowp[1][e];
    const float csum = colp[0][e] + colp[1][e];
    if constexpr (DET) {
      float *dst = a.ws + (uint64_t)lam * 2 * TS * D;
      dst[e] = rsum;
      dst[TS * D + e] = csum;
    } else {
      const int r = e / D;
      const int k = e - r * D;
      if (row0 + r < N) atomicAdd(&a.dX[(row0 + r) * D + k], rsum);
      if (col0 + r < N) atomicAdd(&a.dX[(col0 + r) * D + k], csum);
    }
  }
  if constexpr (STRESS) {
    if (t == 0) {
      const float tl = (lossp[0] + lossp[1]) + (lossp[2] + lossp[3]);
      if constexpr (DET)
        a.ws_loss[lam] = tl;
      else
        atomicAdd(a.loss, tl);
    }
  }
}

// Deterministic second pass: point p in block B = p / TS collects nb + 1
// partials: entry t <= B is the row partial of tile (B, t), entry t > B the
// column partial of tile (B + t - B - 1, B).  A work-group takes 64 points
// of a block (TS / 64 work-groups per block, so the pass has enough of them
// in flight) and holds G groups of 64 d threads (G = 1024 / (64 d), at most
// 4); group g takes the entries t = g mod G with eight accumulators (every
// eighth of its entries, eight loads in flight per thread), and the G group
// sums are added in group order, so the result does not depend on timing.
template <int E>
constexpr int bwd_reduce_groups() {
  return 1024 / E >= 4 ? 4 : (1024 / E >= 2 ? 2 : 1);
}

// Deterministic total of the T per-tile losses by one work-group of NT
// threads: thread t takes entries t, t + NT, ... into eight accumulators
// (entry t + NT m into accumulator m mod 8), then a fixed tree over 1024
// slots (slots past NT hold 0).
template <int NT>
__device__ __forceinline__ void loss_total(const float *__restrict__ part, uint64_t count,
                                           float *__restrict__ loss) {
  __shared__ float buf[1024];
  const int t = threadIdx.x;
  float acc[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  uint64_t e = t;
  for (; e + 7 * NT < count; e += 8 * NT) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[e + NT * u];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] += v[u];
  }
  for (; e < count; e += NT) acc[0] += part[e];
  buf[t] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  for (int x = NT + t; x < 1024; x += NT) buf[x] = 0.0f;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    for (int x = t; x < off; x += NT) buf[x] += buf[x + off];
    __syncthreads();
  }
  if (t == 0) loss[0] = buf[0];
}

constexpr int kReducePoints = 64;  // points per reduce work-group

// With loss != nullptr (the fused stress pass) one more work-group, the
// last, adds the T per-tile losses.
template <int TS, int D>
__global__ __launch_bounds__(kReducePoints * D * bwd_reduce_groups<kReducePoints * D>()) void
edm_bwd_reduce(const float *__restrict__ ws, float *__restrict__ dX, int64_t N, uint32_t nb,
               const float *__restrict__ ws_loss, uint64_t T, float *__restrict__ loss) {
  constexpr int E = kReducePoints * D;
  constexpr int G = bwd_reduce_groups<E>();
  constexpr int S = TS / kReducePoints;  // work-groups per block
  if (blockIdx.x == nb * S) {
    loss_total<E * G>(ws_loss, T, loss);
    return;
  }
  const uint32_t B = blockIdx.x / S;
  const int e = (int)(blockIdx.x % S) * E + (int)(threadIdx.x % E);  // element in the block
  const int g = threadIdx.x / E;
  const int64_t p = (int64_t)B * TS + e / D;
  constexpr int STRIDE = 2 * TS * D;
  const uint64_t tb = tri64(B);
  auto entry = [&](uint32_t t) -> float {
    return t <= B ? ws[(tb + t) * STRIDE + e]
                  : ws[(tri64(t - 1) + B) * STRIDE + TS * D + e];
  };
  const uint32_t cnt = nb + 1;
  float acc[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  if (p < N) {
    uint32_t t = g;
    for (; t + 7 * G < cnt; t += 8 * G) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = entry(t + u * G);
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] += v[u];
    }
    for (; t < cnt; t += G) acc[0] += entry(t);
  }
  const float part =
      ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  if constexpr (G == 1) {
    if (p < N) dX[(uint64_t)B * TS * D + e] = part;
  } else {
    __shared__ float red[G][E];
    const int el = threadIdx.x % E;
    red[g][el] = part;
    __syncthreads();
    if (g == 0 && p < N) {
      float sum = red[0][el];
#pragma unroll
      for (int q = 1; q < G; ++q) sum += red[q][el];
      dX[(uint64_t)B * TS * D + e] = sum;
    }
  }
}

template <int TS, int D, int LAYOUT, bool DET>
static hipError_t launch_bwd_t(const BwdArgs &a) {
  const uint64_t nb = (uint64_t)((a.N + TS - 1) / TS);
  const uint64_t T = nb * (nb + 1) / 2;
  hipError_t e;
  if (!DET) {
    if ((e = launch_fill(a.dX, (uint64_t)a.N * D, 0.0f, a.stream)) != hipSuccess) return e;
  }
  const uint64_t max_blocks = (((uint64_t)1 << 32) - 1) / 256;
  for (uint64_t l0 = 0; l0 < T; l0 += max_blocks) {
    const uint64_t c = T - l0 < max_blocks ? T - l0 : max_blocks;
    hipLaunchKernelGGL((edm_bwd_tile<TS, D, LAYOUT, DET>), dim3((uint32_t)c), dim3(256), 0,
                       a.stream, a, (uint32_t)l0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (DET) {
    hipLaunchKernelGGL((edm_bwd_reduce<TS, D>), dim3((uint32_t)nb * (TS / kReducePoints)),
                       dim3(kReducePoints * D * bwd_reduce_groups<kReducePoints * D>()), 0, a.stream,
                       a.ws, a.dX, a.N, (uint32_t)nb, nullptr, (uint64_t)0, nullptr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int TS, int D>
static hipError_t launch_bwd_d(const BwdArgs &a) {
  if (a.layout == kLayoutFull)
    return a.ws ? launch_bwd_t<TS, D, kLayoutFull, true>(a) : launch_bwd_t<TS, D, kLayoutFull, false>(a);
  if (a.layout == kLayoutStrict)
    return a.ws ? launch_bwd_t<TS, D, kLayoutStrict, true>(a)
                : launch_bwd_t<TS, D, kLayoutStrict, false>(a);
  return a.ws ? launch_bwd_t<TS, D, kLayoutPacked, true>(a)
              : launch_bwd_t<TS, D, kLayoutPacked, false>(a);
}

template <int TS>
static hipError_t launch_bwd_ts(const BwdArgs &a) {
  switch (a.d) {
    case 1: return launch_bwd_d<TS, 1>(a);
    case 2: return launch_bwd_d<TS, 2>(a);
    case 3: return launch_bwd_d<TS, 3>(a);
    case 4: return launch_bwd_d<TS, 4>(a);
    default: return hipErrorInvalidValue;
  }
}

template <int TS, int D, int LAYOUT, bool DET>
static hipError_t launch_stress_t(const BwdArgs &a) {
  const uint64_t nb = (uint64_t)((a.N + TS - 1) / TS);
  const uint64_t T = nb * (nb + 1) / 2;
  hipError_t e;
  if (!DET) {
    if ((e = launch_fill(a.dX, (uint64_t)a.N * D, 0.0f, a.stream)) != hipSuccess) return e;
    if ((e = launch_fill(a.loss, 1, 0.0f, a.stream)) != hipSuccess) return e;
  }
  const uint64_t max_blocks = (((uint64_t)1 << 32) - 1) / 256;
  for (uint64_t l0 = 0; l0 < T; l0 += max_blocks) {
    const uint64_t c = T - l0 < max_blocks ? T - l0 : max_blocks;
    hipLaunchKernelGGL((edm_bwd_tile<TS, D, LAYOUT, DET, true>), dim3((uint32_t)c), dim3(256), 0,
                       a.stream, a, (uint32_t)l0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (DET) {
    // TS / 64 work-groups per block for dX and one more for the loss
    hipLaunchKernelGGL((edm_bwd_reduce<TS, D>), dim3((uint32_t)nb * (TS / kReducePoints) + 1),
                       dim3(kReducePoints * D * bwd_reduce_groups<kReducePoints * D>()), 0, a.stream,
                       a.ws, a.dX, a.N, (uint32_t)nb, a.ws_loss, T, a.loss);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int TS, int D>
static hipError_t launch_stress_d(const BwdArgs &a) {
  const bool det = a.ws != nullptr;
  if (a.layout == kLayoutFull)
    return det ? launch_stress_t<TS, D, kLayoutFull, true>(a) : launch_stress_t<TS, D, kLayoutFull, false>(a);
  if (a.layout == kLayoutStrict)
    return det ? launch_stress_t<TS, D, kLayoutStrict, true>(a)
               : launch_stress_t<TS, D, kLayoutStrict, false>(a);
  return det ? launch_stress_t<TS, D, kLayoutPacked, true>(a)
             : launch_stress_t<TS, D, kLayoutPacked, false>(a);
}

template <int TS>
static hipError_t launch_stress_ts(const BwdArgs &a) {
  switch (a.d) {
    case 1: return launch_stress_d<TS, 1>(a);
    case 2: return launch_stress_d<TS, 2>(a);
    case 3: return launch_stress_d<TS, 3>(a);
    case 4: return launch_stress_d<TS, 4>(a);
    default: return hipErrorInvalidValue;
  }
}

size_t stress_workspace_bytes(int64_t N, int d, int ts) {
  const uint64_t nb = (uint64_t)((N + ts - 1) / ts);
  const uint64_t T = nb * (nb + 1) / 2;
  return (size_t)T * (2 * (size_t)ts * (size_t)d + 1) * sizeof(float);
}

hipError_t launch_stress(int ts, const BwdArgs &a) {
  if (a.N == 0) return launch_fill(a.loss, 1, 0.0f, a.stream);
  switch (ts) {
    case 64: return launch_stress_ts<64>(a);
    case 128: return launch_stress_ts<128>(a);
    case 256: return launch_stress_ts<256>(a);
    default: return hipErrorInvalidValue;
  }
}

size_t backward_workspace_bytes(int64_t N, int d, int ts) {
  const uint64_t nb = (uint64_t)((N + ts - 1) / ts);
  return (size_t)(nb * (nb + 1) / 2) * 2 * (size_t)ts * (size_t)d * sizeof(float);
}

hipError_t launch_backward(int ts, const BwdArgs &a) {
  if (a.N == 0) return hipSuccess;
  switch (ts) {
    case 64: return launch_bwd_ts<64>(a);
    case 128: return launch_bwd_ts<128>(a);
    case 256: return launch_bwd_ts<256>(a);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tdmap
