// Coarsened EDM tiles for gfx950.
//
// The paper's point is that g(lambda) maps *blocks*, so the thread
// organisation inside a block is free (Sec. II-A; Sec. V notes this eases
// shared memory and thread coarsening).  Here a 256-thread work-group owns a
// TS x TS tile of cells:
//   - the tile's TS row points are staged once in LDS (read back with
//     broadcast, all lanes of a row share an address);
//   - each lane keeps its column points in registers;
//   - with VEC (full layout) a lane owns four consecutive columns and
//     stores them with one 16-byte store, so a wave writes TS/4-lane runs of
//     16 bytes: whole 64-byte segments of a row.  Without VEC a lane owns one
//     column and a wave writes 256 contiguous bytes.
// Full-layout stores are non-temporal (the output is written once and not
// re-read); packed-layout stores are plain (see put below).
//
// LTM launches exactly n(n+1)/2 work-groups, tile (I, J) = g(lambda) with
// lambda remapped so that every XCD owns one contiguous range of it
// (xcd_contiguous in device.h).  BB launches n x n and returns at once above
// the diagonal (Sec. III-B), with the same tile body, which makes the two
// directly comparable.
//
// TS = 256: edm_band_kernel below, which writes each tile as 8-row strips
// (one strip per work-group, no LDS, row points through the scalar cache);
// the full layout needs a 16-byte aligned output (else edm_tile_kernel).
// TS = 64 / 128: edm_tile_kernel.
#include "device.h"
#include "kernels.h"

namespace tdmap {

typedef float f4 __attribute__((ext_vector_type(4)));

// Output stores.  Full-layout rows are written whole by one tile each, so
// they bypass the caches (non-temporal).  Packed rows start at arbitrary
// offsets: the 16-byte chunks and cache lines at both ends of a tile's row
// segment are shared with the neighbouring tiles, and plain (cached) stores
// let those parts meet in L2 instead of reaching HBM as separate partial
// line writes (measured faster at every tile size).
template <int LAYOUT, typename T>
__device__ __forceinline__ void put(T v, T *p) {
  if constexpr (LAYOUT == kLayoutFull)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

template <int TS, int D, int LAYOUT, bool VEC, bool BB>
__global__ __launch_bounds__(256) void edm_tile_kernel(EdmArgs a, uint32_t lam0) {
  uint32_t I, J;
  if constexpr (BB) {
    J = blockIdx.x;
    I = blockIdx.y;
    if (J > I) return;
  } else {
    g_lambda(lam0 + xcd_contiguous(blockIdx.x, gridDim.x), I, J);
  }
  constexpr int V = VEC ? 4 : 1;    // cells per lane per row
  constexpr int LPR = TS / V;       // lanes per tile row
  static_assert(256 % LPR == 0, "tile row must divide the work-group");
  constexpr int RPP = 256 / LPR;    // rows per pass
  constexpr int PASSES = TS / RPP;

  const int t = threadIdx.x;
  const int lc = (t % LPR) * V;
  const int lr = t / LPR;
  const int64_t N = a.N;
  const int64_t row0 = (int64_t)I * TS;
  const int64_t col0 = (int64_t)J * TS;

  __shared__ float xs[TS * D];
  for (int e = t; e < TS * D; e += 256) {
    const int r = e / D;
    const int k = e - r * D;
    const int64_t p = row0 + r;
    xs[e] = p < N ? a.X[p * a.ldx + k] : 0.0f;
  }
  float xj[V][D];
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const int64_t p = col0 + lc + q;
#pragma unroll
    for (int k = 0; k < D; ++k) xj[q][k] = p < N ? a.X[p * a.ldx + k] : 0.0f;
  }
  __syncthreads();

  float *__restrict__ out = a.D;
  const bool interior = (J < I) && (row0 + TS <= N);
  static_assert(!VEC || LAYOUT == kLayoutFull, "16-byte stores need the full layout");
  if (interior) {
#pragma unroll 8
    for (int ps = 0; ps < PASSES; ++ps) {
      const int r = lr + ps * RPP;
      float xi[D];
#pragma unroll
      for (int k = 0; k < D; ++k) xi[k] = xs[r * D + k];
      const uint64_t idx = out_index<LAYOUT>(row0 + r, col0 + lc, a.ldd);
      if constexpr (VEC) {
        f4 v;
        v.x = pair_dist<D>(xi, xj[0]);
        v.y = pair_dist<D>(xi, xj[1]);
        v.z = pair_dist<D>(xi, xj[2]);
        v.w = pair_dist<D>(xi, xj[3]);
        put<LAYOUT>(v, reinterpret_cast<f4 *>(out + idx));
      } else {
        put<LAYOUT>(pair_dist<D>(xi, xj[0]), out + idx);
      }
    }
  } else {
    // diagonal or edge tile: keep cells with j <= i < N (j < i for the
    // layout without the diagonal; j < N follows)
    for (int ps = 0; ps < PASSES; ++ps) {
      const int r = lr + ps * RPP;
      const int64_t i = row0 + r;
      if (i >= N) break;
      float xi[D];
#pragma unroll
      for (int k = 0; k < D; ++k) xi[k] = xs[r * D + k];
      const uint64_t idx = out_index<LAYOUT>(i, col0 + lc, a.ldd);
#pragma unroll
      for (int q = 0; q < V; ++q) {
        if (in_triangle<LAYOUT>(i, col0 + lc + q))
          put<LAYOUT>(pair_dist<D>(xi, xj[q]), out + idx + q);
      }
    }
  }
}

// 256 x 256 tiles written as strips.  Tile row I (256 rows) is
// cut into kBandStrips strips of kBandRows rows, and a work-group writes one
// strip of one tile, kBandRows x 256 cells.  LTM: work-group w takes tile
// row I from g(w / kBandStrips) (the paper's block map at the tile level);
// the kBandStrips (I + 1) work-groups of tile row I are then numbered
// u = k (I + 1) + J, strip k outer and tile column J inner, so the
// work-groups in flight finish a few whole rows of the triangle before they
// move down instead of spreading over the many rows of whole tiles (the
// write stream stays within a compact window of addresses; measured 15 %
// faster than whole-tile work-groups at N = 30000).  BB: a kBandStrips n x n
// grid, blockIdx.y = I, blockIdx.x = k n + J, returning at once for J > I.
// A wave owns rows w and w + 4 of the strip, so the row point is uniform
// (read through the scalar cache); there is no LDS and no barrier.  Full
// layout: a lane owns four consecutive columns and each non-temporal
// 16-byte store writes a 1 KB row segment.  Packed layouts (rows start at
// any offset): a lane owns columns l, l + 64, l + 128, l + 192 and each
// plain 4-byte store instruction writes 256 contiguous bytes; the lines
// shared by the segments of tiles J and J + 1 meet in L2, those two
// work-groups being neighbours in w and so on one XCD.  Measured at
// N = 30000: 323 us full (16-byte and 4-byte stores alike), 292 us packed
// (16-byte stores of realigned chunks: 414 us).
constexpr int kBandRows = 8;

// The four column points of lane l.  XV: X is dense (ldx = D) and 16-byte
// aligned, so the 4 D floats of columns c .. c + 3 are D aligned 16-byte
// chunks.
template <int D, bool XV>
__device__ __forceinline__ void band_columns(const float *__restrict__ X, int64_t N, int64_t ldx,
                                             int64_t c, float (&xj)[4][D]) {
  if constexpr (XV) {
    if (c + 3 < N) {
      const f4 *q = reinterpret_cast<const f4 *>(X + c * D);
      float v[4 * D];
#pragma unroll
      for (int m = 0; m < D; ++m) {
        const f4 t = q[m];
        v[4 * m] = t.x;
        v[4 * m + 1] = t.y;
        v[4 * m + 2] = t.z;
        v[4 * m + 3] = t.w;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int k = 0; k < D; ++k) xj[u][k] = v[u * D + k];
      return;
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int k = 0; k < D; ++k) xj[u][k] = c + u < N ? X[(c + u) * ldx + k] : 0.0f;
}

template <int D, int LAYOUT, bool BB, bool XV>
__global__ __launch_bounds__(256) void edm_band_kernel(const float *__restrict__ X, int64_t N,
                                                       int64_t ldx, float *__restrict__ out,
                                                       int64_t ldd, uint32_t w0) {
  constexpr int H = kBandRows;
  constexpr int kBandStrips = 256 / H;
  uint32_t I, J, k;
  if constexpr (BB) {
    I = blockIdx.y;
    k = blockIdx.x / gridDim.y;
    J = blockIdx.x - k * gridDim.y;
    if (J > I) return;
  } else {
    const uint32_t w = w0 + xcd_contiguous(blockIdx.x, gridDim.x);
    uint32_t Jt;
    g_lambda(w / kBandStrips, I, Jt);
    // w - kBandStrips T(I): Jt = w / kBandStrips - T(I)
    const uint32_t u = kBandStrips * Jt + w % kBandStrips;
    k = u / (I + 1);
    J = u - k * (I + 1);
  }
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t row0 = (int64_t)I * 256 + (int64_t)k * H;
  const int64_t c = (int64_t)J * 256 + (threadIdx.x & 63) * 4;
  const bool interior = J < I && row0 + H <= N;
  if constexpr (LAYOUT != kLayoutFull) {
    // packed rows start anywhere: lane l owns columns col0 + l + 64 q and a
    // store instruction writes 256 contiguous bytes (plain stores)
    if (interior) {
      const int64_t cb = (int64_t)J * 256 + (threadIdx.x & 63);
      float xq[4][D];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int m = 0; m < D; ++m) xq[q][m] = X[(cb + 64 * q) * ldx + m];
#pragma unroll
      for (int r = 0; r < H / 4; ++r) {
        const int64_t i = row0 + wv + 4 * r;
        float xi[D];
#pragma unroll
        for (int m = 0; m < D; ++m) xi[m] = X[i * ldx + m];
        float *o = out + out_index<LAYOUT>((uint64_t)i, (uint64_t)cb, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) put<LAYOUT>(pair_dist<D>(xi, xq[q]), o + 64 * q);
      }
      return;
    }
  }
  float xj[4][D];
  band_columns<D, XV>(X, N, ldx, c, xj);
  if (LAYOUT == kLayoutFull && interior) {
#pragma unroll
    for (int r = 0; r < H / 4; ++r) {
      const int64_t i = row0 + wv + 4 * r;
      float xi[D];
#pragma unroll
      for (int m = 0; m < D; ++m) xi[m] = X[i * ldx + m];
      f4 v;
      v.x = pair_dist<D>(xi, xj[0]);
      v.y = pair_dist<D>(xi, xj[1]);
      v.z = pair_dist<D>(xi, xj[2]);
      v.w = pair_dist<D>(xi, xj[3]);
      __builtin_nontemporal_store(v, reinterpret_cast<f4 *>(out + i * ldd + c));
    }
  } else {
    // diagonal or edge strip: rows below N, cells with j <= i
#pragma unroll
    for (int r = 0; r < H / 4; ++r) {
      const int64_t i = row0 + wv + 4 * r;
      if (i >= N) break;
      float xi[D];
#pragma unroll
      for (int m = 0; m < D; ++m) xi[m] = X[i * ldx + m];
      float v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = pair_dist<D>(xi, xj[q]);
      if constexpr (LAYOUT == kLayoutFull) {
        float *o = out + i * ldd + c;
        if (c + 3 <= i) {
          f4 v4 = {v[0], v[1], v[2], v[3]};
          __builtin_nontemporal_store(v4, reinterpret_cast<f4 *>(o));
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (c + q <= i) __builtin_nontemporal_store(v[q], o + q);
        }
      } else {
        const uint64_t idx = out_index<LAYOUT>((uint64_t)i, (uint64_t)c, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (in_triangle<LAYOUT>(i, c + q)) put<LAYOUT>(v[q], out + idx + q);
      }
    }
  }
}

template <int D, int LAYOUT, bool XV>
static hipError_t launch_band(bool bb, const EdmArgs &a) {
  constexpr int kBandStrips = 256 / kBandRows;
  const uint64_t nb = (uint64_t)((a.N + 255) / 256);
  if (bb) {
    hipLaunchKernelGGL((edm_band_kernel<D, LAYOUT, true, XV>), dim3((uint32_t)(kBandStrips * nb), (uint32_t)nb),
                       dim3(256), 0, a.stream, a.X, a.N, a.ldx, a.D, a.ldd, 0u);
    return hipGetLastError();
  }
  const uint64_t W = (uint64_t)kBandStrips * (nb * (nb + 1) / 2);
  if (W > 0xffffffffull) return hipErrorInvalidValue;  // w is 32-bit (N above 4 million)
  uint64_t lo, hi;
  shard_range(W, a.shard, a.nshards, lo, hi);
  const uint64_t max_blocks = (((uint64_t)1 << 32) - 1) / 256;
  for (uint64_t w0 = lo; w0 < hi; w0 += max_blocks) {
    const uint64_t c = hi - w0 < max_blocks ? hi - w0 : max_blocks;
    hipLaunchKernelGGL((edm_band_kernel<D, LAYOUT, false, XV>), dim3((uint32_t)c), dim3(256), 0, a.stream,
                       a.X, a.N, a.ldx, a.D, a.ldd, (uint32_t)w0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int TS, int D, int LAYOUT, bool VEC>
static hipError_t launch_tiled_t(bool bb, const EdmArgs &a) {
  if constexpr (TS == 256 && LAYOUT == kLayoutFull && VEC) {
    // strips of 256-column tiles for the aligned full layout
    const bool xv = a.ldx == D && (reinterpret_cast<uintptr_t>(a.X) & 15) == 0;
    return xv ? launch_band<D, kLayoutFull, true>(bb, a) : launch_band<D, kLayoutFull, false>(bb, a);
  } else {
    const uint64_t nb = (uint64_t)((a.N + TS - 1) / TS);
    if (bb) {
      hipLaunchKernelGGL((edm_tile_kernel<TS, D, LAYOUT, VEC, true>),
                         dim3((uint32_t)nb, (uint32_t)nb), dim3(256), 0, a.stream, a, 0u);
      return hipGetLastError();
    }
    const uint64_t T = nb * (nb + 1) / 2;
    uint64_t lo, hi;
    shard_range(T, a.shard, a.nshards, lo, hi);
    const uint64_t max_blocks = (((uint64_t)1 << 32) - 1) / 256;
    for (uint64_t l0 = lo; l0 < hi; l0 += max_blocks) {
      const uint64_t c = hi - l0 < max_blocks ? hi - l0 : max_blocks;
      hipLaunchKernelGGL((edm_tile_kernel<TS, D, LAYOUT, VEC, false>), dim3((uint32_t)c), dim3(256),
                         0, a.stream, a, (uint32_t)l0);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
}

template <int TS, int D, int LAYOUT>
static hipError_t launch_tiled_packed(bool bb, const EdmArgs &a) {
  if constexpr (TS == 256) {
    const bool xv = a.ldx == D && (reinterpret_cast<uintptr_t>(a.X) & 15) == 0;
    return xv ? launch_band<D, LAYOUT, true>(bb, a) : launch_band<D, LAYOUT, false>(bb, a);
  } else {
    return launch_tiled_t<TS, D, LAYOUT, false>(bb, a);
  }
}

template <int TS, int D>
static hipError_t launch_tiled_d(bool bb, const EdmArgs &a) {
  if (a.layout == kLayoutPacked) return launch_tiled_packed<TS, D, kLayoutPacked>(bb, a);
  if (a.layout == kLayoutStrict) return launch_tiled_packed<TS, D, kLayoutStrict>(bb, a);
  const bool aligned = (a.ldd % 4 == 0) && ((reinterpret_cast<uintptr_t>(a.D) & 15) == 0);
  return aligned ? launch_tiled_t<TS, D, kLayoutFull, true>(bb, a)
                 : launch_tiled_t<TS, D, kLayoutFull, false>(bb, a);
}

template <int TS>
static hipError_t launch_tiled_ts(bool bb, const EdmArgs &a) {
  switch (a.d) {
    case 1: return launch_tiled_d<TS, 1>(bb, a);
    case 2: return launch_tiled_d<TS, 2>(bb, a);
    case 3: return launch_tiled_d<TS, 3>(bb, a);
    case 4: return launch_tiled_d<TS, 4>(bb, a);
    default: return hipErrorInvalidValue;
  }
}

bool tiled_supported(int ts, int d) {
  return (ts == 64 || ts == 128 || ts == 256) && d >= 1 && d <= 4;
}

hipError_t launch_tiled(bool bb, int ts, const EdmArgs &a) {
  if (a.N == 0) return hipSuccess;
  switch (ts) {
    case 64: return launch_tiled_ts<64>(bb, a);
    case 128: return launch_tiled_ts<128>(bb, a);
    case 256: return launch_tiled_ts<256>(bb, a);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tdmap
