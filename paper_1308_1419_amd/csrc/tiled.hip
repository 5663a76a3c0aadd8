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
// TS = 256 with a 16-byte aligned output: edm_band_kernel below, which
// writes each tile as 8-row strips (one strip per work-group, no LDS, row
// points through the scalar cache; packed rows are realigned to 16-byte
// chunks).  TS = 64 / 128, and TS = 256 with an unaligned output:
// edm_tile_kernel.
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

// Interior rows of a 256-column segment in the packed layout with 16-byte
// stores (one row per wave and call).  Packed row i starts at R(i) = i(i+1)/2 (or
// i(i-1)/2 without the diagonal), so the tile's row segment
// [col0, col0 + 256) begins s = (R(i) + col0) mod 4 positions past a
// 16-byte boundary.  Lane l stores the aligned chunk
// holding columns col0 - s + 4l .. col0 - s + 4l + 3; for lanes 1..63 those
// all lie in the segment, so each of them needs the points of columns
// col0 + 4l - 3 .. col0 + 4l + 3 (kept in registers) and picks four of them
// by s, which is uniform across the wave.  The 4 - s head cells and the s
// tail cells (col0 + 256 - s .. col0 + 255) go out in one 4-byte store
// instruction from lanes 0..5: lanes 0..2 own chunk positions 1..3 of the
// first chunk, lanes 3..5 positions 0..2 of the chunk after the last full
// one, and each keeps the point it needs for every s.  The neighbouring
// tiles write the rest of the two shared chunks.
template <int D>
struct PackedWindow {
  float win[7][D];   // columns col0 + 4l - 3 .. col0 + 4l + 3
  float edge[3][D];  // the edge lane's point for s = 1, 2, 3
};

__device__ __forceinline__ float lane_value(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// XV: X is dense (ldx = D) and 16-byte aligned; the window of lane l is
// then read as 2 D aligned 16-byte chunks (columns col0 + 4l - 4 ..
// col0 + 4l + 3) and the edge points are taken from the windows of lanes 0
// and 63 instead of from memory (every lane of the wave must be active).
template <int D, bool XV = false>
__device__ __forceinline__ void packed_window(const float *__restrict__ X, int64_t ldx, int64_t col0,
                                              PackedWindow<D> &w) {
  const int l = threadIdx.x & 63;
  const int64_t c0 = col0 + 4 * l - 4;
  if (XV && c0 >= 0) {
    const f4 *q = reinterpret_cast<const f4 *>(X + c0 * D);
    float v[8 * D];
#pragma unroll
    for (int m = 0; m < 2 * D; ++m) {
      const f4 t = q[m];
      v[4 * m] = t.x;
      v[4 * m + 1] = t.y;
      v[4 * m + 2] = t.z;
      v[4 * m + 3] = t.w;
    }
#pragma unroll
    for (int o = 0; o < 7; ++o)
#pragma unroll
      for (int k = 0; k < D; ++k) w.win[o][k] = v[(o + 1) * D + k];
  } else {
#pragma unroll
    for (int o = 0; o < 7; ++o) {
      const int64_t c = c0 + 1 + o;
#pragma unroll
      for (int k = 0; k < D; ++k) w.win[o][k] = c >= 0 ? X[c * ldx + k] : 0.0f;
    }
  }
  // edge lane e = l (head, l < 3) or l - 3 (tail, 3 <= l < 6); for shift s
  // it owns column col0 + 1 + l - s (head, kept when l + 1 >= s) or
  // col0 + 256 - s + e (tail, kept when e < s), at packed offset
  // A0 + 1 + l or A0 + 253 + l
  const bool head = l < 3;
  const int e = head ? l : l - 3;
  if constexpr (XV) {
    // column col0 + 1 + l - s is lane 0's win[4 + l - s] (index 1..5);
    // column col0 + 256 - s + e is lane 63's win[7 - s + e] (4..6 when kept)
#pragma unroll
    for (int k = 0; k < D; ++k) {
      float h[6], t[7];
#pragma unroll
      for (int o = 1; o <= 5; ++o) h[o] = lane_value(w.win[o][k], 0);
#pragma unroll
      for (int o = 4; o <= 6; ++o) t[o] = lane_value(w.win[o][k], 63);
#pragma unroll
      for (int s = 1; s <= 3; ++s) {
        const int oh = 4 + l - s;
        const int ot = 7 - s + e;
        const float hv = oh <= 1 ? h[1] : oh == 2 ? h[2] : oh == 3 ? h[3] : oh == 4 ? h[4] : h[5];
        const float tv = ot <= 4 ? t[4] : ot == 5 ? t[5] : t[6];
        const bool ok = l < 6 && (head ? l + 1 >= s : e < s);
        w.edge[s - 1][k] = ok ? (head ? hv : tv) : 0.0f;
      }
    }
  } else {
#pragma unroll
    for (int s = 1; s <= 3; ++s) {
      const bool ok = l < 6 && (head ? l + 1 >= s : e < s);
      const int64_t c = head ? col0 + 1 + l - s : col0 + 256 - s + e;
#pragma unroll
      for (int k = 0; k < D; ++k) w.edge[s - 1][k] = ok ? X[c * ldx + k] : 0.0f;
    }
  }
}

// One interior row i of a 256-column segment starting at col0.
template <int D, int LAYOUT>
__device__ __forceinline__ void packed_vec_row(const PackedWindow<D> &w, const float (&xi)[D],
                                               uint64_t i, int64_t col0, float *__restrict__ out) {
  const int l = threadIdx.x & 63;
  const bool head = l < 3;
  const int e = head ? l : l - 3;
  const int eoff = head ? 1 + l : 253 + l;
  const uint64_t first = out_index<LAYOUT>(i, (uint64_t)col0, 0);
  const int sh = (int)(first & 3);
  const uint64_t A0 = first - (uint64_t)sh;
  float v0, v1, v2, v3, ve;
  switch (sh) {
    case 0:
      v0 = pair_dist<D>(xi, w.win[3]); v1 = pair_dist<D>(xi, w.win[4]);
      v2 = pair_dist<D>(xi, w.win[5]); v3 = pair_dist<D>(xi, w.win[6]);
      ve = 0.0f;
      break;
    case 1:
      v0 = pair_dist<D>(xi, w.win[2]); v1 = pair_dist<D>(xi, w.win[3]);
      v2 = pair_dist<D>(xi, w.win[4]); v3 = pair_dist<D>(xi, w.win[5]);
      ve = pair_dist<D>(xi, w.edge[0]);
      break;
    case 2:
      v0 = pair_dist<D>(xi, w.win[1]); v1 = pair_dist<D>(xi, w.win[2]);
      v2 = pair_dist<D>(xi, w.win[3]); v3 = pair_dist<D>(xi, w.win[4]);
      ve = pair_dist<D>(xi, w.edge[1]);
      break;
    default:
      v0 = pair_dist<D>(xi, w.win[0]); v1 = pair_dist<D>(xi, w.win[1]);
      v2 = pair_dist<D>(xi, w.win[2]); v3 = pair_dist<D>(xi, w.win[3]);
      ve = pair_dist<D>(xi, w.edge[2]);
      break;
  }
  if (l > 0 || sh == 0) {
    f4 v = {v0, v1, v2, v3};
    put<LAYOUT>(v, reinterpret_cast<f4 *>(out + A0 + 4 * l));
  }
  if (sh != 0 && l < 6 && (head ? l + 1 >= sh : e < sh)) put<LAYOUT>(ve, out + A0 + eoff);
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
// A wave owns rows w and w + 4 of the strip, 64 lanes x 4 columns each, so
// the row point is uniform (read through the scalar cache) and each store
// writes a 1 KB row segment; there is no LDS and no barrier.  Packed and
// strict rows go through packed_vec_row (plain stores: the chunks shared by
// the segments of tiles J and J + 1 meet in L2, those two work-groups being
// neighbours in w and so on one XCD).  Measured at N = 30000: 325 us full,
// 414 us packed (the packed TS = 64 tile takes 380 us and stays the tuned
// choice there).
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
    // packed rows start anywhere: 16-byte stores of realigned chunks
    if (interior) {
      PackedWindow<D> pw;
      packed_window<D, XV>(X, ldx, (int64_t)J * 256, pw);
#pragma unroll
      for (int r = 0; r < H / 4; ++r) {
        const int64_t i = row0 + wv + 4 * r;
        float xi[D];
#pragma unroll
        for (int m = 0; m < D; ++m) xi[m] = X[i * ldx + m];
        packed_vec_row<D, LAYOUT>(pw, xi, (uint64_t)i, (int64_t)J * 256, out);
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
  const uint64_t max_blocks = (((uint64_t)1 << 32) - 1) / 256;
  for (uint64_t w0 = 0; w0 < W; w0 += max_blocks) {
    const uint64_t c = W - w0 < max_blocks ? W - w0 : max_blocks;
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
  }
  const uint64_t nb = (uint64_t)((a.N + TS - 1) / TS);
  if (bb) {
    hipLaunchKernelGGL((edm_tile_kernel<TS, D, LAYOUT, VEC, true>), dim3((uint32_t)nb, (uint32_t)nb),
                       dim3(256), 0, a.stream, a, 0u);
    return hipGetLastError();
  }
  const uint64_t T = nb * (nb + 1) / 2;
  const uint64_t max_blocks = (((uint64_t)1 << 32) - 1) / 256;
  for (uint64_t l0 = 0; l0 < T; l0 += max_blocks) {
    const uint64_t c = T - l0 < max_blocks ? T - l0 : max_blocks;
    hipLaunchKernelGGL((edm_tile_kernel<TS, D, LAYOUT, VEC, false>), dim3((uint32_t)c), dim3(256), 0,
                       a.stream, a, (uint32_t)l0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int TS, int D, int LAYOUT>
static hipError_t launch_tiled_packed(bool bb, const EdmArgs &a) {
  if constexpr (TS == 256) {
    if ((reinterpret_cast<uintptr_t>(a.D) & 15) == 0) {
      const bool xv = a.ldx == D && (reinterpret_cast<uintptr_t>(a.X) & 15) == 0;
      return xv ? launch_band<D, LAYOUT, true>(bb, a) : launch_band<D, LAYOUT, false>(bb, a);
    }
  }
  return launch_tiled_t<TS, D, LAYOUT, false>(bb, a);
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
