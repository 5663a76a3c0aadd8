// Coarsened EDM tiles for gfx950.
//
// The paper's point is that g(lambda) maps *blocks*, so the thread
// organisation inside a block is free (Sec. II-A; Sec. V notes this eases
// shared memory and thread coarsening).  Here a 256-thread work-group owns a
// TS x TS tile of cells:
//   - the tile's TS row points are staged once in LDS (read back with
//     broadcast, all lanes of a row share an address);
//   - each lane keeps its column points in registers;
//   - with VEC a lane owns four consecutive columns and stores them with one
//     16-byte store, so a wave writes TS/4-lane runs of 16 bytes: whole
//     64-byte segments of a row.  Without VEC (packed rows start at any
//     offset) a lane owns one column and a wave writes 256 contiguous bytes.
// Stores are non-temporal: the output is written once and not re-read, so
// there is no point keeping it in L2.
//
// LTM launches exactly n(n+1)/2 work-groups, tile (I, J) = g(lambda).  BB
// launches n x n and returns at once above the diagonal (Sec. III-B), with
// the same tile body, which makes the two directly comparable.
#include "device.h"
#include "kernels.h"

namespace tdmap {

typedef float f4 __attribute__((ext_vector_type(4)));

// Interior tile rows in the packed layout with 16-byte stores (TS = 256:
// one row per wave and pass).  Packed row i starts at i(i+1)/2, so the
// tile's row segment [col0, col0 + 256) begins s = (i(i+1)/2 + col0) mod 4
// positions past a 16-byte boundary.  Lane l stores the aligned chunk
// holding columns col0 - s + 4l .. col0 - s + 4l + 3; for lanes 1..63 those
// all lie in the segment, so each of them needs the points of columns
// col0 + 4l - 3 .. col0 + 4l + 3 (kept in registers) and picks four of them
// by s, which is uniform across the wave.  Lane 0 writes the 4 - s head
// cells and the s tail cells (col0 + 256 - s .. col0 + 255) one by one; the
// neighbouring tiles write the rest of the two shared chunks.
template <int TS, int D>
__device__ __forceinline__ void packed_vec_rows(const EdmArgs &a, const float *xs, int64_t row0,
                                                int64_t col0, int lr, float *__restrict__ out) {
  static_assert(TS == 256, "one tile row per wave");
  const int l = threadIdx.x & 63;
  float win[7][D];
#pragma unroll
  for (int o = 0; o < 7; ++o) {
    const int64_t c = col0 + 4 * l - 3 + o;
#pragma unroll
    for (int k = 0; k < D; ++k) win[o][k] = c >= 0 ? a.X[c * a.ldx + k] : 0.0f;
  }
  float tail[3][D];
#pragma unroll
  for (int o = 0; o < 3; ++o)
#pragma unroll
    for (int k = 0; k < D; ++k) tail[o][k] = a.X[(col0 + 253 + o) * a.ldx + k];
  constexpr int PASSES = TS / 4;
#pragma unroll 4
  for (int ps = 0; ps < PASSES; ++ps) {
    const int r = lr + ps * 4;
    const uint64_t i = (uint64_t)(row0 + r);
    float xi[D];
#pragma unroll
    for (int k = 0; k < D; ++k) xi[k] = xs[r * D + k];
    const uint64_t first = tri64(i) + (uint64_t)col0;
    const int sh = (int)(first & 3);
    const uint64_t A0 = first - (uint64_t)sh;
    float v0, v1, v2, v3;
    switch (sh) {
      case 0:
        v0 = pair_dist<D>(xi, win[3]); v1 = pair_dist<D>(xi, win[4]);
        v2 = pair_dist<D>(xi, win[5]); v3 = pair_dist<D>(xi, win[6]);
        break;
      case 1:
        v0 = pair_dist<D>(xi, win[2]); v1 = pair_dist<D>(xi, win[3]);
        v2 = pair_dist<D>(xi, win[4]); v3 = pair_dist<D>(xi, win[5]);
        break;
      case 2:
        v0 = pair_dist<D>(xi, win[1]); v1 = pair_dist<D>(xi, win[2]);
        v2 = pair_dist<D>(xi, win[3]); v3 = pair_dist<D>(xi, win[4]);
        break;
      default:
        v0 = pair_dist<D>(xi, win[0]); v1 = pair_dist<D>(xi, win[1]);
        v2 = pair_dist<D>(xi, win[2]); v3 = pair_dist<D>(xi, win[3]);
        break;
    }
    if (l > 0 || sh == 0) {
      f4 v = {v0, v1, v2, v3};
      __builtin_nontemporal_store(v, reinterpret_cast<f4 *>(out + A0 + 4 * l));
    } else {
      // head: chunk positions sh..3 hold columns col0 .. col0 + 3 - sh
      if (sh <= 1) __builtin_nontemporal_store(v1, out + A0 + 1);
      if (sh <= 2) __builtin_nontemporal_store(v2, out + A0 + 2);
      __builtin_nontemporal_store(v3, out + A0 + 3);
      // tail: columns col0 + 256 - sh .. col0 + 255 (tail[o] is column
      // col0 + 253 + o)
      const float t0 = pair_dist<D>(xi, tail[0]);
      const float t1 = pair_dist<D>(xi, tail[1]);
      const float t2 = pair_dist<D>(xi, tail[2]);
      if (sh == 1) {
        __builtin_nontemporal_store(t2, out + A0 + 256);
      } else if (sh == 2) {
        __builtin_nontemporal_store(t1, out + A0 + 256);
        __builtin_nontemporal_store(t2, out + A0 + 257);
      } else {
        __builtin_nontemporal_store(t0, out + A0 + 256);
        __builtin_nontemporal_store(t1, out + A0 + 257);
        __builtin_nontemporal_store(t2, out + A0 + 258);
      }
    }
  }
}

template <int TS, int D, int LAYOUT, bool VEC, bool BB>
__global__ __launch_bounds__(256) void edm_tile_kernel(EdmArgs a, uint32_t lam0) {
  uint32_t I, J;
  if constexpr (BB) {
    J = blockIdx.x;
    I = blockIdx.y;
    if (J > I) return;
  } else {
    g_lambda(lam0 + blockIdx.x, I, J);
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
  if constexpr (VEC && LAYOUT == kLayoutPacked) {
    if (interior) {
      packed_vec_rows<TS, D>(a, xs, row0, col0, lr, out);
      return;
    }
  }
  if (interior && (VEC ? LAYOUT == kLayoutFull : true)) {
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
        __builtin_nontemporal_store(v, reinterpret_cast<f4 *>(out + idx));
      } else {
        __builtin_nontemporal_store(pair_dist<D>(xi, xj[0]), out + idx);
      }
    }
  } else {
    // diagonal or edge tile: keep cells with j <= i < N (j < N follows)
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
        if (col0 + lc + q <= i) __builtin_nontemporal_store(pair_dist<D>(xi, xj[q]), out + idx + q);
      }
    }
  }
}

template <int TS, int D, int LAYOUT, bool VEC>
static hipError_t launch_tiled_t(bool bb, const EdmArgs &a) {
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

template <int TS, int D>
static hipError_t launch_tiled_d(bool bb, const EdmArgs &a) {
  if (a.layout == kLayoutPacked) {
    if constexpr (TS == 256) {
      if ((reinterpret_cast<uintptr_t>(a.D) & 15) == 0)
        return launch_tiled_t<TS, D, kLayoutPacked, true>(bb, a);
    }
    return launch_tiled_t<TS, D, kLayoutPacked, false>(bb, a);
  }
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
