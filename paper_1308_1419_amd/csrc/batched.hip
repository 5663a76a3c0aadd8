// Many independent EDMs in one persistent launch.
//
// Set s (points point_off[s] .. point_off[s+1]) has nb_s = ceil(n_s / TS)
// tile rows and T(nb_s) = nb_s(nb_s+1)/2 tiles.  A scan kernel writes the
// prefix sums P[s] = sum_{t<s} T(nb_t) into the workspace; the global tile
// index g in [0, P[S]) then names set s (P[s] <= g < P[s+1]) and its local
// tile lambda = g - P[s], placed by g(lambda) (Sec. II-A, Eq. (2)) inside
// that set's triangle.
//
// The persistent grid (a few work-groups per CU) splits [0, P[S]) into
// contiguous equal ranges; a work-group finds the set of its first tile by
// binary search and then walks forward, so consecutive tiles it writes are
// neighbours in the set's packed output.
//
// Inside a tile every wave owns whole rows: the row index is uniform across
// the wave, so the row point is read once through the scalar cache, and
// each lane computes TS/64 columns and writes them with 4-byte stores
// (packed rows start at arbitrary offsets).  The stores are plain (cached):
// the cache lines at both ends of a tile's row segment are shared with the
// neighbouring tiles and are combined in L2.
#include "device.h"
#include "kernels.h"

namespace tdmap {

// P[0] = 0, P[s+1] = P[s] + T(ceil(n_s / ts)).  One work-group of 1024
// threads scans 1024 sets at a time with a carry.
__global__ __launch_bounds__(1024) void batched_prefix_kernel(const int64_t *__restrict__ point_off,
                                                              int32_t num_sets, int32_t ts,
                                                              uint64_t *__restrict__ P) {
  __shared__ uint64_t buf[1024];
  __shared__ uint64_t carry;
  const int t = threadIdx.x;
  if (t == 0) {
    carry = 0;
    P[0] = 0;
  }
  __syncthreads();
  for (int32_t base = 0; base < num_sets; base += 1024) {
    const int32_t s = base + t;
    uint64_t v = 0;
    if (s < num_sets) {
      const int64_t n = point_off[s + 1] - point_off[s];
      const uint64_t nb = n > 0 ? (uint64_t)((n + ts - 1) / ts) : 0;
      v = nb * (nb + 1) / 2;
    }
    buf[t] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const uint64_t add = t >= off ? buf[t - off] : 0;
      __syncthreads();
      buf[t] += add;
      __syncthreads();
    }
    if (s < num_sets) P[s + 1] = carry + buf[t];
    __syncthreads();
    if (t == 1023) carry += buf[1023];
    __syncthreads();
  }
}

// Everything a tile needs to know about its set and position.
struct TileRef {
  int32_t s;
  uint32_t I, J;
  int64_t n;
  int64_t p0;
  int64_t o0;
};

__device__ __forceinline__ TileRef locate_tile(const uint64_t *__restrict__ P,
                                               const int64_t *__restrict__ point_off,
                                               const int64_t *__restrict__ out_off, int32_t s,
                                               uint64_t g) {
  while (P[s + 1] <= g) ++s;
  TileRef t;
  t.s = s;
  g_lambda((uint32_t)(g - P[s]), t.I, t.J);
  t.p0 = point_off[s];
  t.n = point_off[s + 1] - t.p0;
  t.o0 = out_off[s];
  return t;
}

// The kernel arguments are separate restrict pointers, so the uniform row
// point loads go through the scalar cache (their wait counter does not
// include the vector stores), and the next tile's column points are loaded
// before the current tile's stores are issued.
template <int TS, int D>
__global__ __launch_bounds__(256) void edm_batched_kernel(const float *__restrict__ X,
                                                          const int64_t *__restrict__ point_off,
                                                          const int64_t *__restrict__ out_off,
                                                          const uint64_t *__restrict__ P,
                                                          int32_t num_sets, float *__restrict__ Dout) {
  constexpr int CPL = TS / 64;
  constexpr int RPW = TS / 4;
  const uint64_t total = P[num_sets];
  const uint64_t G = gridDim.x;
  const uint64_t chunk = (total + G - 1) / G;
  const uint64_t lo = (uint64_t)blockIdx.x * chunk;
  const uint64_t hi = lo + chunk < total ? lo + chunk : total;
  if (lo >= hi) return;

  // largest s with P[s] <= lo (P is non-decreasing, P[0] = 0)
  int32_t s0 = 0, s1 = num_sets;
  while (s1 - s0 > 1) {
    const int32_t mid = (s0 + s1) >> 1;
    if (P[mid] <= lo) s0 = mid; else s1 = mid;
  }

  const int l = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  TileRef cur = locate_tile(P, point_off, out_off, s0, lo);
  float xj[CPL][D];
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    const int64_t j = (int64_t)cur.J * TS + l + 64 * c;
#pragma unroll
    for (int k = 0; k < D; ++k) xj[c][k] = j < cur.n ? X[(cur.p0 + j) * D + k] : 0.0f;
  }
  for (uint64_t g = lo; g < hi; ++g) {
    // prefetch the next tile's column points before this tile's stores
    TileRef nxt = cur;
    float xn[CPL][D];
    if (g + 1 < hi) {
      nxt = locate_tile(P, point_off, out_off, cur.s, g + 1);
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const int64_t j = (int64_t)nxt.J * TS + l + 64 * c;
#pragma unroll
        for (int k = 0; k < D; ++k) xn[c][k] = j < nxt.n ? X[(nxt.p0 + j) * D + k] : 0.0f;
      }
    }
    const float *__restrict__ Xs = X + cur.p0 * D;
    float *__restrict__ out = Dout + cur.o0;
    const int64_t n = cur.n;
    const int64_t row0 = (int64_t)cur.I * TS;
    const int64_t col0 = (int64_t)cur.J * TS;
    const bool interior = (cur.J < cur.I) && (row0 + TS <= n);
    if (interior) {
#pragma unroll 4
      for (int rr = 0; rr < RPW; ++rr) {
        const int64_t i = row0 + rr * 4 + w;
        float xi[D];
#pragma unroll
        for (int k = 0; k < D; ++k) xi[k] = Xs[i * D + k];
        float *__restrict__ o = out + tri64((uint64_t)i) + col0 + l;
#pragma unroll
        for (int c = 0; c < CPL; ++c) o[64 * c] = pair_dist<D>(xi, xj[c]);
      }
    } else {
      for (int rr = 0; rr < RPW; ++rr) {
        const int64_t i = row0 + rr * 4 + w;
        if (i >= n) break;
        float xi[D];
#pragma unroll
        for (int k = 0; k < D; ++k) xi[k] = Xs[i * D + k];
        float *__restrict__ o = out + tri64((uint64_t)i);
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
          const int64_t j = col0 + l + 64 * c;
          if (j <= i) o[j] = pair_dist<D>(xi, xj[c]);
        }
      }
    }
    cur = nxt;
#pragma unroll
    for (int c = 0; c < CPL; ++c)
#pragma unroll
      for (int k = 0; k < D; ++k) xj[c][k] = xn[c][k];
  }
}

// Compute units of the current device (queried per launch: no shared state
// between threads or devices).
static int cu_count() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
    return n;
  return 256;
}

template <int TS, int D>
static hipError_t launch_batched_t(const BatchArgs &a) {
  hipLaunchKernelGGL(batched_prefix_kernel, dim3(1), dim3(1024), 0, a.stream, a.point_off,
                     a.num_sets, TS, a.blk_off);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, edm_batched_kernel<TS, D>, 256, 0) !=
          hipSuccess ||
      per_cu <= 0)
    per_cu = 4;
  const uint32_t grid = (uint32_t)(cu_count() * per_cu);
  hipLaunchKernelGGL((edm_batched_kernel<TS, D>), dim3(grid), dim3(256), 0, a.stream, a.X,
                     a.point_off, a.out_off, a.blk_off, a.num_sets, a.D);
  return hipGetLastError();
}

template <int TS>
static hipError_t launch_batched_ts(const BatchArgs &a) {
  switch (a.d) {
    case 1: return launch_batched_t<TS, 1>(a);
    case 2: return launch_batched_t<TS, 2>(a);
    case 3: return launch_batched_t<TS, 3>(a);
    case 4: return launch_batched_t<TS, 4>(a);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_batched(int ts, const BatchArgs &a) {
  if (a.num_sets == 0) return hipSuccess;
  switch (ts) {
    case 64: return launch_batched_ts<64>(a);
    case 128: return launch_batched_ts<128>(a);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tdmap
