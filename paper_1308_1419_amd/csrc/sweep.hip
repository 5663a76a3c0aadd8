// Packed-layout EDM as a linear sweep of the output.
//
// In the packed layout the index of cell (i, j) is i(i+1)/2 + j, which is
// exactly the block index lambda of Sec. II-A, Eq. (1) for blocks of one
// cell.  So g(lambda) with rho = 1 maps every output position back to its
// cell, and the output can be written in address order: each thread owns
// four consecutive positions (one aligned 16-byte store) and each
// work-group 1024 consecutive positions.  The map runs once per wave (a
// wave's 256 positions span at most a couple of rows); each lane then
// steps from the wave's first cell to its own.
//
// Without the diagonal (strict layout, index i(i-1)/2 + j, j < i) the same
// sweep maps positions with the paper's no-diagonal map (Sec. II-A,
// Eq. (10)); row i then holds i cells instead of i + 1.
//
// The batched variant sweeps the concatenation of every set's packed
// triangle; positions past the end of a set continue in the next one.  Its
// work-groups each own one contiguous stretch of the output and read the
// points of a set from LDS.
#include "device.h"
#include "kernels.h"

namespace tdmap {

typedef float f4 __attribute__((ext_vector_type(4)));

// g(lambda) for 64-bit lambda (packed indices pass 2^32 at N = 92682).  The
// single-precision guess of the row is within one for lambda < 2^40; the
// bounded loops make the result exact.
__device__ __forceinline__ void g_lambda64(uint64_t lam, uint64_t &i, uint64_t &j) {
  const float x = __builtin_fmaf(2.0f, (float)lam, 0.25f);
  const float s = x * __builtin_amdgcn_rsqf(x);
  uint64_t r = (uint64_t)__builtin_fmaxf(s - 0.5f, 0.0f);
  uint64_t t = tri64(r);
  while (t > lam) {
    --r;
    t -= r + 1;
  }
  while (t + r + 1 <= lam) {
    t += r + 1;
    ++r;
  }
  i = r;
  j = lam - t;
}

// Eq. (10) for 64-bit lambda: row i starts at S(i) = i(i-1)/2.
__device__ __forceinline__ void g_nodiag64(uint64_t lam, uint64_t &i, uint64_t &j) {
  const float x = __builtin_fmaf(2.0f, (float)lam, 0.25f);
  const float s = x * __builtin_amdgcn_rsqf(x);
  uint64_t r = (uint64_t)(s + 0.5f);
  if (r == 0) r = 1;
  uint64_t t = (r * (r - 1)) >> 1;
  while (t > lam) {
    --r;
    t -= r;
  }
  while (t + r <= lam) {
    t += r;
    ++r;
  }
  i = r;
  j = lam - t;
}

template <int D>
__device__ __forceinline__ void load_pt(const float *__restrict__ X, int64_t ldx, uint64_t p,
                                        float (&v)[D]) {
#pragma unroll
  for (int k = 0; k < D; ++k) v[k] = X[p * ldx + k];
}

// Column point c of a uniform base, addressed by a 32-bit byte offset
// (c * row_bytes < 2^32 is checked by the caller): the load then takes a
// scalar base and one vector offset, with no 64-bit index arithmetic.
template <int D>
__device__ __forceinline__ void load_pt32(const float *__restrict__ X, uint32_t row_bytes,
                                          uint32_t c, float (&v)[D]) {
  const float *p = reinterpret_cast<const float *>(reinterpret_cast<const char *>(X) + c * row_bytes);
#pragma unroll
  for (int k = 0; k < D; ++k) v[k] = p[k];
}

// One wave writes SW_G consecutive 1 KB pieces (SW_G float4 stores per
// lane, each covering 256 consecutive positions).  When the wave's first
// cell lies in a row of at least SW_G * 256 cells, its positions cover at
// most two rows: the two row points are uniform (scalar loads) and every
// column point load is issued before any arithmetic, so one memory latency
// covers the whole 4 KB.  Short rows (the first few hundred) and the tail
// of the array take a per-lane stepping path.
constexpr int SW_G = 4;
constexpr int SW_WAVE = 256 * SW_G;       // positions per wave
constexpr int SW_BLOCK = 4 * SW_WAVE;     // positions per work-group

// OFF32: contiguous points (ldx == D) and N * D * 4 < 2^32, so a column
// offset is a 32-bit multiple of the constant D * 4.
template <int D, bool STRICT, bool OFF32>
__global__ __launch_bounds__(256) void edm_sweep_kernel(const float *__restrict__ X, int64_t N,
                                                        int64_t ldx, float *__restrict__ out,
                                                        uint64_t total, uint64_t e_base) {
  const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t ew = e_base + (uint64_t)blockIdx.x * SW_BLOCK + (uint64_t)w * SW_WAVE;
  if (ew >= total) return;
  // cells in row i
  auto row_len = [](uint64_t i) -> uint64_t { return STRICT ? i : i + 1; };
  uint64_t iw, jw;
  if constexpr (STRICT)
    g_nodiag64(ew, iw, jw);
  else
    g_lambda64(ew, iw, jw);
  const uint32_t l = threadIdx.x & 63;
  const uint64_t len_w = row_len(iw);
  if (len_w >= (uint64_t)SW_WAVE && ew + SW_WAVE <= total) {
    const uint64_t i1 = iw + 1 < (uint64_t)N ? iw + 1 : iw;  // row below (may be unused)
    float xa[D], xb[D];
    load_pt<D>(X, ldx, iw, xa);
    load_pt<D>(X, ldx, i1, xb);
    float xj[SW_G][4][D];
    bool lo[SW_G][4];
#pragma unroll
    for (int g = 0; g < SW_G; ++g)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if constexpr (OFF32) {
          // every column is below N < 2^31
          const uint32_t j = (uint32_t)jw + 256 * g + 4 * l + q;
          lo[g][q] = j < (uint32_t)len_w;
          load_pt32<D>(X, D * 4u, lo[g][q] ? j : j - (uint32_t)len_w, xj[g][q]);
        } else {
          const uint64_t j = jw + 256 * g + 4 * l + q;
          lo[g][q] = j < len_w;
          load_pt<D>(X, ldx, lo[g][q] ? j : j - len_w, xj[g][q]);
        }
      }
#pragma unroll
    for (int g = 0; g < SW_G; ++g) {
      f4 o;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float xi[D];
#pragma unroll
        for (int k = 0; k < D; ++k) xi[k] = lo[g][q] ? xa[k] : xb[k];
        o[q] = pair_dist<D>(xi, xj[g][q]);
      }
      __builtin_nontemporal_store(o, reinterpret_cast<f4 *>(out + ew + 256 * g + 4 * l));
    }
    return;
  }
  // general path: each lane steps from the wave's first cell to its own
  for (int g = 0; g < SW_G; ++g) {
    const uint64_t e0 = ew + 256 * g + 4 * l;
    if (e0 >= total) break;
    uint64_t i = iw, j = jw + 256 * g + 4 * l;
    while (j >= row_len(i)) {
      j -= row_len(i);
      ++i;
    }
    float xi[D];
    load_pt<D>(X, ldx, i, xi);
    float v[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (e0 + q >= total) break;
      if (j >= row_len(i)) {  // next row
        ++i;
        j = 0;
        load_pt<D>(X, ldx, i, xi);
      }
      float xj[D];
      load_pt<D>(X, ldx, j, xj);
      v[q] = pair_dist<D>(xi, xj);
      ++j;
    }
    if (e0 + 4 <= total) {
      f4 o = {v[0], v[1], v[2], v[3]};
      __builtin_nontemporal_store(o, reinterpret_cast<f4 *>(out + e0));
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (e0 + q < total) __builtin_nontemporal_store(v[q], out + e0 + q);
    }
  }
}

// Batched: the positions [out_off[0], out_off[S]) of the concatenated
// packed triangles, cut into chunks of kBatchChunk consecutive positions.
// set_of finds the set holding position e by a galloping search from a set
// s with out_off[s] <= e; empty sets are skipped.
__device__ __forceinline__ int32_t set_of(const int64_t *__restrict__ oo, int32_t S, int32_t s,
                                          uint64_t e) {
  if ((uint64_t)oo[s + 1] > e) return s;
  // gallop: find hi with oo[hi] > e
  int32_t lo = s + 1, step = 1;
  while (lo + step < S && (uint64_t)oo[lo + step] <= e) {
    lo += step;
    step <<= 1;
  }
  int32_t hi = lo + step < S ? lo + step : S;  // oo[hi] > e (oo[S] = total > e)
  // largest t in [lo, hi) with oo[t] <= e
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if ((uint64_t)oo[mid] <= e) lo = mid; else hi = mid;
  }
  return lo;
}

// A persistent grid of kBatchWgsPerCu 1024-thread work-groups per CU.
// Work-group b of G owns chunks [C b / G, C (b + 1) / G) of the C chunks
// and walks them in address order: every work-group writes one contiguous
// stretch of the output, and the grid is balanced to one chunk.  A chunk
// that lies inside one set of at most kBatchLdsFloats / D points reads the
// set's points from LDS, staged when the walk enters the set, so its loop
// issues no global load and its stores never wait (vmcnt counts loads and
// stores alike, and a wait for a load waits for every store issued before
// it).  Lane l of wave w writes positions c0 + 1024 w + l + 64 q, q < 16:
// each 4-byte store instruction covers 256 contiguous bytes.  The chunk at
// the end of a set, and every chunk of a set too large for LDS, map each
// position on its own (set search and 64-bit g) and read global memory.
constexpr int kBatchThreads = 1024;
constexpr int kBatchPer = 16;                           // positions per lane per chunk
constexpr int kBatchChunk = kBatchThreads * kBatchPer;  // 16384 positions
constexpr int kBatchLdsFloats = 16384;                  // 64 KB
constexpr int kBatchWgsPerCu = 2;

template <int D>
__device__ __forceinline__ void lds_pt(const float *p, float (&v)[D]) {
#pragma unroll
  for (int k = 0; k < D; ++k) v[k] = p[k];
}

template <int D>
__global__ __launch_bounds__(kBatchThreads, 8) void edm_batched_sweep_kernel(
    const float *__restrict__ X, const int64_t *__restrict__ point_off,
    const int64_t *__restrict__ oo, int32_t S, float *__restrict__ out) {
  __shared__ float xs[kBatchLdsFloats];
  const uint64_t first = (uint64_t)oo[0];
  const uint64_t total = (uint64_t)oo[S];
  const uint64_t chunks = (total - first + kBatchChunk - 1) / kBatchChunk;
  const uint64_t G = gridDim.x;
  const uint64_t c_end = chunks * (blockIdx.x + 1) / G;
  const uint32_t t = threadIdx.x;
  const uint32_t off = (t >> 6) * (64 * kBatchPer) + (t & 63);
  // the set of the current chunk's first position, its output range and
  // its points (the same values in every thread)
  int32_t s = 0;
  uint64_t s_beg = first, s_end = (uint64_t)oo[1];
  int64_t p0 = point_off[0], n = point_off[1] - point_off[0];
  int32_t staged = -1;
  for (uint64_t c = chunks * blockIdx.x / G; c < c_end; ++c) {
    const uint64_t c0 = first + c * kBatchChunk;
    if (c0 >= s_end) {
      s = set_of(oo, S, s, c0);
      s_beg = (uint64_t)oo[s];
      s_end = (uint64_t)oo[s + 1];
      p0 = point_off[s];
      n = point_off[s + 1] - p0;
    }
    if (c0 + kBatchChunk <= s_end && n <= kBatchLdsFloats / D) {
      if (staged != s) {
        __syncthreads();  // every wave is done with the previous set
        const float *__restrict__ Xs = X + p0 * D;
        for (int e = (int)t; e < (int)n * D; e += kBatchThreads) xs[e] = Xs[e];
        __syncthreads();
        staged = s;
      }
      // lambda < n(n+1)/2 < 2^28 here: the 32-bit map.  The walk keeps
      // the LDS offsets iD = i D and jD = j D (additions only; j > i is
      // jD > iD, and a row of i + 1 cells is (i + 1) D floats).
      uint32_t i, j;
      g_lambda((uint32_t)(c0 - s_beg) + off, i, j);
      uint32_t iD = i * D, jD = j * D;
      float xi[D], xj[D];
      lds_pt<D>(xs + iD, xi);
#pragma unroll
      for (int q = 0; q < kBatchPer; ++q) {
        if (q > 0) {
          jD += 64 * D;
          if (jD > iD) {
            do {
              iD += D;
              jD -= iD;
            } while (jD > iD);
            lds_pt<D>(xs + iD, xi);
          }
        }
        lds_pt<D>(xs + jD, xj);
        __builtin_nontemporal_store(pair_dist<D>(xi, xj), out + c0 + off + 64 * q);
      }
      continue;
    }
#pragma unroll 1
    for (int q = 0; q < kBatchPer; ++q) {
      const uint64_t e = c0 + off + 64 * q;
      if (e >= total) break;
      int32_t sl = s;
      while ((uint64_t)oo[sl + 1] <= e) ++sl;
      uint64_t i, j;
      g_lambda64(e - (uint64_t)oo[sl], i, j);
      const float *__restrict__ Xl = X + point_off[sl] * D;
      float xi[D], xj[D];
      load_pt<D>(Xl, D, i, xi);
      load_pt<D>(Xl, D, j, xj);
      __builtin_nontemporal_store(pair_dist<D>(xi, xj), out + e);
    }
  }
}

template <int D, bool STRICT, bool OFF32>
static hipError_t launch_sweep_t(const EdmArgs &a) {
  const uint64_t total = STRICT ? (uint64_t)a.N * (uint64_t)(a.N - 1) / 2
                                : (uint64_t)a.N * (uint64_t)(a.N + 1) / 2;
  const uint64_t per_launch = (uint64_t)SW_BLOCK * (((uint64_t)1 << 31) / 256);
  for (uint64_t b = 0; b < total; b += per_launch) {
    const uint64_t c = total - b < per_launch ? total - b : per_launch;
    hipLaunchKernelGGL((edm_sweep_kernel<D, STRICT, OFF32>), dim3((uint32_t)((c + SW_BLOCK - 1) / SW_BLOCK)),
                       dim3(256), 0, a.stream, a.X, a.N, a.ldx, a.D, b + c, b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <int D>
static hipError_t launch_sweep_d(const EdmArgs &a) {
  const bool strict = a.layout == kLayoutStrict;
  const bool off32 = a.ldx == D && (uint64_t)a.N * D * 4u < ((uint64_t)1 << 32);
  if (strict)
    return off32 ? launch_sweep_t<D, true, true>(a) : launch_sweep_t<D, true, false>(a);
  return off32 ? launch_sweep_t<D, false, true>(a) : launch_sweep_t<D, false, false>(a);
}

bool sweep_supported(const EdmArgs &a) {
  return (a.layout == kLayoutPacked || a.layout == kLayoutStrict) && a.d >= 1 && a.d <= 4 &&
         (reinterpret_cast<uintptr_t>(a.D) & 15) == 0;
}

hipError_t launch_sweep(const EdmArgs &a) {
  if (a.N == 0) return hipSuccess;
  switch (a.d) {
    case 1: return launch_sweep_d<1>(a);
    case 2: return launch_sweep_d<2>(a);
    case 3: return launch_sweep_d<3>(a);
    case 4: return launch_sweep_d<4>(a);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_batched_sweep(const BatchArgs &a) {
  if (a.num_sets == 0) return hipSuccess;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  const dim3 grid((uint32_t)(cus * kBatchWgsPerCu));
#define TD_BSWEEP(DD)                                                                          \
  hipLaunchKernelGGL(edm_batched_sweep_kernel<DD>, grid, dim3(kBatchThreads), 0, a.stream, a.X, \
                     a.point_off, a.out_off, a.num_sets, a.D)
  switch (a.d) {
    case 1: TD_BSWEEP(1); break;
    case 2: TD_BSWEEP(2); break;
    case 3: TD_BSWEEP(3); break;
    case 4: TD_BSWEEP(4); break;
    default: return hipErrorInvalidValue;
  }
#undef TD_BSWEEP
  return hipGetLastError();
}

}  // namespace tdmap
