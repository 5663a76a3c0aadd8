// Device-side building blocks shared by every tdmap kernel (gfx950).
//
// - g_lambda: the block map of Sec. II-A, Eq. (2) with an exact integer
//   fix-up (Sec. V notes that block-level conditionals repair any error of
//   at most one).
// - pair distance: the per-pair function of Sec. IV, Eq. (17), written once
//   so that every strategy produces bit-identical values.
// - output addressing for the full and packed layouts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tdmap {

constexpr int kLayoutFull = 0;
constexpr int kLayoutPacked = 1;
constexpr int kLayoutStrict = 2;  // packed without the diagonal: i(i-1)/2 + j, j < i

__device__ __forceinline__ uint64_t tri64(uint64_t i) { return i * (i + 1) >> 1; }

// g(lambda) = (i, j), i = floor(sqrt(1/4 + 2 lambda) - 1/2), j = lambda - i(i+1)/2.
// The square root is taken as x * rsq(x) (the reciprocal-square-root form
// the paper found fastest, Sec. III-A, Eq. (16)); the single-precision guess
// is within one row of the true i for every lambda < 2^32 (relative error of
// a few ulp on a value below 2^17), and two integer compares against the row
// starts T(i) and T(i+1) make it exact.  lambda is uniform across a
// work-group, so the compares run on the scalar unit.
__device__ __forceinline__ void g_lambda(uint32_t lam, uint32_t &i, uint32_t &j) {
  const float x = __builtin_fmaf(2.0f, (float)lam, 0.25f);
  const float s = x * __builtin_amdgcn_rsqf(x);
  uint32_t r = (uint32_t)__builtin_fmaxf(s - 0.5f, 0.0f);
  uint64_t t = tri64(r);
  if (t > lam) {
    --r;
    t -= (uint64_t)r + 1;  // T(r) = T(r+1) - (r+1)
  } else if (t + r + 1 <= lam) {
    t += (uint64_t)r + 1;  // T(r+1) = T(r) + r + 1
    ++r;
  }
  i = r;
  j = (uint32_t)(lam - t);
}

// The map without the diagonal (Sec. II-A, Eq. (10)): lambda enumerates the
// cells j < i row by row, row i starting at S(i) = i(i-1)/2, and
// i = floor(sqrt(1/4 + 2 lambda) + 1/2), j = lambda - S(i) (the column is
// taken from the row start of this enumeration; see the readings of the
// paper).  Same single-precision guess and integer fix-up as g_lambda.
__device__ __forceinline__ void g_nodiag(uint32_t lam, uint32_t &i, uint32_t &j) {
  const float x = __builtin_fmaf(2.0f, (float)lam, 0.25f);
  const float s = x * __builtin_amdgcn_rsqf(x);
  uint32_t r = (uint32_t)(s + 0.5f);
  if (r == 0) r = 1;
  uint64_t t = ((uint64_t)r * (r - 1)) >> 1;  // S(r)
  if (t > lam) {
    --r;
    t -= r;  // S(r) = S(r+1) - r
  } else if (t + r <= lam) {
    t += r;  // S(r+1) = S(r) + r
    ++r;
  }
  i = r;
  j = (uint32_t)(lam - t);
}

// Work-group b of a 1D launch of nblk work-groups runs on XCD b mod 8 (the
// dispatcher deals work-groups to the eight XCDs in turn).  This returns a
// block index under which every XCD owns one contiguous range: tiles that
// are neighbours in lambda (the same tile row, adjacent columns) then run on
// the same XCD at about the same time, so the cache lines their row segments
// share meet in that XCD's L2 instead of travelling to HBM twice.
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t b, uint32_t nblk) {
  const uint32_t xcd = b & 7, per = nblk >> 3, extra = nblk & 7;
  return xcd * per + (xcd < extra ? xcd : extra) + (b >> 3);
}

// The paper's three ways of taking the row of g(lambda) (Sec. III-A), kept
// for the mapping-cost measurements; only variant 0 is exact everywhere.
//   0: the fix-up map above (rsq guess + integer correction);
//   1: LTM-X, i = floor(sqrtf(1/4 + 2 lambda) - 1/2) with the default
//      (correctly rounded) single-precision square root, no correction;
//   2: LTM-R, sqrt(x) = x * rsq(x) (Eq. (16)) with epsilon = 1e-4 added
//      before the floor, no correction.
// Variants 1 and 2 can be off by one row once lambda is large; j is then
// computed from the wrong row start (it wraps as an unsigned value).
__device__ __forceinline__ void g_lambda_variant(uint32_t lam, int variant, uint32_t &i,
                                                 uint32_t &j) {
  if (variant == 0) {
    g_lambda(lam, i, j);
    return;
  }
  const float x = __builtin_fmaf(2.0f, (float)lam, 0.25f);
  float r;
  if (variant == 1)
    r = sqrtf(x) - 0.5f;
  else
    r = x * __builtin_amdgcn_rsqf(x) - 0.5f + 1e-4f;
  i = (uint32_t)__builtin_floorf(__builtin_fmaxf(r, 0.0f));
  j = (uint32_t)(lam - (uint32_t)tri64(i));
}

// Squared distance then square root, in a fixed operation order:
// s = t_0^2, s = fma(t_k, t_k, s) for k = 1..d-1, D = v_sqrt_f32(s).
// v_sqrt_f32 is accurate to 1 ulp; with d <= 4 the whole value is within a
// few units of FP32 roundoff of the exact distance.
template <int D>
__device__ __forceinline__ float pair_dist(const float (&a)[D], const float (&b)[D]) {
  float t = a[0] - b[0];
  float s = t * t;
#pragma unroll
  for (int k = 1; k < D; ++k) {
    t = a[k] - b[k];
    s = __builtin_fmaf(t, t, s);
  }
  return __builtin_amdgcn_sqrtf(s);
}

// Same arithmetic for a run-time feature count (points read in place).
__device__ __forceinline__ float pair_dist_rt(const float *__restrict__ a,
                                              const float *__restrict__ b, int d) {
  float t = a[0] - b[0];
  float s = t * t;
  for (int k = 1; k < d; ++k) {
    t = a[k] - b[k];
    s = __builtin_fmaf(t, t, s);
  }
  return __builtin_amdgcn_sqrtf(s);
}

template <int D>
__device__ __forceinline__ void load_point(const float *__restrict__ X, int64_t ldx,
                                           int64_t p, float (&v)[D]) {
#pragma unroll
  for (int k = 0; k < D; ++k) v[k] = X[p * ldx + k];
}

// Distance of cells (i, j) read straight from X; D = 0 selects the run-time
// feature loop.
template <int D>
__device__ __forceinline__ float cell_dist(const float *__restrict__ X, int64_t ldx, int d,
                                           int64_t i, int64_t j) {
  if constexpr (D == 0) {
    return pair_dist_rt(X + i * ldx, X + j * ldx, d);
  } else {
    float a[D], b[D];
    load_point<D>(X, ldx, i, a);
    load_point<D>(X, ldx, j, b);
    return pair_dist<D>(a, b);
  }
}

template <int LAYOUT>
__device__ __forceinline__ uint64_t out_index(uint64_t i, uint64_t j, int64_t ldd) {
  if constexpr (LAYOUT == kLayoutFull) {
    return i * (uint64_t)ldd + j;
  } else if constexpr (LAYOUT == kLayoutPacked) {
    return tri64(i) + j;
  } else {
    return ((i * (i - 1)) >> 1) + j;  // 0 for i = 0, which holds no cell
  }
}

// Whether cell (i, j) belongs to the layout's triangle (i < N is separate).
template <int LAYOUT>
__device__ __forceinline__ bool in_triangle(int64_t i, int64_t j) {
  if constexpr (LAYOUT == kLayoutStrict) return j < i;
  return j <= i;
}

// Launch statistics gathered by the instrumented kernels:
// [0] blocks, [1] fully idle blocks, [2] idle threads.
__device__ __forceinline__ void count_block(unsigned long long *counts, int live, int lanes) {
  const int total = __syncthreads_count(live);
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    atomicAdd(&counts[0], 1ull);
    if (total == 0) atomicAdd(&counts[1], 1ull);
    if (lanes - total) atomicAdd(&counts[2], (unsigned long long)(lanes - total));
  }
}

}  // namespace tdmap
