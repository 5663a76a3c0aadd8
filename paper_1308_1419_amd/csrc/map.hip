// tdmap_map_blocks: g(lambda) for a range of block indices (Sec. II-A, Eq. (2));
// tdmap_map_blocks_nodiag: the map without the diagonal (Eq. (10)).
#include "device.h"
#include "kernels.h"

namespace tdmap {

// One lane per lambda.  Unlike the EDM kernels, lambda varies across the
// wave here, so the fix-up compares run per lane.
template <bool NODIAG>
__global__ __launch_bounds__(256) void map_blocks_kernel(uint64_t lambda0, uint64_t count,
                                                         uint32_t *__restrict__ ij) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  uint32_t i, j;
  if constexpr (NODIAG)
    g_nodiag((uint32_t)(lambda0 + t), i, j);
  else
    g_lambda((uint32_t)(lambda0 + t), i, j);
  uint2 v;
  v.x = i;
  v.y = j;
  reinterpret_cast<uint2 *>(ij)[t] = v;
}

__global__ __launch_bounds__(256) void map_blocks_variant_kernel(uint64_t lambda0, uint64_t count,
                                                                 int variant,
                                                                 uint32_t *__restrict__ ij) {
  const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  uint32_t i, j;
  g_lambda_variant((uint32_t)(lambda0 + t), variant, i, j);
  uint2 v;
  v.x = i;
  v.y = j;
  reinterpret_cast<uint2 *>(ij)[t] = v;
}

__global__ __launch_bounds__(256) void fill_kernel(float *__restrict__ p, uint64_t n, float v) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride) p[t] = v;
}

template <bool NODIAG>
static hipError_t launch_map_t(uint64_t lambda0, uint64_t count, uint32_t *ij, hipStream_t stream) {
  // at most 2^32 lanes per launch: split the range
  const uint64_t per_launch = (uint64_t)1 << 31;
  for (uint64_t done = 0; done < count; done += per_launch) {
    const uint64_t c = count - done < per_launch ? count - done : per_launch;
    const uint32_t blocks = (uint32_t)((c + 255) / 256);
    hipLaunchKernelGGL(map_blocks_kernel<NODIAG>, dim3(blocks), dim3(256), 0, stream,
                       lambda0 + done, c, ij + 2 * done);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_map_blocks(uint64_t lambda0, uint64_t count, uint32_t *ij, hipStream_t stream) {
  return launch_map_t<false>(lambda0, count, ij, stream);
}

hipError_t launch_map_blocks_nodiag(uint64_t lambda0, uint64_t count, uint32_t *ij,
                                    hipStream_t stream) {
  return launch_map_t<true>(lambda0, count, ij, stream);
}

hipError_t launch_map_blocks_variant(uint64_t lambda0, uint64_t count, int variant, uint32_t *ij,
                                     hipStream_t stream) {
  const uint64_t per_launch = (uint64_t)1 << 31;
  for (uint64_t done = 0; done < count; done += per_launch) {
    const uint64_t c = count - done < per_launch ? count - done : per_launch;
    const uint32_t blocks = (uint32_t)((c + 255) / 256);
    hipLaunchKernelGGL(map_blocks_variant_kernel, dim3(blocks), dim3(256), 0, stream,
                       lambda0 + done, c, variant, ij + 2 * done);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Write-stream reference: one thread per 16-byte chunk, non-temporal
// stores, consecutive threads on consecutive chunks (the plainest store
// stream a kernel can issue).  p is 16-byte aligned; the last n % 4 floats
// are written by thread 0 of the last block.
typedef float f4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void stream_fill_kernel(float *__restrict__ p, uint64_t chunks,
                                                          uint64_t n, float v, uint64_t c0) {
  const uint64_t c = c0 + (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (c < chunks) {
    const f4 x = {v, v, v, v};
    __builtin_nontemporal_store(x, reinterpret_cast<f4 *>(p) + c);
  }
  if (c == chunks) {
    for (uint64_t e = 4 * chunks; e < n; ++e) p[e] = v;
  }
}

hipError_t launch_stream_fill(float *p, uint64_t n, float v, hipStream_t stream) {
  const uint64_t chunks = n / 4;
  // chunks + 1 threads (the extra one writes the tail), at most 2^31 per launch
  const uint64_t per_launch = (uint64_t)1 << 31;
  for (uint64_t c0 = 0; c0 <= chunks; c0 += per_launch) {
    const uint64_t c = chunks + 1 - c0 < per_launch ? chunks + 1 - c0 : per_launch;
    hipLaunchKernelGGL(stream_fill_kernel, dim3((uint32_t)((c + 255) / 256)), dim3(256), 0, stream,
                       p, chunks, n, v, c0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_fill(float *p, uint64_t n, float v, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, p, n, v);
  return hipGetLastError();
}

}  // namespace tdmap
