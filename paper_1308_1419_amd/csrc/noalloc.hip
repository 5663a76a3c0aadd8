// The Gram-form EDM with its workspace in a static device array, for
// callers that cannot allocate device memory (code under stream capture,
// serving loops or harnesses that forbid allocation).
//
// The array below is the workspace tdmap_edm takes from its caller for the
// Gram precisions: the BF16 copy of the points (and, split, their low
// parts) and the squared norms.  Each GPU the library runs on holds its own
// copy of the array from the first call there until the process ends.  In
// host code the array's name only stands for the device symbol, so its
// device address is taken once per device with hipGetSymbolAddress and
// only that address is passed to the kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "kernels.h"
#include "tdmap.h"

namespace {

constexpr size_t kScratchBytes = TDMAP_NOALLOC_SCRATCH_BYTES;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::vector<void *> g_scratch_ptr;  // by device ordinal

// Device address of `scratch` on the current device, taken on the first
// call there.
hipError_t scratch_address(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
  if (g_scratch_ptr[dev] == nullptr) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" {

int tdmap_edm_gram_noalloc(const float *X, int64_t N, int32_t d, int64_t ldx, float *D,
                           int32_t precision, int32_t rho, void *stream) {
  if (N < 0 || d < 1 || ldx < d) return TDMAP_ERR_INVALID;
  if (precision != TDMAP_BF16_GRAM && precision != TDMAP_BF16X3_GRAM) return TDMAP_ERR_INVALID;
  if (rho != 0 && rho != 128 && rho != 256) return TDMAP_ERR_UNSUPPORTED;
  if (N == 0) return TDMAP_OK;
  if (X == nullptr || D == nullptr) return TDMAP_ERR_INVALID;
  if (!tdmap::gram_supported(N, 128) || !tdmap::gram_supported(N, 256))
    return TDMAP_ERR_UNSUPPORTED;
  const bool split = precision == TDMAP_BF16X3_GRAM;
  if (tdmap::gram_workspace_bytes(N, d, split) > kScratchBytes) return TDMAP_ERR_UNSUPPORTED;
  int ts = rho;
  if (ts == 0) {
    // the autotuner's decision for this configuration if tdmap_edm has
    // made one; this entry point never times candidates itself
    ts = tdmap_tuned_rho(TDMAP_OP_EDM, TDMAP_LTM, 256 + precision, d, N);
    if (ts != 128 && ts != 256) ts = 256;
  }
  void *ws = nullptr;
  hipError_t e = scratch_address(&ws);
  if (e == hipSuccess) e = tdmap::launch_gram(X, N, d, ldx, D, ws, split, ts, (hipStream_t)stream);
  if (e != hipSuccess) return tdmap::record_hip_error(e, "tdmap_edm_gram_noalloc");
  return TDMAP_OK;
}

}  // extern "C"
