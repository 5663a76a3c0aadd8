// Host-side launchers of the tdmap kernels (internal; the public interface
// is include/tdmap.h).  Each returns the HIP status of its launches.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tdmap {

struct EdmArgs {
  const float *X;
  int64_t N;
  int d;
  int64_t ldx;
  float *D;
  int64_t ldd;
  int layout;
  hipStream_t stream;
  // mapping-cost (dummy) kernels only
  uint32_t *sink = nullptr;
  uint32_t never = 0;
  int variant = 0;
  // LTM tile and strip launches: only the blocks of shard `shard` of
  // `nshards` equal ranges of the block index space
  uint32_t shard = 0;
  uint32_t nshards = 1;
};

// Block range [lo, hi) of shard s of P over a space of W blocks.
inline void shard_range(uint64_t W, uint32_t s, uint32_t P, uint64_t &lo, uint64_t &hi) {
  lo = W * s / P;
  hi = W * (s + 1) / P;
}

// g(lambda) for lambda0 .. lambda0 + count - 1 (caller checks the range).
hipError_t launch_map_blocks(uint64_t lambda0, uint64_t count, uint32_t *ij, hipStream_t stream);
hipError_t launch_map_blocks_nodiag(uint64_t lambda0, uint64_t count, uint32_t *ij,
                                    hipStream_t stream);

// Paper-style launch: rho x rho threads, one cell per thread.  With
// counts != nullptr the instrumented variant counts instead of storing.
hipError_t launch_cell(int strategy, int rho, const EdmArgs &a, unsigned long long *counts);

// The paper's dummy kernel for a strategy (map and filter only); for LTM,
// a.variant picks the square root (0 exact fix-up, 1 sqrtf, 2 rsq + eps).
hipError_t launch_dummy(int strategy, int rho, const EdmArgs &a);

// g(lambda) export under a map variant (see g_lambda_variant).
hipError_t launch_map_blocks_variant(uint64_t lambda0, uint64_t count, int variant, uint32_t *ij,
                                     hipStream_t stream);

// Coarsened tile launch (LTM on a 1D g(lambda) grid, or BB on an n x n grid).
bool tiled_supported(int ts, int d);
hipError_t launch_tiled(bool bb, int ts, const EdmArgs &a);

struct BwdArgs {
  const float *X;
  int64_t N;
  int d;
  int64_t ldx;
  const float *dD;
  int64_t ldd;
  int layout;
  float *dX;
  float *ws;  // per-tile partial sums (deterministic mode), else nullptr
  hipStream_t stream;
  // stress mode: dD holds the targets delta, loss receives
  // L = sum_{j<i} (D_ij - delta_ij)^2 (one float), ws_loss the per-tile
  // partial losses (deterministic mode)
  float *loss = nullptr;
  float *ws_loss = nullptr;
};

// Backward over g(lambda) tiles of edge ts (64, 128 or 256); d in 1..4.
size_t backward_workspace_bytes(int64_t N, int d, int ts);
hipError_t launch_backward(int ts, const BwdArgs &a);
// Stress loss and its gradient in one pass (ts 64, 128 or 256): the per-tile
// loss partials follow the dX partials in the workspace.
size_t stress_workspace_bytes(int64_t N, int d, int ts);
hipError_t launch_stress(int ts, const BwdArgs &a);

struct BatchArgs {
  const float *X;          // concatenated points, pitch d
  int d;
  int32_t num_sets;
  const int64_t *point_off;
  const int64_t *out_off;
  float *D;
  uint64_t *blk_off;       // workspace: num_sets + 1 tile-count prefix sums
  hipStream_t stream;
};

// One prefix-sum launch plus one persistent launch; ts is 64 or 128.
hipError_t launch_batched(int ts, const BatchArgs &a);

struct GramArgs {
  const float *X;      // FP32 points (exact recompute)
  int64_t N;
  int d;
  int64_t ldx;
  const uint16_t *Xb;  // BF16 points, padded: ceil(N/256)*256 rows of KP features
  const uint16_t *Xlo; // split mode: BF16 low parts x - hi, same layout; else nullptr
  const float *nrm;    // squared norms of the represented points
  int KP;              // features padded to a multiple of 16
  float *D;            // packed output
  unsigned long long *rec_count;  // instrumented launches: recomputed pairs
};

// BF16 Gram-form EDM (packed), workspace of gram_workspace_bytes(N, d,
// split); split = the hi + lo representation with three products.  ts
// selects the kernel: 128 the eight-wave tiles, 256 the 32-row strips.
size_t gram_workspace_bytes(int64_t N, int d, bool split);
bool gram_supported(int64_t N, int ts);
hipError_t launch_gram(const float *X, int64_t N, int d, int64_t ldx, float *D, void *ws, bool split,
                       int ts, hipStream_t stream, uint32_t shard = 0, uint32_t nshards = 1);
// The same launch with every recomputed pair (i, j), j <= i < N, counted
// into *count (zeroed first).
hipError_t launch_gram_count(const float *X, int64_t N, int d, int64_t ldx, float *D, void *ws,
                             bool split, int ts, unsigned long long *count, hipStream_t stream);

// Packed layout written as a linear sweep (g at one-cell granularity).
bool sweep_supported(const EdmArgs &a);
hipError_t launch_sweep(const EdmArgs &a);
// Batched packed sweep with a persistent grid (two 1024-thread work-groups
// per CU, each owning one contiguous stretch of the output).
hipError_t launch_batched_sweep(const BatchArgs &a);

// Keeps the HIP message of a failed call for tdmap_last_error() and
// returns TDMAP_ERR_HIP.
int record_hip_error(hipError_t e, const char *where);

// Fill n floats with a value (a kernel, not a memset, so it can sit in a
// captured graph).
hipError_t launch_fill(float *p, uint64_t n, float v, hipStream_t stream);
// n floats = v with 16-byte non-temporal stores (p 16-byte aligned).
hipError_t launch_stream_fill(float *p, uint64_t n, float v, hipStream_t stream);

}  // namespace tdmap
