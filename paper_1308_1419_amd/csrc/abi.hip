// The C ABI of include/tdmap.h: argument validation, dispatch to the
// kernels, the tile autotuner and the closed-form launch statistics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "kernels.h"
#include "tdmap.h"

namespace {

thread_local std::string g_last_error;

int hip_fail(hipError_t e, const char *where) {
  g_last_error = std::string(where) + ": " + hipGetErrorString(e);
  return TDMAP_ERR_HIP;
}

#define TD_HIP(call, where)                    \
  do {                                         \
    hipError_t e_ = (call);                    \
    if (e_ != hipSuccess) return hip_fail(e_, where); \
  } while (0)

inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
inline uint64_t tri(uint64_t n) { return n * (n + 1) / 2; }

bool is_cell_rho(int rho) { return rho == 8 || rho == 16 || rho == 32; }

// ---------------------------------------------------------------------------
// autotuner: times each candidate tile on the caller's stream and buffers on
// first use of a configuration, keeps the fastest.
// ---------------------------------------------------------------------------

using TuneKey = std::tuple<int, int, int, int, int>;  // op, strategy, layout, d, log2 bucket
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tuned;

int size_bucket(int64_t size) {
  int b = 0;
  while (b < 62 && ((int64_t)1 << b) < size) ++b;
  return b;
}

int tuned_lookup(const TuneKey &k) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tuned.find(k);
  return it == g_tuned.end() ? 0 : it->second;
}

void tuned_store(const TuneKey &k, int v) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tuned[k] = v;
}

// Runs launch(c) for every candidate c: one warm-up each, then `reps`
// rounds in which every candidate is timed over `burst` back-to-back
// launches, median of its per-launch times.  The rounds interleave the
// candidates because the device's speed drifts over a burst of launches
// (clocks settle), which would otherwise favour whichever candidate is
// timed first; the bursts keep the launch latency and the first launch
// after an idle gap out of the comparison.  Returns the fastest candidate
// (0 on error, with *status set).
template <class F>
int autotune(const std::vector<int> &cands, hipStream_t s, F launch, int *status) {
  hipEvent_t ev[2];
  *status = TDMAP_OK;
  if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess) {
    *status = TDMAP_ERR_HIP;
    g_last_error = "autotune: hipEventCreate failed";
    return 0;
  }
  const int reps = 5;
  const int burst = 3;
  std::vector<std::vector<float>> ms(cands.size());
  for (size_t k = 0; k < cands.size() && *status == TDMAP_OK; ++k) {
    const hipError_t e = launch(cands[k]);
    if (e != hipSuccess) *status = hip_fail(e, "autotune launch");
  }
  for (int r = 0; r < reps && *status == TDMAP_OK; ++r) {
    for (size_t k = 0; k < cands.size(); ++k) {
      hipError_t e = hipEventRecord(ev[0], s);
      for (int b = 0; b < burst && e == hipSuccess; ++b) e = launch(cands[k]);
      if (e == hipSuccess) e = hipEventRecord(ev[1], s);
      if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
      if (e != hipSuccess) {
        *status = hip_fail(e, "autotune run");
        break;
      }
      float t = 0.0f;
      (void)hipEventElapsedTime(&t, ev[0], ev[1]);
      ms[k].push_back(t / burst);
    }
  }
  int best = 0;
  float best_ms = 0.0f;
  if (*status == TDMAP_OK) {
    for (size_t k = 0; k < cands.size(); ++k) {
      std::sort(ms[k].begin(), ms[k].end());
      const float med = ms[k][ms[k].size() / 2];
      if (best == 0 || med < best_ms) {
        best = cands[k];
        best_ms = med;
      }
    }
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  return *status == TDMAP_OK ? best : 0;
}

// ---------------------------------------------------------------------------
// closed-form launch statistics (Sec. II-A, Sec. III-B)
// ---------------------------------------------------------------------------

void rec_shape_host(uint64_t nb, uint64_t &m, uint64_t &k) {
  uint64_t best = 0;
  for (uint64_t mm = 16; mm >= 1; --mm) {
    uint64_t kk = 0;
    while ((mm << kk) < nb) ++kk;
    if (best == 0 || (mm << kk) < best) {
      best = mm << kk;
      m = mm;
      k = kk;
    }
  }
}

bool waste_closed_form(int strategy, int64_t N, int rho, int64_t out[3]) {
  const uint64_t n = ceil_div((uint64_t)N, (uint64_t)rho);
  const uint64_t P = tri((uint64_t)N);
  const uint64_t lanes = (uint64_t)rho * rho;
  uint64_t blocks = 0, idle = 0;
  switch (strategy) {
    case TDMAP_LTM:
      blocks = tri(n);
      break;
    case TDMAP_BB:
      blocks = n * n;
      idle = n * (n - (n > 0)) / 2;
      break;
    case TDMAP_UTM:
      blocks = ceil_div(P, lanes);
      break;
    case TDMAP_RB: {
      const uint64_t rows = (N % 2 == 0) ? N + 1 : N;
      const uint64_t cols = (N % 2 == 0) ? N / 2 : N / 2 + 1;
      blocks = ceil_div(rows, rho) * ceil_div(cols, rho);
      if (N == 0) blocks = 0;
      break;
    }
    case TDMAP_REC: {
      if (n == 0) break;
      uint64_t m = 1, k = 0;
      rec_shape_host(n, m, k);
      // diagonal pass: m x m blocks per base square, upper m(m-1)/2 idle,
      // and base rows at or past n idle on and below the base diagonal
      blocks = (m * m) << k;
      idle = (m * (m - 1) / 2) << k;
      for (uint64_t q = 0; q < (1ull << k); ++q)
        for (uint64_t by = 0; by < m; ++by)
          if (q * m + by >= n) idle += by + 1;
      for (uint64_t lev = 0; lev < k; ++lev) {
        const uint64_t s = m << lev;
        for (uint64_t q = 0; q < (1ull << (k - 1 - lev)); ++q) {
          blocks += s * s;
          const uint64_t r0 = (2 * q + 1) * s;
          if (r0 + s > n) idle += s * std::min<uint64_t>(s, r0 + s - n);
        }
      }
      break;
    }
    default:
      return false;
  }
  out[0] = (int64_t)blocks;
  out[1] = (int64_t)idle;
  out[2] = (int64_t)(blocks * lanes - P);
  return true;
}

int validate_edm_common(const float *X, int64_t N, int32_t d, int64_t ldx, const void *D,
                        int64_t ldd, int32_t layout) {
  if (N < 0 || d < 1 || ldx < d) return TDMAP_ERR_INVALID;
  if (layout != TDMAP_FULL && layout != TDMAP_PACKED && layout != TDMAP_PACKED_STRICT)
    return TDMAP_ERR_INVALID;
  if (N == 0) return TDMAP_OK;
  if (X == nullptr) return TDMAP_ERR_INVALID;
  // without the diagonal a single point has no cell, so D may then be NULL
  if (D == nullptr && !(layout == TDMAP_PACKED_STRICT && N == 1)) return TDMAP_ERR_INVALID;
  if (layout == TDMAP_FULL && ldd < N) return TDMAP_ERR_INVALID;
  return TDMAP_OK;
}

// Validation and kernel choice of the Gram precisions (rho 0, 128 or 256);
// with tune, rho = 0 runs the autotuner on the first call of a
// configuration, otherwise it takes the cached choice or the strips.
int gram_prepare(const float *X, int64_t N, int32_t d, int64_t ldx, float *D, int32_t layout,
                 int32_t strategy, int32_t rho, int32_t precision, void *workspace,
                 size_t ws_bytes, void *stream, bool tune, int *ts_out) {
  const bool split = precision == TDMAP_BF16X3_GRAM;
  if (strategy != TDMAP_LTM || layout != TDMAP_PACKED || (rho != 0 && rho != 128 && rho != 256))
    return TDMAP_ERR_UNSUPPORTED;
  if (N == 0) return TDMAP_OK;
  if (!tdmap::gram_supported(N, 128) || !tdmap::gram_supported(N, 256))
    return TDMAP_ERR_UNSUPPORTED;
  if (workspace == nullptr || ws_bytes < tdmap::gram_workspace_bytes(N, d, split))
    return TDMAP_ERR_WORKSPACE;
  // the BF16 copies are written and read as 16-byte chunks
  if ((reinterpret_cast<uintptr_t>(workspace) & 15) != 0) return TDMAP_ERR_INVALID;
  int ts = rho;
  if (ts == 0) {
    const TuneKey key(TDMAP_OP_EDM, strategy, 256 + precision, d, size_bucket(N));
    ts = tuned_lookup(key);
    if (ts == 0 && tune) {
      hipStream_t s = (hipStream_t)stream;
      int st = TDMAP_OK;
      ts = autotune({128, 256}, s,
                    [&](int c) { return tdmap::launch_gram(X, N, d, ldx, D, workspace, split, c, s); },
                    &st);
      if (st != TDMAP_OK) return st;
      tuned_store(key, ts);
    }
    if (ts == 0) ts = 256;
  }
  *ts_out = ts;
  return TDMAP_OK;
}

}  // namespace

int tdmap::record_hip_error(hipError_t e, const char *where) { return hip_fail(e, where); }

extern "C" {

const char *tdmap_status_string(int32_t status) {
  switch (status) {
    case TDMAP_OK: return "success";
    case TDMAP_ERR_INVALID: return "invalid argument";
    case TDMAP_ERR_UNSUPPORTED: return "unsupported configuration";
    case TDMAP_ERR_WORKSPACE: return "workspace missing or too small";
    case TDMAP_ERR_HIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char *tdmap_last_error(void) { return g_last_error.c_str(); }

void tdmap_autotune_reset(void) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tuned.clear();
}

int32_t tdmap_tuned_rho(int32_t op, int32_t strategy, int32_t layout, int32_t d, int64_t size) {
  if (op != TDMAP_OP_EDM) strategy = 0;
  if (op == TDMAP_OP_BATCHED)
    layout = size_bucket(layout);  // the mean set size in points
  else if (op != TDMAP_OP_EDM)
    layout = 0;
  return tuned_lookup(TuneKey(op, strategy, layout, d, size_bucket(size)));
}

int tdmap_map_blocks(uint64_t lambda0, uint64_t count, uint32_t *ij, void *stream) {
  if (count == 0) return TDMAP_OK;
  if (ij == nullptr) return TDMAP_ERR_INVALID;
  if (lambda0 > ((uint64_t)1 << 32) || count > ((uint64_t)1 << 32) - lambda0)
    return TDMAP_ERR_UNSUPPORTED;
  TD_HIP(tdmap::launch_map_blocks(lambda0, count, ij, (hipStream_t)stream), "tdmap_map_blocks");
  return TDMAP_OK;
}

int tdmap_map_blocks_nodiag(uint64_t lambda0, uint64_t count, uint32_t *ij, void *stream) {
  if (count == 0) return TDMAP_OK;
  if (ij == nullptr) return TDMAP_ERR_INVALID;
  if (lambda0 > ((uint64_t)1 << 32) || count > ((uint64_t)1 << 32) - lambda0)
    return TDMAP_ERR_UNSUPPORTED;
  TD_HIP(tdmap::launch_map_blocks_nodiag(lambda0, count, ij, (hipStream_t)stream),
         "tdmap_map_blocks_nodiag");
  return TDMAP_OK;
}

size_t tdmap_workspace_size(int32_t op, int64_t N, int32_t d, int32_t num_sets, int32_t rho,
                            int32_t flags) {
  if (N < 0 || d < 1) return 0;
  switch (op) {
    case TDMAP_OP_EDM:
      if (flags != TDMAP_BF16_GRAM && flags != TDMAP_BF16X3_GRAM) return 0;
      return tdmap::gram_workspace_bytes(N, d, flags == TDMAP_BF16X3_GRAM);
    case TDMAP_OP_BACKWARD:
      if (!flags || d > 4) return 0;
      if (rho == 0)
        return std::max({tdmap::backward_workspace_bytes(N, d, 64),
                         tdmap::backward_workspace_bytes(N, d, 128),
                         tdmap::backward_workspace_bytes(N, d, 256)});
      if (rho != 64 && rho != 128 && rho != 256) return 0;
      return tdmap::backward_workspace_bytes(N, d, rho);
    case TDMAP_OP_STRESS:
      if (!flags || d > 4) return 0;
      if (rho == 0)
        return std::max({tdmap::stress_workspace_bytes(N, d, 64),
                         tdmap::stress_workspace_bytes(N, d, 128),
                         tdmap::stress_workspace_bytes(N, d, 256)});
      if (rho != 64 && rho != 128 && rho != 256) return 0;
      return tdmap::stress_workspace_bytes(N, d, rho);
    case TDMAP_OP_BATCHED:
      if (num_sets < 0) return 0;
      return (size_t)(num_sets + 1) * sizeof(uint64_t);
    default:
      return 0;
  }
}

int tdmap_edm(const float *X, int64_t N, int32_t d, int64_t ldx, float *D, int64_t ldd,
              int32_t layout, int32_t strategy, int32_t rho, int32_t precision, void *workspace,
              size_t ws_bytes, void *stream) {
  int st = validate_edm_common(X, N, d, ldx, D, ldd, layout);
  if (st != TDMAP_OK) return st;
  if (strategy < TDMAP_LTM || strategy > TDMAP_REC) return TDMAP_ERR_INVALID;
  if (precision != TDMAP_FP32 && precision != TDMAP_BF16_GRAM && precision != TDMAP_BF16X3_GRAM)
    return TDMAP_ERR_INVALID;
  if (!(rho == 0 || rho == 1 || is_cell_rho(rho) || rho == 64 || rho == 128 || rho == 256))
    return TDMAP_ERR_INVALID;
  if (precision != TDMAP_FP32) {
    int ts = 0;
    st = gram_prepare(X, N, d, ldx, D, layout, strategy, rho, precision, workspace, ws_bytes,
                      stream, true, &ts);
    if (st != TDMAP_OK || N == 0) return st;
    TD_HIP(tdmap::launch_gram(X, N, d, ldx, D, workspace, precision == TDMAP_BF16X3_GRAM, ts,
                              (hipStream_t)stream),
           "tdmap_edm");
    return TDMAP_OK;
  }
  const bool tiled = !is_cell_rho(rho);
  if (tiled && strategy != TDMAP_LTM && strategy != TDMAP_BB) return TDMAP_ERR_UNSUPPORTED;
  if (layout == TDMAP_PACKED_STRICT && !tiled) return TDMAP_ERR_UNSUPPORTED;
  if (tiled && d > 4) return TDMAP_ERR_UNSUPPORTED;
  if (rho == 1 && (strategy != TDMAP_LTM || layout == TDMAP_FULL ||
                   (reinterpret_cast<uintptr_t>(D) & 15) != 0))
    return TDMAP_ERR_UNSUPPORTED;
  if (N == 0) return TDMAP_OK;
  // block index limits: lambda and the UTM thread index are 32-bit
  const uint64_t edge = tiled ? (rho > 1 ? (uint64_t)rho : 64) : (uint64_t)rho;
  const uint64_t nb = ceil_div((uint64_t)N, edge);
  if (tri(nb) > 0xffffffffull) return TDMAP_ERR_UNSUPPORTED;
  if (strategy == TDMAP_UTM && tri((uint64_t)N) > 0xffffffffull) return TDMAP_ERR_UNSUPPORTED;
  if (strategy == TDMAP_BB && nb > 0x7fffffffull) return TDMAP_ERR_UNSUPPORTED;

  hipStream_t s = (hipStream_t)stream;
  tdmap::EdmArgs a{X, N, d, ldx, D, ldd, layout, s};
  if (!tiled) {
    TD_HIP(tdmap::launch_cell(strategy, rho, a, nullptr), "tdmap_edm");
    return TDMAP_OK;
  }
  const bool bb = strategy == TDMAP_BB;
  // rho = 1: the packed linear sweep (g at one-cell granularity)
  auto run = [&](int c) {
    return c == 1 ? tdmap::launch_sweep(a) : tdmap::launch_tiled(bb, c, a);
  };
  int ts = rho;
  if (ts == 0) {
    // an output that rules out the 16-byte stores (full layout) or the sweep
    // (packed layouts) is tuned under its own key
    const bool aligned = (reinterpret_cast<uintptr_t>(D) & 15) == 0 &&
                         (layout != TDMAP_FULL || ldd % 4 == 0);
    const TuneKey key(TDMAP_OP_EDM, strategy, layout + (aligned ? 0 : 64), d, size_bucket(N));
    ts = tuned_lookup(key);
    if (ts == 0) {
      std::vector<int> cands{64, 128, 256};
      if (!bb && tdmap::sweep_supported(a)) cands.insert(cands.begin(), 1);
      ts = autotune(cands, s, run, &st);
      if (st != TDMAP_OK) return st;
      tuned_store(key, ts);
    }
  }
  TD_HIP(run(ts), "tdmap_edm");
  return TDMAP_OK;
}

int tdmap_edm_shard(const float *X, int64_t N, int32_t d, int64_t ldx, float *D, int64_t ldd,
                    int32_t layout, int32_t strategy, int32_t rho, int32_t precision,
                    void *workspace, size_t ws_bytes, int32_t shard, int32_t num_shards,
                    void *stream) {
  int st = validate_edm_common(X, N, d, ldx, D, ldd, layout);
  if (st != TDMAP_OK) return st;
  if (strategy < TDMAP_LTM || strategy > TDMAP_REC) return TDMAP_ERR_INVALID;
  if (precision != TDMAP_FP32 && precision != TDMAP_BF16_GRAM && precision != TDMAP_BF16X3_GRAM)
    return TDMAP_ERR_INVALID;
  if (num_shards < 1 || shard < 0 || shard >= num_shards) return TDMAP_ERR_INVALID;
  // every shard must cut the same block space: the kernel is named, never tuned
  if (strategy != TDMAP_LTM) return TDMAP_ERR_UNSUPPORTED;
  if (precision != TDMAP_FP32) {
    if (rho != 128 && rho != 256) return TDMAP_ERR_UNSUPPORTED;
    int ts = 0;
    st = gram_prepare(X, N, d, ldx, D, layout, strategy, rho, precision, workspace, ws_bytes,
                      stream, false, &ts);
    if (st != TDMAP_OK || N == 0) return st;
    TD_HIP(tdmap::launch_gram(X, N, d, ldx, D, workspace, precision == TDMAP_BF16X3_GRAM, ts,
                              (hipStream_t)stream, (uint32_t)shard, (uint32_t)num_shards),
           "tdmap_edm_shard");
    return TDMAP_OK;
  }
  if (rho != 64 && rho != 128 && rho != 256) return TDMAP_ERR_UNSUPPORTED;
  if (d > 4) return TDMAP_ERR_UNSUPPORTED;
  if (N == 0) return TDMAP_OK;
  const uint64_t nb = ceil_div((uint64_t)N, (uint64_t)rho);
  if (tri(nb) > 0xffffffffull) return TDMAP_ERR_UNSUPPORTED;
  tdmap::EdmArgs a{X, N, d, ldx, D, ldd, layout, (hipStream_t)stream};
  a.shard = (uint32_t)shard;
  a.nshards = (uint32_t)num_shards;
  TD_HIP(tdmap::launch_tiled(false, rho, a), "tdmap_edm_shard");
  return TDMAP_OK;
}

int tdmap_gram_recompute_count(const float *X, int64_t N, int32_t d, int64_t ldx, float *D,
                               int32_t precision, int32_t rho, void *workspace, size_t ws_bytes,
                               uint64_t *count, void *stream) {
  int st = validate_edm_common(X, N, d, ldx, D, 0, TDMAP_PACKED);
  if (st != TDMAP_OK) return st;
  if (count == nullptr) return TDMAP_ERR_INVALID;
  if (precision != TDMAP_BF16_GRAM && precision != TDMAP_BF16X3_GRAM) return TDMAP_ERR_INVALID;
  if (!(rho == 0 || rho == 128 || rho == 256)) return TDMAP_ERR_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  int ts = 0;
  st = gram_prepare(X, N, d, ldx, D, TDMAP_PACKED, TDMAP_LTM, rho, precision, workspace, ws_bytes,
                    stream, false, &ts);
  if (st != TDMAP_OK) return st;
  if (N == 0) {
    TD_HIP(tdmap::launch_fill(reinterpret_cast<float *>(count), 2, 0.0f, s),
           "tdmap_gram_recompute_count");
    return TDMAP_OK;
  }
  TD_HIP(tdmap::launch_gram_count(X, N, d, ldx, D, workspace, precision == TDMAP_BF16X3_GRAM, ts,
                                  reinterpret_cast<unsigned long long *>(count), s),
         "tdmap_gram_recompute_count");
  return TDMAP_OK;
}

int tdmap_edm_backward(const float *X, int64_t N, int32_t d, int64_t ldx, const float *dD,
                       int64_t ldd, int32_t layout, float *dX, int32_t rho, int32_t deterministic,
                       void *workspace, size_t ws_bytes, void *stream) {
  int st = validate_edm_common(X, N, d, ldx, dD, ldd, layout);
  if (st != TDMAP_OK) return st;
  if (N > 0 && dX == nullptr) return TDMAP_ERR_INVALID;
  if (rho != 0 && rho != 64 && rho != 128 && rho != 256) return TDMAP_ERR_INVALID;
  if (d > 4) return TDMAP_ERR_UNSUPPORTED;
  if (N == 0) return TDMAP_OK;
  const uint64_t nb = ceil_div((uint64_t)N, rho ? (uint64_t)rho : 64);
  if (tri(nb) > 0xffffffffull) return TDMAP_ERR_UNSUPPORTED;
  const bool det = deterministic != 0;
  if (det) {
    const size_t need = tdmap_workspace_size(TDMAP_OP_BACKWARD, N, d, 0, rho, 1);
    if (workspace == nullptr || ws_bytes < need) return TDMAP_ERR_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  tdmap::BwdArgs a{X, N, d, ldx, dD, ldd, layout, dX,
                   det ? reinterpret_cast<float *>(workspace) : nullptr, s};
  int ts = rho;
  if (ts == 0) {
    const TuneKey key(TDMAP_OP_BACKWARD, 0, 0, d, size_bucket(N));
    ts = tuned_lookup(key);
    if (ts == 0) {
      ts = autotune({64, 128, 256}, s, [&](int c) { return tdmap::launch_backward(c, a); }, &st);
      if (st != TDMAP_OK) return st;
      tuned_store(key, ts);
    }
  }
  TD_HIP(tdmap::launch_backward(ts, a), "tdmap_edm_backward");
  return TDMAP_OK;
}

int tdmap_stress_backward(const float *X, int64_t N, int32_t d, int64_t ldx, const float *delta,
                          int64_t ldd, int32_t layout, float *dX, float *loss, int32_t rho,
                          int32_t deterministic, void *workspace, size_t ws_bytes,
                          void *stream) {
  int st = validate_edm_common(X, N, d, ldx, delta, ldd, layout);
  if (st != TDMAP_OK) return st;
  if (loss == nullptr || (N > 0 && dX == nullptr)) return TDMAP_ERR_INVALID;
  if (rho != 0 && rho != 64 && rho != 128 && rho != 256) return TDMAP_ERR_INVALID;
  if (d > 4) return TDMAP_ERR_UNSUPPORTED;
  const uint64_t nb = ceil_div((uint64_t)N, rho ? (uint64_t)rho : 64);
  if (tri(nb) > 0xffffffffull) return TDMAP_ERR_UNSUPPORTED;
  const bool det = deterministic != 0;
  if (det && N > 0) {
    const size_t need = tdmap_workspace_size(TDMAP_OP_STRESS, N, d, 0, rho, 1);
    if (workspace == nullptr || ws_bytes < need) return TDMAP_ERR_WORKSPACE;
  }
  hipStream_t s = (hipStream_t)stream;
  tdmap::BwdArgs a{X, N, d, ldx, delta, ldd, layout, dX, nullptr, s};
  a.loss = loss;
  auto run = [&](int c) {
    if (det) {
      // gradient partials of T tiles, then the T loss partials
      const uint64_t nbc = ceil_div((uint64_t)N, (uint64_t)c);
      a.ws = reinterpret_cast<float *>(workspace);
      a.ws_loss = a.ws + tri(nbc) * 2 * (uint64_t)c * (uint64_t)d;
    }
    return tdmap::launch_stress(c, a);
  };
  int ts = rho;
  if (ts == 0 && N > 0) {
    const TuneKey key(TDMAP_OP_STRESS, 0, 0, d, size_bucket(N));
    ts = tuned_lookup(key);
    if (ts == 0) {
      ts = autotune({64, 128, 256}, s, run, &st);
      if (st != TDMAP_OK) return st;
      tuned_store(key, ts);
    }
  }
  TD_HIP(run(ts ? ts : 64), "tdmap_stress_backward");
  return TDMAP_OK;
}

int tdmap_edm_batched(const float *X_cat, int32_t d, int32_t num_sets, const int64_t *point_off,
                      const int64_t *out_off, float *D_cat, int32_t rho, void *workspace,
                      size_t ws_bytes, void *stream) {
  if (num_sets < 0 || d < 1) return TDMAP_ERR_INVALID;
  if (rho != 0 && rho != 1 && rho != 64 && rho != 128) return TDMAP_ERR_INVALID;
  if (num_sets == 0) return TDMAP_OK;
  if (X_cat == nullptr || point_off == nullptr || out_off == nullptr || D_cat == nullptr)
    return TDMAP_ERR_INVALID;
  if (d > 4) return TDMAP_ERR_UNSUPPORTED;
  const size_t need = tdmap_workspace_size(TDMAP_OP_BATCHED, 0, d, num_sets, rho, 0);
  if (workspace == nullptr || ws_bytes < need) return TDMAP_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  tdmap::BatchArgs a{X_cat, d, num_sets, point_off, out_off, D_cat,
                     reinterpret_cast<uint64_t *>(workspace), s};
  // rho = 1: persistent linear sweep of the concatenated packed output;
  // 64 / 128: persistent walk over the prefix-summed tile space
  auto run = [&](int c) {
    return c == 1 ? tdmap::launch_batched_sweep(a) : tdmap::launch_batched(c, a);
  };
  int ts = rho;
  int st = TDMAP_OK;
  if (ts == 0) {
    // the decision depends on the set sizes as well as their number (the
    // sweep stages a set in LDS only up to 16384 / d points): key it on the
    // mean set size too, read back from point_off[num_sets]
    int64_t total = 0;
    TD_HIP(hipMemcpyAsync(&total, point_off + num_sets, sizeof(total), hipMemcpyDeviceToHost, s),
           "tdmap_edm_batched");
    TD_HIP(hipStreamSynchronize(s), "tdmap_edm_batched");
    if (total < 0) return TDMAP_ERR_INVALID;
    const TuneKey key(TDMAP_OP_BATCHED, 0, size_bucket(total / num_sets), d,
                      size_bucket(num_sets));
    ts = tuned_lookup(key);
    if (ts == 0) {
      ts = autotune({1, 64, 128}, s, run, &st);
      if (st != TDMAP_OK) return st;
      tuned_store(key, ts);
    }
  }
  TD_HIP(run(ts), "tdmap_edm_batched");
  return TDMAP_OK;
}

int tdmap_stream_fill(float *buf, uint64_t n, float value, void *stream) {
  if (n == 0) return TDMAP_OK;
  if (buf == nullptr || (reinterpret_cast<uintptr_t>(buf) & 15) != 0) return TDMAP_ERR_INVALID;
  TD_HIP(tdmap::launch_stream_fill(buf, n, value, (hipStream_t)stream), "tdmap_stream_fill");
  return TDMAP_OK;
}

int tdmap_waste_counts(int32_t strategy, int64_t N, int32_t rho, int64_t out[3]) {
  if (out == nullptr || N < 0 || rho < 1) return TDMAP_ERR_INVALID;
  return waste_closed_form(strategy, N, rho, out) ? TDMAP_OK : TDMAP_ERR_INVALID;
}

int tdmap_map_blocks_variant(uint64_t lambda0, uint64_t count, int32_t variant, uint32_t *ij,
                             void *stream) {
  if (variant < 0 || variant > 2) return TDMAP_ERR_INVALID;
  if (count == 0) return TDMAP_OK;
  if (ij == nullptr) return TDMAP_ERR_INVALID;
  if (lambda0 > ((uint64_t)1 << 32) || count > ((uint64_t)1 << 32) - lambda0)
    return TDMAP_ERR_UNSUPPORTED;
  TD_HIP(tdmap::launch_map_blocks_variant(lambda0, count, variant, ij, (hipStream_t)stream),
         "tdmap_map_blocks_variant");
  return TDMAP_OK;
}

int tdmap_dummy(int32_t strategy, int32_t variant, int64_t N, int32_t rho, uint32_t never,
                uint32_t *sink, void *stream) {
  if (sink == nullptr || N < 0) return TDMAP_ERR_INVALID;
  if (strategy < TDMAP_LTM || strategy > TDMAP_REC) return TDMAP_ERR_INVALID;
  if (variant < 0 || variant > 2 || (variant != 0 && strategy != TDMAP_LTM)) return TDMAP_ERR_INVALID;
  if (!is_cell_rho(rho)) return TDMAP_ERR_UNSUPPORTED;
  const uint64_t nb = ceil_div((uint64_t)N, (uint64_t)rho);
  if (tri(nb) > 0xffffffffull) return TDMAP_ERR_UNSUPPORTED;
  if (strategy == TDMAP_UTM && tri((uint64_t)N) > 0xffffffffull) return TDMAP_ERR_UNSUPPORTED;
  tdmap::EdmArgs a{nullptr, N, 1, 1, nullptr, 0, TDMAP_PACKED, (hipStream_t)stream};
  a.sink = sink;
  a.never = never;
  a.variant = variant;
  TD_HIP(tdmap::launch_dummy(strategy, rho, a), "tdmap_dummy");
  return TDMAP_OK;
}

int tdmap_count_waste(int32_t strategy, int64_t N, int32_t rho, uint64_t *counts, void *stream) {
  if (counts == nullptr || N < 0) return TDMAP_ERR_INVALID;
  if (strategy < TDMAP_LTM || strategy > TDMAP_REC) return TDMAP_ERR_INVALID;
  if (!is_cell_rho(rho)) return TDMAP_ERR_UNSUPPORTED;
  const uint64_t nb = ceil_div((uint64_t)N, (uint64_t)rho);
  if (tri(nb) > 0xffffffffull) return TDMAP_ERR_UNSUPPORTED;
  if (strategy == TDMAP_UTM && tri((uint64_t)N) > 0xffffffffull) return TDMAP_ERR_UNSUPPORTED;
  hipStream_t s = (hipStream_t)stream;
  TD_HIP(tdmap::launch_fill(reinterpret_cast<float *>(counts), 6, 0.0f, s), "tdmap_count_waste");
  tdmap::EdmArgs a{nullptr, N, 1, 1, nullptr, 0, TDMAP_PACKED, s};
  TD_HIP(tdmap::launch_cell(strategy, rho, a, reinterpret_cast<unsigned long long *>(counts)),
         "tdmap_count_waste");
  return TDMAP_OK;
}

}  // extern "C"
