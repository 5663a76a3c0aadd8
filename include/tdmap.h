/*
 * tdmap -- triangular-domain kernels for MI355X (gfx950): the lower-
 * triangular Euclidean distance map launched through the block map g(lambda)
 * of Navarro & Hitschfeld, "Improving the GPU space of computation under
 * triangular domain problems" (arXiv 1308.1419), next to the strategies that
 * paper compares against.
 *
 * Conventions for every entry point
 * ---------------------------------
 * - Plain C ABI.  Pointers marked "device" must point to device memory of
 *   the current HIP device; "host" pointers to host memory.  The caller owns
 *   every buffer (inputs, outputs and workspaces); the library allocates no
 *   device memory.  Its only state is the autotuner cache (host, guarded by
 *   a mutex) and a per-thread copy of the last HIP error message.
 * - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *   GPU work is enqueued asynchronously on it; no entry point synchronises
 *   the host except the autotuner on its first call for a configuration,
 *   which times candidate launches on `stream`.
 * - Every call returns a tdmap_status.  Arguments are validated before any
 *   launch; on a validation error nothing is enqueued.  A failed launch
 *   returns TDMAP_ERR_HIP and tdmap_last_error() gives the HIP message.
 *   Nothing throws across the ABI.
 * - A problem of size N has the N(N+1)/2 cells (i, j), 0 <= j <= i < N
 *   (Sec. II-A).  N = 0 is a successful no-op.
 * - Points are an N x d row-major FP32 array with row pitch ldx >= d
 *   (in elements); point i is X[i*ldx .. i*ldx + d).
 * - Output layouts:
 *     TDMAP_FULL   : N x N row-major FP32 with row pitch ldd >= N (elements);
 *                    only cells with j <= i are written, every j > i cell is
 *                    left untouched.
 *     TDMAP_PACKED : N(N+1)/2 FP32, cell (i, j) at i(i+1)/2 + j (64-bit
 *                    offsets; ldd is ignored).
 *     TDMAP_PACKED_STRICT : the problem without the diagonal (Sec. II-A,
 *                    Eq. (10)): N(N-1)/2 FP32, cell (i, j), j < i, at
 *                    i(i-1)/2 + j (64-bit offsets; ldd is ignored); this
 *                    is the row-major strictly-lower pair list, e.g. a
 *                    collision or interaction table.  With N = 1 there is
 *                    no cell and the output pointer may be NULL.
 * - Inputs and outputs must not overlap (undefined behaviour otherwise).
 */
#ifndef TDMAP_H
#define TDMAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TDMAP_OK = 0,
    TDMAP_ERR_INVALID = 1,      /* a NULL pointer, a negative size, ldx < d, ldd < N, ... */
    TDMAP_ERR_UNSUPPORTED = 2,  /* valid but not implemented (e.g. a size past 2^32 blocks) */
    TDMAP_ERR_WORKSPACE = 3,    /* workspace missing or smaller than tdmap_workspace_size */
    TDMAP_ERR_HIP = 4           /* a HIP call failed; see tdmap_last_error() */
} tdmap_status;

/* Space-of-computation strategies (Sec. II-A and Sec. III-B). */
typedef enum {
    TDMAP_LTM = 0,  /* 1D grid of exactly n(n+1)/2 blocks, block lambda -> g(lambda) (Sec. II-A, Eq. (2)) */
    TDMAP_BB = 1,   /* n x n grid, blocks above the diagonal return at once (Sec. III-B) */
    TDMAP_UTM = 2,  /* per-thread upper-triangular map of Avril et al. (Sec. III-B), half-turned */
    TDMAP_RB = 3,   /* rectangular box of Jung et al. (Sec. III-B) */
    TDMAP_REC = 4   /* recursive partition of Ries et al.: a diagonal pass + k level launches (Sec. III-B) */
} tdmap_strategy;

typedef enum { TDMAP_FULL = 0, TDMAP_PACKED = 1, TDMAP_PACKED_STRICT = 2 } tdmap_layout;

typedef enum {
    TDMAP_FP32 = 0,      /* difference form sqrt(sum_k (x_ik - x_jk)^2) in FP32 */
    TDMAP_BF16_GRAM = 1, /* ||x||^2 + ||y||^2 - 2 x.y with BF16 MFMA, FP32 accumulate,
                            FP32 difference-form recompute of near-zero distances */
    TDMAP_BF16X3_GRAM = 2 /* the same Gram form with x = hi + lo, hi = bf16(x),
                             lo = bf16(x - hi) and x.y taken as hi.hi' + hi.lo' + lo.hi'
                             (three MFMA products): representation error 2^-16 |x|
                             instead of 2^-8 |x| */
} tdmap_precision;

typedef enum {
  TDMAP_OP_EDM = 0,
  TDMAP_OP_BACKWARD = 1,
  TDMAP_OP_BATCHED = 2,
  TDMAP_OP_STRESS = 3
} tdmap_op;

/*
 * g(lambda) over a range of block indices (Sec. II-A, Eq. (2); the row is
 * i = floor(sqrt(1/4 + 2 lambda) - 1/2), the column j = lambda - i(i+1)/2).
 * The device computes a single-precision guess of i and corrects it with
 * exact integer compares (the block-level fix-up the conclusion, Sec. V,
 * says suffices while the error is at most 1), so the map is exact for
 * every lambda < 2^32.
 *   ij      device, 2*count uint32: ij[2t] = i, ij[2t+1] = j for
 *           lambda = lambda0 + t.
 * Errors: INVALID if ij is NULL while count > 0; UNSUPPORTED if
 * lambda0 + count > 2^32.
 */
int tdmap_map_blocks(uint64_t lambda0, uint64_t count, uint32_t *ij, void *stream);

/*
 * The map without the diagonal (Sec. II-A, Eq. (10)): lambda enumerates the
 * cells (i, j), 0 <= j < i, row by row, i = floor(sqrt(1/4 + 2 lambda) + 1/2)
 * and j = lambda - i(i-1)/2 (the column is taken from this enumeration's
 * row start; with i(i+1)/2 as printed it would be negative).  Same exact
 * fix-up, argument meaning and errors as tdmap_map_blocks.
 */
int tdmap_map_blocks_nodiag(uint64_t lambda0, uint64_t count, uint32_t *ij, void *stream);

/*
 * Lower-triangular Euclidean distance map D_ij = sqrt(sum_k (x_ik - x_jk)^2),
 * 0 <= j <= i < N (the EDM problem of Sec. IV, Eq. (17)), computed by the
 * chosen space-of-computation strategy.
 *   X        device, N x d FP32, row pitch ldx.
 *   D        device, output in `layout` (pitch ldd for TDMAP_FULL).
 *   strategy one of tdmap_strategy.
 *   rho      the dimensional block size (Sec. II-A):
 *              1         : (LTM, TDMAP_PACKED or TDMAP_PACKED_STRICT, D
 *                          16-byte aligned) blocks of one cell: g(lambda)
 *                          (Eq. (10) for the strict layout) maps every
 *                          packed position to its cell and the output is
 *                          written as one linear sweep, four positions per
 *                          thread;
 *              8, 16, 32 : rho x rho threads per block, one cell per thread,
 *                          as the paper launches every strategy;
 *              64, 128  : (LTM, BB) rho x rho cell tiles per 256-thread
 *                          work-group (full layout: four consecutive cells
 *                          per thread and row; packed layouts: one cell per
 *                          thread and row); LTM tiles are taken by g(lambda)
 *                          with every XCD owning one contiguous range of
 *                          lambda;
 *              256       : (LTM, BB) 256 x 256 tiles, each written by 32
 *                          work-groups of 8 rows (strips).  LTM: the tile
 *                          row comes from g(lambda) on the strip index
 *                          divided by 32, and the strips of a tile row are
 *                          taken strip by strip across the row.  Full
 *                          layout: four consecutive cells per thread and
 *                          row, 16-byte stores (D 16-byte aligned and ldd a
 *                          multiple of 4, else the 256-cell tile of the
 *                          rho = 64 / 128 form); packed layouts: four cells
 *                          64 apart per thread and row;
 *              0         : (LTM, BB) chosen by the autotuner among the
 *                          tiles (and, for LTM with a packed layout and an
 *                          aligned D, the sweep rho = 1), timed on the
 *                          first call for a (layout, strategy, d, size)
 *                          class.
 *   precision TDMAP_FP32 for every strategy; TDMAP_BF16_GRAM and
 *            TDMAP_BF16X3_GRAM only with TDMAP_LTM, TDMAP_PACKED and rho = 0,
 *            128 or 256 (128: eight-wave work-groups, each over two 128 x 128
 *            tiles side by side; 256: eight-wave work-groups, each over a
 *            32-row strip of a 256 x 256 tile, the strips of a tile row taken
 *            strip by strip across the row; 0: the autotuner's choice
 *            between the two).  Both kernels compute every 32 x 32 block with
 *            the same MFMA products in the same order, so their outputs are
 *            bitwise identical.  D may start at any 4-byte boundary.  Their
 *            error per pair that is not recomputed is at most
 *            r (|x_i| + |x_j|) + E / (D - r (|x_i| + |x_j|)) + 4 u32 D with
 *            r = 2^-8 (BF16) or 2^-16 (BF16X3), u32 = 2^-24 and E the FP32
 *            accumulation bound 2 (m d + 4) u32 (|x_i|^2 + |x_j|^2)(1 + 2^-8)^2
 *            (m = 1 or 3; BF16X3 adds 2^-15 (1 + 2^-8)^2 |x_i| |x_j| for the
 *            dropped lo.lo'); pairs with G <= (n_i + n_j)/4 are recomputed in
 *            FP32 difference form and meet the FP32 rule below.
 *   layout   TDMAP_PACKED_STRICT only with TDMAP_FP32, LTM or BB and
 *            rho = 0, 1 (LTM), 64, 128 or 256.
 *   workspace device scratch of at least
 *            tdmap_workspace_size(TDMAP_OP_EDM, N, d, 0, rho, precision)
 *            bytes, 16-byte aligned (0 for TDMAP_FP32; may then be NULL).
 * Every strategy writes the same cells with the same per-pair arithmetic,
 * so their outputs are bitwise identical.  FP32 results are within a
 * relative 1e-6 of the exact distance of the FP32 inputs (squared distances
 * below 2^-126 excepted), and exactly 0 where x_i == x_j.
 * Errors: INVALID for NULL pointers, N < 0, d < 1, ldx < d, ldd < N (FULL),
 * an unknown enum or a Gram workspace that is not 16-byte aligned;
 * UNSUPPORTED for a (strategy, rho, precision, layout) combination listed
 * above as unavailable, d > 4 with tiled rho, or sizes past the 32-bit block
 * index; WORKSPACE if the workspace is too small.
 */
int tdmap_edm(const float *X, int64_t N, int32_t d, int64_t ldx,
              float *D, int64_t ldd, int32_t layout, int32_t strategy,
              int32_t rho, int32_t precision,
              void *workspace, size_t ws_bytes, void *stream);

/*
 * One shard of tdmap_edm, the per-device share of a run split over
 * num_shards devices (or streams): with tdmap_edm's arguments it writes only
 * the cells of the blocks whose index lies in
 *   [shard * W / num_shards, (shard + 1) * W / num_shards)
 * of the launch's block index space of W blocks.  The blocks are placed by
 * g(lambda) (Sec. II-A, Eq. (2)), so the shards are equal to one block and
 * need no exchange; the union of all shards' writes is tdmap_edm's output
 * for the same kernel, bit for bit, and different shards write disjoint
 * cells.  Every shard must cut the same block space, so the kernel is named:
 *   strategy  TDMAP_LTM.
 *   rho       TDMAP_FP32: 64, 128 or 256 (the tiles and strips of tdmap_edm,
 *             d <= 4); the Gram precisions: 128 or 256.
 *   shard, num_shards  0 <= shard < num_shards.
 * A Gram shard rounds the whole of X to BF16 into its own workspace.
 * Errors: as tdmap_edm; INVALID for a bad shard or num_shards; UNSUPPORTED
 * for another strategy, rho 0, 1, 8, 16 or 32.
 */
int tdmap_edm_shard(const float *X, int64_t N, int32_t d, int64_t ldx,
                    float *D, int64_t ldd, int32_t layout, int32_t strategy,
                    int32_t rho, int32_t precision, void *workspace, size_t ws_bytes,
                    int32_t shard, int32_t num_shards, void *stream);

/*
 * Instrumented Gram-form EDM: the launch tdmap_edm makes for the same
 * arguments (precision TDMAP_BF16_GRAM or TDMAP_BF16X3_GRAM, layout
 * TDMAP_PACKED, strategy TDMAP_LTM; rho 128 or 256 picks the kernel, 0 the
 * autotuner's choice, or 256 if that configuration is not tuned yet), with
 * the same output, that also counts the pairs (i, j), j <= i < N, which took
 * the FP32 difference-form recompute (G <= (n_i + n_j)/4).  It reports the
 * size of the recompute path on a workload; it is a separate build of the
 * kernel (one atomic add per wave that recomputes), never the one timed.
 *   count  device, one uint64, overwritten.
 * Other arguments and errors as for tdmap_edm; INVALID for a NULL count.
 */
int tdmap_gram_recompute_count(const float *X, int64_t N, int32_t d, int64_t ldx,
                               float *D, int32_t precision, int32_t rho,
                               void *workspace, size_t ws_bytes, uint64_t *count,
                               void *stream);

/*
 * The Gram-form EDM without a workspace argument, for callers that cannot
 * allocate device memory: code under stream capture, serving loops and
 * harnesses that forbid allocation.  It computes what tdmap_edm computes
 * for the same X, N, d, ldx, D, precision and rho with layout TDMAP_PACKED
 * and strategy TDMAP_LTM (the same kernels, bitwise the same output), but
 * keeps the BF16 copy of the points and their norms in a static device
 * array of TDMAP_NOALLOC_SCRATCH_BYTES that each GPU holds from the
 * library's first call there until the process ends.  It allocates no
 * memory and makes no allocating call.
 *   X, N, d, ldx, D  as for tdmap_edm (D packed, any 4-byte alignment).
 *   precision        TDMAP_BF16_GRAM or TDMAP_BF16X3_GRAM.
 *   rho              128 or 256 picks the kernel; 0 takes the autotuner's
 *                    decision if tdmap_edm has already tuned this
 *                    configuration, else 256.  It never times candidates.
 * Every call on one GPU uses that GPU's one array, which keeps the last
 * call's contents: calls that can overlap on one GPU (several streams or
 * host threads) race on it and must be serialised by the caller.
 * Errors: INVALID as for tdmap_edm or for another precision; UNSUPPORTED for
 * rho other than 0, 128, 256, for sizes past the kernels' 32-bit block
 * index, or when tdmap_workspace_size(TDMAP_OP_EDM, N, d, 0, rho,
 * precision) exceeds TDMAP_NOALLOC_SCRATCH_BYTES (32 MiB: N = 100000 with
 * d = 64 fits in both precisions); HIP if the array's device address cannot
 * be taken or a launch fails.
 */
#define TDMAP_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int tdmap_edm_gram_noalloc(const float *X, int64_t N, int32_t d, int64_t ldx,
                           float *D, int32_t precision, int32_t rho, void *stream);

/*
 * Gradient through the EDM: given dD_ij = dL/dD_ij for the cells of the
 * triangle, writes dX_i = sum_{j<i} dD_ij (x_i - x_j)/D_ij
 *                       - sum_{k>i} dD_ki (x_k - x_i)/D_ki,
 * a term being 0 where D = 0 (for finite dD); diagonal cells of dD are
 * ignored.  The tiles are enumerated by g(lambda) as in the forward map.
 * This operation is not in the paper; it differentiates the EDM of Sec. IV,
 * Eq. (17).
 *   X      device, N x d FP32, pitch ldx.    dD device, `layout` (pitch ldd;
 *          any of the three layouts).
 *   dX     device, N x d FP32, row pitch d, overwritten.
 *   rho    tile edge: 0 (autotuned), 64, 128 or 256.
 *   deterministic  1: per-tile partial sums in the workspace, reduced in a
 *          fixed order (bitwise reproducible); 0: partial sums added with
 *          atomics (no workspace, order-dependent last bits).
 *   workspace  device, tdmap_workspace_size(TDMAP_OP_BACKWARD, N, d, 0, rho,
 *          deterministic) bytes (0 when deterministic = 0).
 * d must be 1..4.  Errors as for tdmap_edm.
 */
int tdmap_edm_backward(const float *X, int64_t N, int32_t d, int64_t ldx,
                       const float *dD, int64_t ldd, int32_t layout,
                       float *dX, int32_t rho, int32_t deterministic,
                       void *workspace, size_t ws_bytes, void *stream);

/*
 * Stress loss and its gradient in one pass over the targets:
 *   L = sum_{j<i} (D_ij - delta_ij)^2,
 *   dX = the gradient above with dD_ij = 2 (D_ij - delta_ij),
 * D being the EDM of X (Sec. IV, Eq. (17)) computed inside the tiles and
 * never stored.  The tiles are enumerated by g(lambda) as in the forward
 * map.  This operation is not in the paper: it is the fitting objective of
 * metric multidimensional scaling over the triangle the paper maps.
 *   X      device, N x d FP32, pitch ldx.
 *   delta  device, targets in `layout` (pitch ldd); diagonal cells and the
 *          upper triangle of the full layout are not read into the sum.
 *   dX     device, N x d FP32, row pitch d, overwritten.
 *   loss   device, one FP32, overwritten with L (0 when N <= 1).
 *   rho    tile edge: 0 (autotuned), 64, 128 or 256.
 *   deterministic  1: per-tile partial gradients and losses in the
 *          workspace, reduced in a fixed order (bitwise reproducible);
 *          0: atomics (no workspace).
 *   workspace  device, tdmap_workspace_size(TDMAP_OP_STRESS, N, d, 0, rho,
 *          deterministic) bytes (0 when deterministic = 0).
 * d must be 1..4.  Errors as for tdmap_edm_backward; `loss` must be
 * non-NULL.
 */
int tdmap_stress_backward(const float *X, int64_t N, int32_t d, int64_t ldx,
                          const float *delta, int64_t ldd, int32_t layout,
                          float *dX, float *loss, int32_t rho,
                          int32_t deterministic, void *workspace,
                          size_t ws_bytes, void *stream);

/*
 * Many independent EDMs in one persistent launch (not in the paper; each
 * set is the EDM of Sec. IV on its own points).  Set s owns points
 * X_cat[point_off[s] .. point_off[s+1]) and writes its packed triangle at
 * D_cat + out_off[s].  The work-groups walk the concatenation of every
 * set's g(lambda) tile space (a prefix sum of n_s(n_s+1)/2 block counts).
 *   X_cat      device, (point_off[S]) x d FP32, pitch d.
 *   point_off  device, S+1 int64, non-decreasing, point_off[0] = 0.
 *   out_off    device, S+1 int64, out_off[s+1] - out_off[s] =
 *              n_s(n_s+1)/2 with n_s = point_off[s+1] - point_off[s];
 *              out_off[0] may be above 0 (D_cat[0 .. out_off[0]) is not
 *              written).
 *   rho        1: one-cell blocks: a persistent grid sweeps the
 *              concatenated packed output; each work-group owns one
 *              contiguous stretch of 16384-position chunks and reads a set's
 *              points from LDS (sets of up to 16384 / d points; larger sets
 *              read global memory);
 *              64 or 128: a persistent grid walks TS x TS tiles in
 *              contiguous ranges;
 *              0: autotuned.
 *   workspace  device, tdmap_workspace_size(TDMAP_OP_BATCHED, 0, d, S, rho, 0)
 *              bytes.
 * The offsets are not read on the host, except that rho = 0 reads
 * point_off[num_sets] back (one synchronisation of `stream`) to key the
 * autotuner on the mean set size as well as on num_sets; pass rho to avoid
 * it.  X_cat and D_cat must be non-NULL whenever num_sets > 0, even if every
 * set is empty; inconsistent offsets are undefined behaviour.  d must be
 * 1..4.  Errors as for tdmap_edm.
 */
int tdmap_edm_batched(const float *X_cat, int32_t d, int32_t num_sets,
                      const int64_t *point_off, const int64_t *out_off,
                      float *D_cat, int32_t rho,
                      void *workspace, size_t ws_bytes, void *stream);

/* Bytes of device workspace an operation needs (0 if none).  `flags` is the
 * precision for TDMAP_OP_EDM, `deterministic` for TDMAP_OP_BACKWARD and
 * TDMAP_OP_STRESS, and unused for TDMAP_OP_BATCHED.  Pure host arithmetic. */
size_t tdmap_workspace_size(int32_t op, int64_t N, int32_t d, int32_t num_sets,
                            int32_t rho, int32_t flags);

/*
 * Write-stream reference for the roofline: sets buf[0 .. n) to `value` with
 * one 16-byte non-temporal store per thread, consecutive threads on
 * consecutive chunks.  Not part of the paper's method; it measures the
 * store rate the device reaches on a plain linear stream, against which the
 * EDM's store rate is read.
 *   buf  device, 16-byte aligned, n floats.
 * Errors: INVALID for a NULL or misaligned buf with n > 0.
 */
int tdmap_stream_fill(float *buf, uint64_t n, float value, void *stream);

/*
 * Launch statistics of a strategy, in closed form (host only): out[0] =
 * blocks launched, out[1] = fully idle blocks (blocks that write no cell),
 * out[2] = idle threads (threads that write no cell), for the one-cell-per-
 * thread launch with rho x rho blocks.  Sec. II-A: BB leaves n(n-1)/2 blocks
 * idle, LTM none (its idle threads are the upper halves of the n diagonal
 * blocks, about n/2 block equivalents).
 * Errors: INVALID for a NULL out, N < 0, rho < 1 or an unknown strategy.
 */
int tdmap_waste_counts(int32_t strategy, int64_t N, int32_t rho, int64_t out[3]);

/*
 * The same statistics counted on the device by an instrumented variant of
 * the strategy's kernel (it evaluates the map and filters exactly as the
 * timed kernel does, and counts instead of storing).
 *   counts  device, 3 uint64 (blocks, fully idle blocks, idle threads),
 *           overwritten.
 * rho must be 8, 16 or 32.
 */
int tdmap_count_waste(int32_t strategy, int64_t N, int32_t rho,
                      uint64_t *counts, void *stream);

/*
 * The same map under the paper's three ways of taking the row (Sec. III-A),
 * for measuring their accuracy: variant 0 is the exact map above; 1 is
 * LTM-X, floor(sqrtf(1/4 + 2 lambda) - 1/2) with the default single-precision
 * square root; 2 is LTM-R, sqrt(x) = x * rsq(x) (Eq. (16)) with
 * epsilon = 1e-4 added before the floor.  Variants 1 and 2 are not corrected:
 * past some lambda they can name the wrong row (and j is then computed from
 * that row's start, wrapping as an unsigned value).
 * Errors: INVALID for an unknown variant or a NULL ij; UNSUPPORTED past 2^32.
 */
int tdmap_map_blocks_variant(uint64_t lambda0, uint64_t count, int32_t variant, uint32_t *ij,
                             void *stream);

/*
 * The paper's dummy kernel (Sec. III-A, Sec. IV): the strategy's launch with
 * rho x rho blocks where every thread only computes its cell (i, j) and
 * applies the strategy's filters.  It measures the cost of the space of
 * computation itself.  The paper writes i + j to a fixed address; here the
 * write happens only when i + j equals `never` (pass a value no cell has,
 * e.g. 0xffffffff), which keeps the map live without every thread storing to
 * one address.  `variant` selects the LTM row computation as in
 * tdmap_map_blocks_variant (must be 0 for other strategies).
 *   sink  device, one uint32 (written only if some cell has i + j == never).
 * rho must be 8, 16 or 32.  Nothing else is written.
 */
int tdmap_dummy(int32_t strategy, int32_t variant, int64_t N, int32_t rho, uint32_t never,
                uint32_t *sink, void *stream);

/* Tile edge the autotuner has chosen for a call with rho = 0, or 0 if that
 * configuration has not been tuned yet.  `strategy` and `layout` are those
 * of the call (ignored for TDMAP_OP_BACKWARD, TDMAP_OP_STRESS and
 * TDMAP_OP_BATCHED, except as below); `size`
 * is N for TDMAP_OP_EDM, TDMAP_OP_BACKWARD and
 * TDMAP_OP_STRESS, and num_sets for TDMAP_OP_BATCHED, whose `layout` is
 * the mean set size in points (point_off[num_sets] / num_sets, rounded
 * down; the key takes ceil(log2) of it).  Decisions are cached per
 * (op, strategy, layout, d, ceil(log2(size))); for TDMAP_OP_EDM an
 * output that is not 16-byte aligned (or a full-layout pitch that is not a
 * multiple of 4) is tuned apart, under layout + 64, the Gram precisions
 * under layout 256 + precision. */
int32_t tdmap_tuned_rho(int32_t op, int32_t strategy, int32_t layout, int32_t d, int64_t size);

/* Forget every autotuner decision. */
void tdmap_autotune_reset(void);

/* Static description of a status code (never NULL). */
const char *tdmap_status_string(int32_t status);

/* Message of the last HIP failure on the calling thread ("" if none). */
const char *tdmap_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TDMAP_H */
