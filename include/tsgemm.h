/*
 * tsgemm.h -- C ABI of libtsgemm, tall & skinny matrix products on AMD
 * Instinct MI355X (gfx950).
 *
 * The two products follow the problem statement of Ernst, Hager, Thies and
 * Wellein, "Performance Engineering for Real and Complex Tall & Skinny Matrix
 * Multiplication Kernels on GPUs" (arXiv 1905.03136), Section 1.1:
 *   A is K x M and B is K x N ("tall": K is the long dimension, "skinny":
 *   M, N in [1, 64]); C is the small M x N matrix.
 *   TSMTTSM:  C = A^T B          TSMM:  B = A C
 * on row-major block vectors (Section 1.2: one row of a block vector holds
 * one entry of each of its vectors), in real (D) and complex (Z) double
 * precision.
 *
 * Layout (all matrices row-major, leading dimensions count ELEMENTS):
 *   A(k, m) = A[k * lda + m],  B(k, n) = B[k * ldb + n],  C(m, n) = C[m * ldc + n]
 * Complex elements are interleaved (re, im) pairs of the storage type.
 *
 * Conventions shared by every entry point:
 *  - Pointers to matrices are DEVICE pointers owned by the caller; the library
 *    never frees or retains them.  `stream` is a hipStream_t (NULL = the null
 *    stream).
 *  - Calls are stream-ordered and asynchronous: they return once the work is
 *    enqueued.  A kernel fault surfaces at the caller's next synchronisation.
 *  - All arguments are validated on the host before any HIP call; invalid
 *    arguments return TSG_E_ARG or TSG_E_UNSUPPORTED and enqueue nothing.
 *  - Every result is deterministic: the same inputs on the same device give
 *    the same bits, run after run (the cross-block reduction has a fixed
 *    order).
 *  - The library owns a per-(device, stream) workspace that it allocates on
 *    first need (hipMalloc) and keeps until tsg_finalize().  Growing it while
 *    the stream is being captured into a graph is impossible and returns
 *    TSG_E_CAPTURE; call the operation once outside capture (or tsg_reserve)
 *    first.  Calls that run concurrently on different streams use different
 *    workspaces; calls on one stream are ordered by the stream.  A workspace
 *    that a later call outgrows is retired, not freed, until tsg_finalize(),
 *    so a graph that captured it stays valid.  A captured TSMTTSM writes its
 *    partial sums into the capture stream's workspace whichever stream the
 *    graph is replayed on: replays must not overlap in time with calls on
 *    the capture stream or with replays of other graphs captured there.
 *  - No C++ exception crosses this interface.  tsg_last_error() gives a
 *    thread-local text for the last non-OK status of the calling thread.
 */
#ifndef TSGEMM_H
#define TSGEMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Storage type of the tall matrices A and B, and the arithmetic.
 * TSG_R64 / TSG_C128 are the paper's D and Z types (Section 1.1).
 * The other four are the precision form: A and B are stored in binary32
 * (real, or complex as two binary32; half the HBM traffic) while the small
 * matrix C stays binary64 / complex128.  TSG_R32 / TSG_C64 compute in
 * binary64 on the exactly widened values; TSG_R32_ACC32 / TSG_C64_ACC32
 * form the products in binary32 and sum them in binary32 over stretches of
 * at most 32 rows, all further sums (over stretches, threads, blocks) in
 * binary64 -- see tsg_tsmttsm and tsg_tsmm for the error of each. */
typedef enum {
    TSG_R64 = 0,
    TSG_C128 = 1,
    TSG_R32 = 2,
    TSG_C64 = 3,
    TSG_R32_ACC32 = 4,
    TSG_C64_ACC32 = 5
} tsg_dtype;

/* op(A) of TSMTTSM: the transpose, or for complex types the conjugate
 * transpose (the Hermitian product A^H B that Gram-Schmidt orthogonalisation
 * needs, Section 1.2).  TSG_OP_C on a real type is the same as TSG_OP_T.
 * TSG_OP_N (no transpose) is only meaningful for TSMM's small operand, see
 * tsg_tsmm_op. */
typedef enum {
    TSG_OP_T = 0,
    TSG_OP_C = 1,
    TSG_OP_N = 2
} tsg_op;

typedef enum {
    TSG_OK = 0,
    TSG_E_ARG = 1,          /* invalid argument (sizes, strides, pointers, alignment) */
    TSG_E_UNSUPPORTED = 2,  /* valid but outside the supported range (M or N > 64)    */
    TSG_E_NOMEM = 3,        /* workspace allocation failed or exceeds TSG_MAX_WORKSPACE */
    TSG_E_HIP = 4,          /* a HIP runtime call failed (no device, launch failure)  */
    TSG_E_CAPTURE = 5       /* workspace must grow while the stream is being captured */
} tsg_status;

/*
 * TSMTTSM (Section 3; Listing 1 defines the sum):
 *   C[m * ldc + n] = sum_{k=0}^{K-1} op(A(k, m)) * B(k, n),   0 <= m < M, 0 <= n < N
 * C is overwritten (never read).  K = 0 writes zeros.
 *
 * dt       storage type of A and B.  C is double (real types) or
 *          interleaved complex double (complex types).
 * op       TSG_OP_T or TSG_OP_C (conjugates A; complex types only).
 * K        rows of A and B, K >= 0 (64-bit; any size that fits in memory).
 * M, N     columns of A and B, 1 <= M, N <= 64 (else TSG_E_UNSUPPORTED).
 * A, lda   device pointer and leading dimension, lda >= M.
 * B, ldb   device pointer and leading dimension, ldb >= N.
 * C, ldc   device pointer and leading dimension, ldc >= N.
 * Pointers must be aligned to the storage element size (8 B for TSG_R64,
 * 16 B for TSG_C128, 4 B for TSG_R32 and TSG_R32_ACC32, 8 B for TSG_C64 and
 * TSG_C64_ACC32) and may be NULL only when K == 0 (A, B).  C must not
 * overlap A or B.
 *
 * Arithmetic: binary64 fused multiply-adds for TSG_R64 / TSG_C128.  For the
 * precision form (TSG_R32 / TSG_C64) the binary32 values are widened exactly
 * to binary64; a product of two of them has at most 48 significant bits and
 * is therefore formed exactly (error-free, as a compensated product would
 * make it), and the products are accumulated in binary64, as is the
 * reduction across threads and blocks.  The result differs from the binary64
 * sum of the stored binary32 values only by binary64 rounding.
 * TSG_R32_ACC32 / TSG_C64_ACC32: binary32 products summed in binary32 over
 * stretches of at most 32 rows of a thread, each stretch sum then added in
 * binary64; every entry is within c 2^-24 sum_k |op(a_km)| |b_kn| of the
 * exact sum of the stored values (|.| the modulus for complex values),
 * c = 34 (real) or 66 (each part of a complex entry, which sums two real
 * products per row).  Complex kernels in Gauss's three-product form (binary32
 * sums of Ar Br, Ai Bi and (Ar + Ai)(Br + Bi), combined in binary64) give
 * c = 34 for the real part and c = 106 for the imaginary part, which cancels
 * where the parts of the data do.  Where binary64 arithmetic on the widened
 * values is as fast, the library uses it instead (more accurate, within the
 * same bound).
 */
tsg_status tsg_tsmttsm(tsg_dtype dt, tsg_op op, int64_t K, int32_t M, int32_t N,
                       const void *A, int64_t lda, const void *B, int64_t ldb,
                       void *C, int64_t ldc, void *stream);

/*
 * TSMTTSM that allocates nothing, for callers that cannot call hipMalloc:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Same operation, arguments, validation and kernels as
 * tsg_tsmttsm (so the same bits), but the per-block partial sums go to a
 * fixed scratch array of 32 MiB that the library holds on each device for
 * the life of the process, instead of the per-stream workspace.
 *  - Its device address is resolved once per device, by tsg_init(device) or
 *    by the first call on that device; neither allocates.
 *  - A call whose partial sums would exceed the 32 MiB returns
 *    TSG_E_UNSUPPORTED and enqueues nothing.  (The library sizes
 *    every TSMTTSM grid so that its partial sums, one slot of M N (x2
 *    complex) doubles per block, fit in the 32 MiB, so no shape of the
 *    supported range is refused.)
 *  - Every call on one device shares that device's scratch and leaves its
 *    partial sums there: calls that overlap in time on one device (different
 *    streams, or host threads) race and give wrong results.  Order them on
 *    one stream, or use tsg_tsmttsm.  Nothing in the scratch needs to start
 *    at zero (each block writes its whole slot before the fold reads it).
 */
tsg_status tsg_tsmttsm_noalloc(tsg_dtype dt, tsg_op op, int64_t K, int32_t M, int32_t N,
                               const void *A, int64_t lda, const void *B, int64_t ldb,
                               void *C, int64_t ldc, void *stream);

/*
 * TSMM (Section 4):
 *   B(k, n) = alpha * sum_{m=0}^{M-1} opA(A(k, m)) * C[m * ldc + n] + beta * B(k, n)
 * opA conjugates A when conjA != 0 (complex types only).  alpha and beta are
 * real.  beta == 0 means B is not read (NaNs in B do not propagate); the
 * paper's TSMM is alpha = 1, beta = 0.
 *
 * dt       storage type of A and B; C is double / complex double as above.
 * K        rows of A and B, K >= 0; K = 0 does nothing.
 * M, N     1 <= M, N <= 64.
 * A, lda   lda >= M.     C, ldc  ldc >= N (C is M x N).     B, ldb  ldb >= N.
 * Alignment as for tsg_tsmttsm.  B must not overlap A or C.
 *
 * Arithmetic: binary64 fused multiply-adds; for TSG_R32 / TSG_C64 the
 * binary32 inputs are widened exactly, the sum over m is taken in binary64
 * and the result is rounded once to binary32.  TSG_R32_ACC32 /
 * TSG_C64_ACC32: C is rounded to binary32 and the sum over m (at most 64
 * products) taken in binary32, alpha and beta B in binary64, the result
 * rounded once to binary32: within (M + 3) 2^-24 sum_m |a_km| |c_mn| plus
 * one binary32 rounding of the result (per real part; complex: 2M + 3, or
 * with Gauss's three-product form M + 3 for the real part and 3M + 13 for
 * the imaginary part).
 */
tsg_status tsg_tsmm(tsg_dtype dt, int32_t conjA, int64_t K, int32_t M, int32_t N,
                    const void *A, int64_t lda, const void *C, int64_t ldc,
                    void *B, int64_t ldb, double alpha, double beta, void *stream);

/*
 * TSMM with an operation on the small matrix:
 *   B(k, n) = alpha * sum_m opA(A(k, m)) * opC(C)(m, n) + beta * B(k, n)
 * opC = TSG_OP_N: opC(C)(m, n) = C[m * ldc + n]   (C stored M x N, ldc >= N);
 * opC = TSG_OP_T: opC(C)(m, n) = C[n * ldc + m]   (C stored N x M, ldc >= M);
 * opC = TSG_OP_C: conj(C[n * ldc + m])            (complex; real types as T).
 * The transposed forms are what the gradients of TSMTTSM need
 * (dA = B dC^T, dA = B dC^H); the small matrix is transposed while it is
 * staged on chip, so no copy of it is made.  Otherwise as tsg_tsmm, which
 * equals tsg_tsmm_op with TSG_OP_N.
 */
tsg_status tsg_tsmm_op(tsg_dtype dt, int32_t conjA, tsg_op opC, int64_t K, int32_t M, int32_t N,
                       const void *A, int64_t lda, const void *C, int64_t ldc,
                       void *B, int64_t ldb, double alpha, double beta, void *stream);

/* ---- batched block orthogonalisation (one persistent launch) ----
 * Classical Gram-Schmidt of a block W against an orthonormal basis V needs
 * both products (Section 1.2): C = V^T W, then W <- W - V C.  The batched form
 * runs that step for `count` independent instances (real binary64; each with
 * its own K_i, M_i <= 64, N_i <= 16; 1 <= count <= 1024) in ONE persistent
 * kernel launch over a device work queue.  A one-block set-up kernel builds
 * the queue on the device: instances ordered by decreasing input size
 * K_i (M_i + N_i), each cut into K-slab items (TSMTTSM partial sums of about
 * 4 MiB of input, at most 256 per instance) followed, one instance later,
 * by its row-slab items (the TSMM update).  The last slab item of an
 * instance to finish folds the instance's partials in slab order into C_i
 * and marks it ready; an update item starts once its instance is ready.
 * Every item an update waits for precedes it in the queue and never waits
 * itself, so the launch cannot deadlock.  Results are deterministic: the
 * slab boundaries and every summation order are fixed by the queue, not by
 * which block takes which item.  C_i is computed in binary64 by matrix-core
 * products of four rows, summed over the slab's rows, then over slabs in
 * order; the update is W <- W + V (-C) with the same products.
 *
 * Descriptor of instance i (all device pointers, row-major):
 *   V (K x M, ldv >= M) read only; W (K x N, ldw >= N) updated in place;
 *   C (M x N, ldc >= N) written with V^T W of the OLD W.  W must not overlap
 *   V or C, and instances must not overlap each other's W or C. */
typedef struct {
    int64_t K;
    int32_t M, N;
    const double *V;
    int64_t ldv;
    double *W;
    int64_t ldw;
    double *C;
    int64_t ldc;
} tsg_orth_desc;

typedef struct tsg_orth_plan_t *tsg_orth_plan;

/*
 * One batched orthogonalisation step (Section 1.2) for `count` instances
 * whose descriptors lie in DEVICE memory (d_descs, 8-byte aligned, read by
 * the set-up kernel on the stream, so they may be written by earlier work on
 * the same stream).  `workspace` is caller-owned device memory of ws_bytes
 * bytes, 256-byte aligned; tsg_workspace_size(TSG_KIND_ORTH, TSG_R64, K, M,
 * N, count) gives enough for any `count` instances with K_i <= K, M_i <= M
 * and N_i <= N and contiguous rows.  Two kernel launches on `stream` (the
 * set-up kernel, then the persistent kernel); no allocation, no host
 * synchronisation, so the call can be captured into a graph and replayed.
 * The workspace holds the queue and partial sums of one call: calls that
 * share a workspace must not overlap in time.
 * Host-side errors (nothing enqueued): TSG_E_ARG (null pointers, count < 1,
 * misaligned workspace or descriptors, ws_bytes below the queue's own
 * size), TSG_E_UNSUPPORTED (count > 1024), TSG_E_HIP.  Device-side checks of
 * the descriptors (as listed for tsg_orth_plan_create) and of the workspace
 * capacity leave every C_i and W_i untouched and are reported by
 * tsg_orth_batched_check.
 */
tsg_status tsg_orth_batched(const tsg_orth_desc *d_descs, int32_t count, void *workspace, size_t ws_bytes,
                            void *stream);
/* Waits for the device, then reports the outcome of the last tsg_orth_batched
 * call on `workspace` and clears it: TSG_OK; TSG_E_ARG (a descriptor failed
 * the device-side checks: nothing was done); TSG_E_NOMEM (the batch needs
 * more workspace: nothing was done); TSG_E_HIP (an update waited past its
 * spin limit: results invalid). */
tsg_status tsg_orth_batched_check(void *workspace);

/* Build a plan for `count` instances (1..1024; host array of descriptors,
 * read only during the call) on the current device: validates them on the
 * host, allocates the plan's workspace, uploads the descriptors, runs the
 * set-up kernel once (queue as for tsg_orth_batched) and captures one launch
 * of the persistent kernel into a hipGraph on a private stream.
 * rows_per_item > 0 fixes the slab height of every instance; <= 0 picks it
 * per instance (about 4 MiB of input per slab, at most 256 slabs per
 * instance) and cuts the updates at the end of the queue into half and
 * quarter slabs.
 * Errors: TSG_E_ARG (null plan/descs, count < 1, K_i < 0, M_i or N_i < 1,
 * ld too small, null or misaligned pointer with K_i > 0, null C_i),
 * TSG_E_UNSUPPORTED (count > 1024, M_i > 64, N_i > 16, slab height too large
 * for the leading dimensions), TSG_E_NOMEM, TSG_E_HIP.  Allocates: never
 * call it while a stream is being captured.  `stream` is unused (reserved). */
tsg_status tsg_orth_plan_create(tsg_orth_plan *plan, int32_t count, const tsg_orth_desc *descs,
                                int64_t rows_per_item, void *stream);
/* Replay the plan's graph on `stream` (a stream of the plan's device;
 * asynchronous).  Launches of one plan must not overlap: they share its
 * counters. */
tsg_status tsg_orth_plan_launch(tsg_orth_plan plan, void *stream);
/* Launch the persistent kernel directly (no graph) on `stream`; may itself be
 * captured by the caller.  Same ordering rule as tsg_orth_plan_launch. */
tsg_status tsg_orth_plan_run(tsg_orth_plan plan, void *stream);
/* Waits for the device, then returns TSG_OK, or TSG_E_HIP if a wait of an
 * update item for its instance's C_i ran past the spin limit in a launch since
 * the last check (the results of that launch are then invalid); clears the
 * flag. */
tsg_status tsg_orth_plan_check(tsg_orth_plan plan);
/* Bound on the sleeps (about 0.2 us each) of one wait; default 2^23.  Stored
 * on the device, so it applies to graph replays too.  Waits for the device
 * first.  Meant for tests of the error path: 0 makes every update item give
 * up at once and raise the flag (its results are then invalid). */
tsg_status tsg_orth_plan_set_spin_limit(tsg_orth_plan plan, uint32_t limit);
/* Waits for the device, then frees the plan (null is ignored). */
void tsg_orth_plan_destroy(tsg_orth_plan plan);

/* Make sure the workspace of (current device, stream) can serve a TSMTTSM of
 * this shape without allocating, e.g. before capturing the stream into a
 * graph.  May allocate (hipMalloc); returns TSG_E_CAPTURE if the stream is
 * being captured and the workspace is too small. */
tsg_status tsg_reserve(tsg_dtype dt, int64_t K, int32_t M, int32_t N, void *stream);

/* Operations whose workspace tsg_workspace_size reports. */
typedef enum {
    TSG_KIND_TSMTTSM = 0,  /* tsg_tsmttsm: per-block partial sums of one launch        */
    TSG_KIND_TSMM = 1,     /* tsg_tsmm: none (0 bytes)                                 */
    TSG_KIND_ORTH = 2      /* tsg_orth_batched: queue and partial sums of one call     */
} tsg_op_kind;

/* Bytes of workspace an operation uses on the current device:
 * TSG_KIND_TSMTTSM: a TSMTTSM of shape (K, M, N) and storage type dt (count
 * ignored) -- what tsg_tsmttsm keeps per stream and tsg_tsmttsm_noalloc
 * needs of its scratch;  TSG_KIND_TSMM: 0;  TSG_KIND_ORTH (dt = TSG_R64): a
 * tsg_orth_batched call of `count` instances with K_i <= K, M_i <= M,
 * N_i <= N.  Returns 0 for shapes outside the supported range. */
size_t tsg_workspace_size(int32_t op_kind, tsg_dtype dt, int64_t K, int32_t M, int32_t N, int32_t count);

/* Optional set-up for `device` (queries device properties); calls do it
 * lazily otherwise.  Returns TSG_E_HIP without a usable device. */
tsg_status tsg_init(int32_t device);

/* Free every workspace of every device.  No call may be in flight. */
void tsg_finalize(void);

/* Static text for a status code. */
const char *tsg_status_string(tsg_status s);

/* Thread-local description of the calling thread's last error ("" if none). */
const char *tsg_last_error(void);

/* Name of the kernel variant the library would launch for this problem with
 * contiguous rows (lda = M, ldb = N) and 16-byte aligned operands
 * (diagnostics and profiling).  op_kind: 0 = TSMTTSM, 1 = TSMM.  Returns a
 * static string, "" if the shape is invalid. */
const char *tsg_kernel_name(int32_t op_kind, tsg_dtype dt, int32_t conj, int32_t M, int32_t N);

/* ---- bandwidth probes (define the achievable bandwidth b_s of the roofline) ----
 * The paper measures b_s with a read-only thread-local sum (the TSMTTSM
 * pattern) and a read + write stream (the TSMM pattern), Section 1.6, Table 1.
 * tsg_stream_read reads `bytes` from device pointer x; tsg_stream_copy copies
 * `bytes` from src to dst (non-overlapping).  Pointers must be 16-byte aligned
 * and bytes a multiple of 16 (else TSG_E_ARG).  Asynchronous on `stream`; time
 * them with events.  tsg_stream_read keeps a small internal sink buffer. */
tsg_status tsg_stream_read(const void *x, size_t bytes, void *stream);
tsg_status tsg_stream_copy(const void *src, void *dst, size_t bytes, void *stream);

/* The grid of Table 1 (Section 1.6): bandwidth against occupancy and loads in
 * flight, extended by a write stream.  Reads x in chunks of 256 threads x
 * loads_in_flight (1, 2, 4, 8 or 16) 16-byte non-temporal loads issued
 * together, and per chunk writes its share of y (y_bytes / chunks, from the
 * loaded values; stream_stores != 0: non-temporal stores, else cached), so
 * y_bytes : x_bytes sets the write:read ratio (0: read only, as Table 1).
 * blocks_per_cu (1..32) blocks of 256 threads per compute unit set the
 * occupancy.  *moved (may be NULL) receives the bytes read and written.
 * x, y device pointers, 16-byte aligned; x_bytes must cover one chunk.
 * Asynchronous; time it with events.  TSG_E_ARG on invalid arguments. */
tsg_status tsg_stream_probe(const void *x, size_t x_bytes, void *y, size_t y_bytes, int32_t blocks_per_cu,
                            int32_t loads_in_flight, int32_t stream_stores, size_t *moved, void *stream);

/* Peak arithmetic rates (Section 1.6 computes the FP64 peak from the clock
 * and unit counts; these measure it): register-only loops with independent
 * accumulator chains on the matrix cores (binary64 or binary32 16x16x4
 * products), on the vector unit (binary64 FMA), or both from the same waves.
 * blocks_per_cu (1..32) blocks of 256 threads per compute unit, `iters` loop
 * iterations; *flops (may be NULL) receives the flops of the launch.
 * Asynchronous; time it with events. */
typedef enum {
    TSG_PEAK_MFMA_F64 = 0,
    TSG_PEAK_VALU_F64 = 1,
    TSG_PEAK_MFMA_F32 = 2,
    TSG_PEAK_MIXED_F64 = 3
} tsg_peak_kind;
tsg_status tsg_peak_probe(int32_t kind, int32_t blocks_per_cu, int64_t iters, double *flops, void *stream);

/* Memory latency by pointer chasing (Section 5.3 measures latency to apply
 * Little's law): one lane follows next[] from index 0 for `steps` dependent
 * loads (after 64 warm-up loads).  out[0] = elapsed shader clocks, out[1] =
 * elapsed ticks of the 100 MHz constant clock, out[2] = the final index (all
 * device memory, int64).  `next` is a device array of indices into itself
 * that the caller builds (a random cycle over a working set of the chosen
 * size).  Asynchronous. */
tsg_status tsg_latency_probe(const int64_t *next, int64_t steps, int64_t *out, void *stream);

/* ---- tuning hooks (used by the autotuner; not needed for ordinary calls) ----
 * The library holds many generated kernel variants; normally it picks the one
 * tuned for (operation, dtype, M, N).  tsg_force_variant(name) makes the
 * calling thread's following calls use the named variant instead (a call it
 * cannot serve returns TSG_E_UNSUPPORTED); NULL or "" restores the automatic
 * choice.  Returns TSG_E_ARG for an unknown name.  tsg_variant_count and
 * tsg_variant_name(i) enumerate the compiled variants (static strings). */
tsg_status tsg_force_variant(const char *name);
int32_t tsg_variant_count(void);
const char *tsg_variant_name(int32_t i);

/* tsg_set_grid_limit(blocks) caps the number of blocks of the calling thread's
 * following TSMTTSM and TSMM launches (0 removes the cap; negative values
 * return TSG_E_ARG).  With a small cap every block works through many tiles
 * of a short matrix, which lets tests cover the multi-tile paths of each
 * kernel (register rings, staging reuse) without matrices of millions of rows.
 * Results stay within the usual bounds (TSMTTSM partial sums are folded in a
 * different grouping, so floating-point results may differ in rounding). */
tsg_status tsg_set_grid_limit(int32_t blocks);

/* Ablation of the cross-block reduction of TSMTTSM (the paper's Section 3.2
 * and 5.5 compare reduction variants against K).  Affects the calling
 * thread's following TSMTTSM calls whose grid has more than one block:
 *   TSG_REDUCE_FOLD    the default: per-block partials summed by a second
 *                      kernel in a fixed order (bitwise reproducible);
 *   TSG_REDUCE_ATOMIC  every block's partial added into C with global FP64
 *                      atomics (C cleared first); the order of the additions
 *                      and so the rounding varies from run to run;
 *   TSG_REDUCE_NONE    no reduction: the partials stay in the workspace and C
 *                      is NOT written (a timing lower bound only).
 * Any other value returns TSG_E_ARG. */
enum { TSG_REDUCE_FOLD = 0, TSG_REDUCE_ATOMIC = 1, TSG_REDUCE_NONE = 2 };
tsg_status tsg_set_reduction(int32_t mode);

#ifdef __cplusplus
}
#endif

#endif /* TSGEMM_H */
