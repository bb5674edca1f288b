/*
 * spamm.h - C-ABI of an MI355X (gfx950) library for approximate products
 * C ~= A B of matrices with exponential decay, stored as quadtrees of dense
 * leaf blocks, under three schemes: Truncmul (multiply truncated inputs),
 * SpAMM (skip sub-matrix products whose norm product is below tau) and
 * Hybrid (SpAMM on truncated inputs, same tau).
 *
 * Method: A. G. Artemov, "Approximate multiplication of nearly sparse
 * matrices with decay in a fully recursive distributed task-based parallel
 * framework", arXiv:1906.08148.  Section / algorithm references below are to
 * that paper.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All device memory comes from one caller-provided *arena* (for example a
 *   torch uint8 tensor); the library sub-allocates in it and never calls
 *   hipMalloc for matrix data.  Small pinned host staging is allocated once
 *   per context with hipHostMalloc.
 * - Work is enqueued on the context's stream (a hipStream_t passed as void*;
 *   NULL is the legacy default stream).  Calls that must size an allocation
 *   read a count back and synchronise that stream; this is stated per call.
 * - Every function returns a spamm_status; no exception crosses the ABI.  On
 *   an error, output handles are set to NULL and nothing is left allocated.
 *   spamm_last_error() gives a message for the last failing call.
 * - Matrix handles are immutable once returned (like the registered chunks
 *   of Sec. 4.1): derived handles (spamm_truncate) share leaf storage, which
 *   stays alive until every handle referring to it is released.
 * - A context and its handles are used by one host thread at a time.
 *
 * Storage of a matrix (Sec. 2, Sec. 4.2, Sec. 4.4)
 * ------------------------------------------------
 * n x n, leaf size bs; G = ceil(n/bs) rounded up to a power of two, L =
 * log2(G).  Level l (0 = root, L = leaves) has 4^l nodes in Morton (Z) order,
 * row bit above column bit, so the children of node m are 4m..4m+3.  A leaf
 * with no non-zero value is null and has no storage.  Every node carries its
 * FP64 squared Frobenius norm; a parent's is the sum of its four children's,
 * taken as ((c0 + c1) + c2) + c3.
 */
#ifndef SPAMM_H
#define SPAMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum spamm_status {
  SPAMM_OK = 0,
  SPAMM_EINVAL = 1,       /* bad argument: tau < 0 / NaN / Inf, n < 1, ld < n,
                             leaf not in {16,32,64,128,256}, NULL pointer,
                             ...                                              */
  SPAMM_ESHAPE = 2,       /* A and B (or D) differ in n or leaf size           */
  SPAMM_ENOMEM = 3,       /* the arena cannot hold the result                 */
  SPAMM_ENONFINITE = 4,   /* NaN or Inf in an input matrix                    */
  SPAMM_EUNSUPPORTED = 5, /* not supported: precision/leaf combination not
                             built, a needed FP64 copy absent, or a batch too
                             large for one counting pass                     */
  SPAMM_EDEVICE = 6       /* a HIP call failed (message in spamm_last_error)  */
} spamm_status;

/* Approximation scheme (Sec. 3; names as in Sec. 5). */
typedef enum spamm_mode {
  SPAMM_TRUNCMUL = 0, /* truncate A and B, form every non-null leaf product   */
  SPAMM_SPAMM = 1,    /* form leaf products with ||A_ik||_F ||B_kj||_F >= tau */
  SPAMM_HYBRID = 2,   /* SPAMM on A and B truncated with the same tau         */
  SPAMM_SPAMM_SYM = 3, /* SPAMM for the square of a symmetric A (B = A, the
                          same handle; an epilogue matrix D must be symmetric
                          too).  C = A A is symmetric, so only the C leaves
                          (I, J) with I <= J are decided by the norm test and
                          formed; each leaf below the diagonal takes its
                          mirror's decision, skipped bound and norm and is
                          written as the transpose of its mirror (n_kept and
                          flops count the formed products; the kept list
                          holds them).  If A's null map (or D's) is not
                          symmetric, every C leaf is formed as in SPAMM.
                          The caller asserts that A (and D) are symmetric. */
  SPAMM_HYBRID_SYM = 4 /* the same for Hybrid: A is truncated in mirror
                          pairs (spamm_truncate_symmetric), which keeps a
                          symmetric null map symmetric; if the truncated
                          null map is symmetric, the upper C leaves are
                          formed and mirrored as above, else the full
                          Hybrid product is formed.  The check runs on the
                          device; no extra synchronisation.                */
} spamm_mode;

/* Arithmetic of the leaf products.  The norms, the tau tests and all error
 * accounting are FP64 in every precision. */
typedef enum spamm_prec {
  SPAMM_F64 = 0,   /* FP64 inputs, FP64 accumulation (MFMA f64)              */
  SPAMM_F32 = 1,   /* FP32 inputs, FP32 accumulation (MFMA f32)              */
  SPAMM_BF16 = 2,  /* BF16 inputs, FP32 accumulation (MFMA bf16)             */
  SPAMM_BF16X3 = 3 /* split BF16: hi*hi + hi*lo + lo*hi, FP32 accumulation   */
} spamm_prec;

/* Leaf-store copies a matrix may hold (bit mask). */
#define SPAMM_STORE_F64 1u
#define SPAMM_STORE_F32 2u
#define SPAMM_STORE_BF16 4u /* hi = bf16(x) and lo = bf16(x - hi) */

typedef void* spamm_stream; /* a hipStream_t */
typedef struct spamm_ctx spamm_ctx;
typedef struct spamm_mat spamm_mat;

/* Accounting of one product (FP64; Sec. 3, Thms 1-3). */
typedef struct spamm_stats {
  int64_t n_kept;       /* leaf products formed                              */
  int64_t n_candidates; /* leaf triples with both operands non-null          */
  int64_t c_nonnull;    /* non-null leaves of C                              */
  double flops;         /* 2 * bs^3 * n_kept (Sec. 5.3 flop count)           */
  double B1;            /* sum over C leaves of b_ij, where b_ij is the sum of
                           ||A_ik||_F ||B_kj||_F over skipped non-null k     */
  double B2;            /* (sum of b_ij^2)^(1/2) >= ||E_SpAMM||_F             */
  double dA, dB;        /* Frobenius norm dropped by truncating A and B      */
  double normA, normB;  /* ||A||_F, ||B||_F of the untruncated inputs        */
  double normA_used;    /* ||A~||_F of the operand actually multiplied       */
  double err_bound;     /* bound on ||A B - C||_F from the terms above       */
  double trace;         /* trace of C (sum of diagonal-leaf diagonals)       */
  double normC;         /* ||C||_F                                           */
  double prec_bound;    /* bound on ||C - C_kept||_F from rounding, where
                           C_kept is the exact sum of the kept products: per
                           C leaf with m kept products of order bs, c(m) times
                           the sum of their ||A_ik||_F ||B_kj||_F, with c(m) =
                           e_in + gamma_n mag for the compute precision (input
                           representation error e_in, n = bs + m + 1 roundings,
                           3 bs + m + 1 for split BF16); root-sum-square over
                           C leaves.  Covers the product before an epilogue.
                           The total error against A B is at most err_bound +
                           prec_bound.                                       */
  double val_err;       /* ||C - C_FP64||_F, C_FP64 the same kept products in
                           FP64, measured when SPAMM_OPT_VALIDATE is on;
                           -1 when it is off                                 */
} spamm_stats;

/* Optional epilogue: C = alpha * (approximate A B) + beta * D, with D a
 * matrix of the same n and leaf size.  Leaves of D enter C whether or not a
 * product lands there.  NULL means alpha = 1, beta = 0. */
typedef struct spamm_epilogue {
  double alpha;
  double beta;
  const spamm_mat* D;
} spamm_epilogue;

/* One request of a batched multiply (see spamm_multiply_batch). */
typedef struct spamm_request {
  const spamm_mat* A;
  const spamm_mat* B;
  double tau;
  int32_t mode; /* spamm_mode */
  int32_t prec; /* spamm_prec */
  const spamm_epilogue* ep; /* may be NULL */
} spamm_request;

typedef struct spamm_mat_info {
  int64_t n;
  int32_t leaf, G, L;
  int64_t nonnull;      /* non-null leaves                                  */
  uint32_t stores;      /* SPAMM_STORE_* copies held                         */
  int32_t has_plan;     /* 1 if the handle came from a multiply              */
  int64_t n_kept;       /* products of that multiply                         */
  size_t device_bytes;  /* arena bytes referenced by this handle             */
} spamm_mat_info;

/* Device time per kernel class, from HIP events recorded on the context's
 * stream around each launch (only while timing is enabled). */
typedef struct spamm_timing {
  double build_ms;    /* leaf scan, compaction, copies                     */
  double trunc_ms;    /* truncation                                        */
  double prune_ms;    /* counting pass, scan, fill                         */
  double gemm_ms;     /* persistent leaf-GEMM launches                     */
  double pyramid_ms;  /* norm pyramids                                     */
  int64_t build_launches, trunc_launches, prune_launches, gemm_launches, pyramid_launches;
  double gemm_flops;  /* 2 * bs^3 * (products) over the timed GEMM launches */
  int64_t gemm_quad_launches;  /* of gemm_launches, those on quads (SPAMM_OPT_GEMM_QUAD) */
} spamm_timing;

/* Name of a status code (static string). */
const char* spamm_status_string(spamm_status s);

/* Message of the last failing call on this context (static per context;
 * valid until the next call). */
const char* spamm_last_error(const spamm_ctx* ctx);

/* Create a context on HIP device `device`, sub-allocating from the device
 * buffer [arena, arena + arena_bytes) (caller-owned, 256-byte aligned, must
 * outlive the context) and enqueueing on `stream`.  Errors: EINVAL (NULL
 * out/arena, arena_bytes < 1 MiB, misaligned arena), EDEVICE. */
spamm_status spamm_ctx_create(int device, void* arena, size_t arena_bytes,
                              spamm_stream stream, spamm_ctx** out);

/* Destroy a context.  Every handle must have been released; the call
 * synchronises the stream first. */
spamm_status spamm_ctx_destroy(spamm_ctx* ctx);

/* Change the stream later calls enqueue on. */
spamm_status spamm_ctx_set_stream(spamm_ctx* ctx, spamm_stream stream);

/* Tunable behaviour of a context (spamm_ctx_set_option / get_option).
 *  SPAMM_OPT_GEMM_TILE  1: 16 x 16 MFMA tiles (default); 0: 32 x 32 tiles
 *                       for FP32 / BF16 leaf products where a wave's tile
 *                       allows it.  FP64 always takes 16 x 16.
 *  SPAMM_OPT_PLACEMENT  0: each request's C leaves in eight Morton slices,
 *                       one per XCD (default); 1: request after request.
 *  SPAMM_OPT_GRAPH      0: launch the kernels of a batch one by one
 *                       (default); 1: capture the kernels that follow the
 *                       sizing read-back into one HIP graph per batch and
 *                       launch that (an instantiated graph of the same shape
 *                       is updated in place).  Ignored while event timing
 *                       is on.
 *  SPAMM_OPT_UNIT_ORDER c in 1..1024: the C leaves (quads) an XCD works on
 *                       are dealt round-robin over its workgroups in chunks
 *                       of c consecutive ones, so the workgroups move
 *                       through the slice together (less L2 traffic); 0:
 *                       each workgroup takes a contiguous range of equal
 *                       cost; -1 (default): per launch, 1 when the C leaves
 *                       average fewer than 16 products, else 0, and 0 for
 *                       quads.
 *  SPAMM_OPT_VALIDATE   0 (default): spamm_stats.val_err = -1; 1: every
 *                       product that is not FP64 runs beside an FP64 twin
 *                       (same operands, tau, mode and epilogue) in the same
 *                       batch, and val_err = ||C - C_FP64||_F over the same
 *                       kept products (0 for FP64 products).  Needs the FP64
 *                       copy of A and B (EUNSUPPORTED otherwise); costs the
 *                       FP64 products and one synchronisation.
 *  SPAMM_OPT_GEMM_QUAD  1: the C leaves of a leaf-64 product that are
 *                       children of one quadtree node (up to four) run in one
 *                       workgroup over the merged k order of their products,
 *                       so that every A and B leaf staged serves both
 *                       children of its row or column half (half the operand
 *                       reads when all four keep a k); each C leaf still sums
 *                       its own products k ascending.  Quads take 16 x 16
 *                       MFMA tiles whatever GEMM_TILE says.  0: every C leaf
 *                       is one work unit of the one-leaf GEMM.  -1 (default):
 *                       quads for a launch group (one precision) whose C
 *                       leaves average at least 32 (FP64), 128 (FP32) or 16
 *                       (BF16, split BF16) kept products, the one-leaf GEMM
 *                       below.  Leaves 128 and 256: with 1 each 128 x 128
 *                       tile of a C leaf runs on the same kernel as a quad
 *                       of its four 64 x 64 blocks (a product is bs / 64
 *                       merged steps, every block keeps every step); -1
 *                       takes that for FP64 only.  Leaves 16 and 32 ignore
 *                       the option.
 * PLACEMENT, GRAPH and UNIT_ORDER give bitwise identical results; GEMM_TILE
 * and GEMM_QUAD change the order of the sums inside one MFMA or one k-panel
 * (results stay within the precision's tolerance).  Errors: EINVAL (unknown
 * key or value; values are 0 or 1, and -1 for UNIT_ORDER and GEMM_QUAD). */
typedef enum {
  SPAMM_OPT_GEMM_TILE = 0,
  SPAMM_OPT_PLACEMENT = 1,
  SPAMM_OPT_GRAPH = 2,
  SPAMM_OPT_UNIT_ORDER = 3,
  SPAMM_OPT_VALIDATE = 4,
  SPAMM_OPT_GEMM_QUAD = 5
} spamm_option;

spamm_status spamm_ctx_set_option(spamm_ctx* ctx, spamm_option key, int64_t value);
spamm_status spamm_ctx_get_option(const spamm_ctx* ctx, spamm_option key, int64_t* value);

/* Arena occupancy in bytes (host outputs, any may be NULL). */
spamm_status spamm_ctx_arena_info(const spamm_ctx* ctx, size_t* used,
                                  size_t* free_bytes, size_t* largest_free);

/* Turn event timing on (enable = 1) or off (0) for later calls; when `out`
 * is non-NULL, synchronise the stream and write the totals since the last
 * reset; reset = 1 clears them afterwards.  Errors: EINVAL, EDEVICE. */
spamm_status spamm_ctx_timing(spamm_ctx* ctx, int32_t enable, int32_t reset,
                              spamm_timing* out);

/* Build a matrix from a dense FP64 row-major n x n device buffer with leading
 * dimension ld (Sec. 2; Sec. 4.2 null blocks; Sec. 4.4 dense leaves kept when
 * they hold a non-zero).  The input is read once for norms and flags and once
 * more for the non-null leaves; it may be freed after the stream has passed
 * this call.  `stores` chooses the leaf copies (F64 always recommended).
 * Synchronises once (non-null count and non-finite flag).
 * Errors: EINVAL, ENONFINITE, ENOMEM, EDEVICE. */
spamm_status spamm_build(spamm_ctx* ctx, const double* dense, int64_t n,
                         int64_t ld, int32_t leaf, uint32_t stores,
                         spamm_mat** out);

/* Build from a list of nblocks leaf blocks: coords[2t], coords[2t+1] = (I, J)
 * (device int32, 0 <= I, J < ceil(n/leaf)), data = nblocks x leaf x leaf FP64
 * row-major (device).  Unlisted leaves are zero; listed all-zero blocks are
 * null; entries past row/column n must be zero (EINVAL otherwise); a
 * coordinate listed twice is EINVAL.  Synchronises once.
 * Errors: EINVAL, ENONFINITE, ENOMEM, EDEVICE. */
spamm_status spamm_build_blocks(spamm_ctx* ctx, int64_t n, int32_t leaf,
                                int64_t nblocks, const int32_t* coords,
                                const double* data, uint32_t stores,
                                spamm_mat** out);

/* One list of leaf blocks for spamm_build_blocks_batch (the arguments of
 * spamm_build_blocks). */
typedef struct spamm_block_list {
  int64_t n;
  int32_t leaf;
  uint32_t stores;
  int64_t nblocks;
  const int32_t* coords; /* device, 2 * nblocks */
  const double* data;    /* device, nblocks * leaf * leaf */
} spamm_block_list;

/* spamm_build_blocks for `count` lists at once (Sec. 2; Sec. 4.2): each
 * out[t] equals what spamm_build_blocks returns for lists[t], bit for bit,
 * but the batch synchronises once for all lists and builds their norm
 * pyramids in one launch.  The device inputs are read by kernels queued on
 * the context's stream: keep them unchanged until that stream has passed
 * this call.  On error (the first failing list's status) no out[t] is
 * allocated.  Errors: EINVAL, ENONFINITE, ENOMEM, EDEVICE. */
spamm_status spamm_build_blocks_batch(spamm_ctx* ctx, int32_t count,
                                      const spamm_block_list* lists,
                                      spamm_mat** out);

/* Input truncation with a global Frobenius budget (Sec. 3; the leaf-block
 * form): order the non-null leaves by (squared norm, Morton key) and drop the
 * longest prefix whose summed squared norm is <= tau^2, so that
 * ||in - out||_F <= tau.  The result shares leaf storage with `in`.
 * `dropped_sq` (host, nullable) receives the dropped squared norm.
 * Synchronises once.  Errors: EINVAL, ENOMEM, EDEVICE. */
spamm_status spamm_truncate(spamm_ctx* ctx, const spamm_mat* in, double tau,
                            spamm_mat** out, double* dropped_sq);

/* The same truncation in mirror pairs, for a symmetric matrix (a reading:
 * Sec. 3's truncation, which the paper never applies to symmetric pairs,
 * Sec. 5.4): leaf (I, K), I < K, and leaf (K, I) form one unit of weight
 * s_IK + s_KI (FP64 sum; a diagonal leaf is a unit of its own); units with
 * a non-null leaf are ordered by (weight, Morton key of the upper leaf) and
 * the longest prefix whose summed weights are <= tau^2 is dropped, both
 * leaves of a unit together.  ||in - out||_F <= tau still holds, and a
 * symmetric null map stays symmetric, so mirror leaves whose norms differ
 * only by rounding are never split.  SPAMM_HYBRID_SYM truncates its operand
 * this way; a symmetric product (a purification iterate) is truncated this
 * way after the multiply.  Storage, `dropped_sq`, synchronisation and errors
 * as spamm_truncate. */
spamm_status spamm_truncate_symmetric(spamm_ctx* ctx, const spamm_mat* in, double tau,
                                      spamm_mat** out, double* dropped_sq);

/* Element-wise input truncation, the truncated matrix of Thm. 1 (Sec. 3):
 * every entry with |a_ij| < tau becomes zero, so each dropped entry is below
 * tau.  A leaf with no non-zero entry left becomes null; the others keep
 * their slots in a new store holding the same copies as `in`, written again
 * from the thresholded FP64 values, and the norm pyramid is rebuilt.
 * `dropped_sq` (host, nullable) receives the squared Frobenius norm of the
 * dropped entries (FP64, summed in a fixed order).  Multiplying two such
 * results with tau = 0 in SPAMM_TRUNCMUL mode gives the element-wise
 * Truncmul product of the theorem.  Needs the FP64 copy of `in`
 * (EUNSUPPORTED otherwise).  Synchronises once.
 * Errors: EINVAL, EUNSUPPORTED, ENOMEM, EDEVICE. */
spamm_status spamm_truncate_elementwise(spamm_ctx* ctx, const spamm_mat* in, double tau,
                                        spamm_mat** out, double* dropped_sq);

/* C ~= A B (Alg. 1 with the null rule of Alg. 2; the mode selects Truncmul,
 * SpAMM or Hybrid).  A leaf triple (i,k,j) is formed when A_ik and B_kj are
 * non-null and, for SpAMM/Hybrid, sqrt(s_ik) * sqrt(s_kj) >= tau in FP64.
 * Products of one C leaf are accumulated by one workgroup in ascending k, so
 * results are bitwise reproducible.  C is a new handle whose leaves are FP64
 * (prec F64) or FP32 (other precisions), with its own norm pyramid and the
 * list of formed products (spamm_kept).  Missing compute copies of A/B are
 * derived and cached.  A and B may be the same handle.  `st` may be NULL.
 * Synchronises once to size C, and once more when `st` is given.
 * Errors: EINVAL, ESHAPE, ENOMEM, EUNSUPPORTED, EDEVICE. */
spamm_status spamm_multiply(spamm_ctx* ctx, const spamm_mat* A,
                            const spamm_mat* B, double tau, spamm_mode mode,
                            spamm_prec prec, const spamm_epilogue* ep,
                            spamm_mat** C, spamm_stats* st);

/* `count` multiplies as one batch: truncation, pruning and the C pyramids run
 * as batched kernels and every leaf product of every request goes out in one
 * persistent GEMM launch per (precision, leaf size).  C_out[r] and st_out[r]
 * (nullable array) receive request r's result; each equals what
 * spamm_multiply returns for that request alone, bit for bit.  On error no
 * C_out is allocated.  Same errors as spamm_multiply; EUNSUPPORTED also when
 * the batch is too large for one counting pass (the sum over requests of
 * G^3, times the total number of C leaves G^2, reaches 2^62): split it. */
spamm_status spamm_multiply_batch(spamm_ctx* ctx, int32_t count,
                                  const spamm_request* reqs,
                                  spamm_mat** C_out, spamm_stats* st_out);

/* FP64 squared Frobenius norms of level `level` (0 = root .. L = leaves) in
 * Morton order, or all levels root first when level = -1, copied to the host
 * buffer out[cap]; *count receives the number of values (4^level, or
 * (4^(L+1) - 1) / 3).  Null nodes read 0.  Synchronises.
 * Errors: EINVAL (bad level, cap too small), EDEVICE. */
spamm_status spamm_norms(spamm_ctx* ctx, const spamm_mat* m, int32_t level,
                         double* out, int64_t cap, int64_t* count);

/* The leaf products formed by the multiply that produced C, as host int32
 * triples ijk[3t..3t+2] = (I, K, J), ordered by the Morton key of (I, J) and
 * then K ascending.  *count receives the number of triples; with cap too
 * small nothing is written and EINVAL is returned with *count set.
 * Synchronises.  Errors: EINVAL (no plan on this handle), EDEVICE. */
spamm_status spamm_kept(spamm_ctx* ctx, const spamm_mat* C, int32_t* ijk,
                        int64_t cap, int64_t* count);

/* Per-leaf skipped-product bound b_IJ of the multiply that produced C (FP64,
 * G*G values in Morton order, host).  Synchronises. */
spamm_status spamm_skipped_bound(spamm_ctx* ctx, const spamm_mat* C,
                                 double* out, int64_t cap);

/* Write the matrix as dense FP64 row-major n x n into device memory `out`
 * with leading dimension ld (null leaves become zeros).  Asynchronous.
 * Errors: EINVAL, EDEVICE. */
spamm_status spamm_to_dense(spamm_ctx* ctx, const spamm_mat* m, double* out,
                            int64_t ld);

/* Gershgorin bounds of the spectrum of a square matrix: *lo = min over rows
 * i < n of a_ii - sum_{j != i} |a_ij|, *hi = max of a_ii + sum_{j != i}
 * |a_ij| (host doubles), from the FP64 leaf copy (FP32 when that is the only
 * copy), in FP64.  Used to scale a matrix into [0, 1] before purification
 * (the density-matrix purification the paper's introduction cites).
 * Synchronises.  Errors: EINVAL, ENOMEM, EDEVICE. */
spamm_status spamm_gershgorin(spamm_ctx* ctx, const spamm_mat* m, double* lo,
                              double* hi);

/* spamm_gershgorin for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  The same bounds, computed by the same kernels, are written
 * stream-ordered to the caller's device buffer bounds[0] = lo, bounds[1] =
 * hi (two doubles); nothing is synchronised and nothing is allocated: the
 * per-leaf-row partial bounds live in a static device array of 1024 leaf
 * rows (16 KiB per device, held until the process ends), so m must have
 * G <= 1024 leaf rows (n <= 1024 * leaf; EUNSUPPORTED otherwise, before
 * any launch).  Every
 * call on one device shares that array: calls that overlap on one device
 * (other streams or contexts, other threads) race and must be ordered by
 * the caller.  Errors: EINVAL (NULL argument, foreign handle), EUNSUPPORTED
 * (no FP64/FP32 copy, G > 1024), EDEVICE (launch failure, scratch address
 * not found at context creation). */
spamm_status spamm_gershgorin_static(spamm_ctx* ctx, const spamm_mat* m,
                                     double* bounds);

/* Copy `count` leaves (block row ij[2t], block column ij[2t+1], host int32)
 * of a matrix into `out` (host, FP64, count * bs * bs values, leaf t
 * row-major at t * bs * bs); null leaves give zeros, entries beyond n are the
 * zero padding.  For checking a few blocks of a large result (Sec. 4.2
 * layout: a leaf is one bs x bs block).  Synchronises.
 * Errors: EINVAL (null pointer, count < 0, a coordinate outside the grid),
 * ENOMEM, EDEVICE. */
spamm_status spamm_leaves(spamm_ctx* ctx, const spamm_mat* m, const int32_t* ij,
                          int64_t count, double* out);

/* Describe a handle (host output). */
spamm_status spamm_mat_info_get(const spamm_mat* m, spamm_mat_info* out);

/* Release a handle (shared leaf storage is freed with its last user).
 * Stream-ordered: the memory is reused only by work enqueued later on the
 * same stream.  NULL is accepted. */
spamm_status spamm_release(spamm_ctx* ctx, spamm_mat* m);

#ifdef __cplusplus
}
#endif
#endif /* SPAMM_H */
