/*
 * spamm.h -- C ABI of the MI355X SpAMM library (libspamm.so).
 *
 * Sparse Approximate Matrix Multiply (Bock & Challacombe, "An Optimized Sparse
 * Approximate Matrix Multiply for Matrices with Decay"): C ~= A B for matrices
 * whose entries decay away from the diagonal.  Each operand is held as a
 * quadtree of n_b x n_b dense leaves with a Frobenius norm per node (Sec. II.A
 * and II.B); a sub-product A_ik B_kj is skipped whenever
 * ||A_ik||_F ||B_kj||_F < tau (Eq. norm condition), at every tier.
 *
 * Conventions
 *  - Every call returns an int status: SPAMM_OK (0) or a negative SPAMM_E_*
 *    code; spamm_strerror() names it and spamm_last_error() gives the detail
 *    of the calling thread's last failure.  Nothing is thrown across the ABI.
 *  - Matrix pointers are DEVICE pointers (FP32, row-major, leading dimension
 *    n, square n x n).  `stream` is a hipStream_t (NULL = the null stream).
 *    Work is enqueued on that stream; pointers must stay valid until the
 *    stream has passed the work.
 *  - Host pointers are named `host` and are written synchronously.
 *  - Sizes are element counts unless stated otherwise.
 *  - Limits: leaf n_b in {16, 32, 64}; tiles per dimension N = n_p / n_b at
 *    most 1024 (so n <= 1024 n_b); tau finite, tau = 0 or tau >= 1e-150.
 */
#ifndef SPAMM_H
#define SPAMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define SPAMM_OK            0
#define SPAMM_E_INVAL      -1   /* bad argument (null pointer, size, leaf, tau) */
#define SPAMM_E_NONFINITE  -2   /* NaN or Inf in the input matrix             */
#define SPAMM_E_NOMEM      -3   /* device allocation failed                   */
#define SPAMM_E_HIP        -4   /* a HIP runtime call failed (see last_error) */
#define SPAMM_E_RANGE      -5   /* host buffer too small / size over a limit  */
#define SPAMM_E_MISMATCH   -6   /* operands of different n or leaf size       */
#define SPAMM_E_BUSY       -7   /* server queue full; submit again later      */
#define SPAMM_PENDING       1   /* server request queued or running (poll)    */

/* ---- precision of the leaf products (split precision) -------------------- */
#define SPAMM_PREC_FP32        0   /* every kept product in FP32 (MFMA, FP32 accumulation) */
#define SPAMM_PREC_SPLIT_BF16  1   /* LOW products on BF16 operands, HIGH ones in FP32      */
#define SPAMM_PREC_SPLIT_FP16  2   /* LOW products on scaled FP16 operands, HIGH ones FP32  */
#define SPAMM_PREC_SPLIT_BF16X3 3  /* LOW products on BF16 operands, HIGH ones compensated: */
                                   /* three BF16 products of the entries' two BF16 parts   */

/* Tree build flags. */
#define SPAMM_TREE_BF16        1u  /* also keep BF16 copies of the leaves (split precision) */
#define SPAMM_TREE_SUBNORMS    2u  /* n_b = 64: also keep the norms of the 32 x 32 sub-blocks */
                                   /* (sub-leaf culling); the whole pyramid is then that of  */
                                   /* a tree with 32 x 32 leaves                            */
#define SPAMM_TREE_FP16        4u  /* also keep FP16 copies of the leaves, each leaf scaled  */
                                   /* by a power of two fixed by its squared norm (split    */
                                   /* precision SPAMM_PREC_SPLIT_FP16); not with BF16       */

typedef struct spamm_tree spamm_tree;   /* one operand: packed leaves + norms  */
typedef struct spamm_plan spamm_plan;   /* one product's kept task list        */

/* Statistics of one product (filled by spamm_plan_stats / spamm_multiply_ex). */
typedef struct spamm_stats {
    int32_t depth;            /* d: tiers 0..d                                  */
    int32_t leaf;             /* n_b                                            */
    int64_t kept[32];         /* kept node triples per tier t = 0..d            */
    int64_t tasks;            /* K = kept[d]: leaf products performed           */
    int64_t tasks_low;        /* of which LOW (BF16 operands; split precision)   */
    int64_t block_entries;    /* (k, mask) entries scheduled, HIGH list         */
    int64_t block_entries_low;/* (k, mask) entries scheduled, LOW list          */
    double  flops;            /* 2 n_b^3 K; sub-leaf culling: 2 (n_b/2)^3 subtasks */
    double  symbolic_ms;      /* cull time (events), or -1 when not timed        */
    double  numeric_ms;       /* leaf-GEMM time (events), or -1 when not timed   */
    int64_t subtasks;         /* sub-leaf culling: 32 x 32 sub-products performed */
                              /* by the last spamm_numeric of the plan, else 0     */
} spamm_stats;

/* ---- operands -------------------------------------------------------------- */

/*
 * Build the quadtree of A (Sec. II.A, II.B).
 *   A      device pointer, n x n FP32 row-major (lda = n); read only by work
 *          enqueued here; the caller keeps it alive until `stream` passes it.
 *   n      matrix order, n >= 1.
 *   leaf   n_b in {16, 32, 64}.  Depth d = smallest d >= 0 with n_b 2^d >= n;
 *          A is zero-padded to n_p = n_b 2^d (padding is never read from A).
 *   out    receives the handle.  The tree owns copies: the packed leaves
 *          (FP32, leaves in linear-index order of Eq. linear index, each
 *          stored twice: as is for the left operand and transposed for the
 *          right operand) and the squared Frobenius norms of all tiers in
 *          FP64 (leaf: pairwise sum of squares over the leaf's row-major
 *          flattened index; parent: (s11 + s12) + (s21 + s22)).
 * Synchronizes `stream` once, to read the root norm; a non-finite root means
 * NaN/Inf in A -> SPAMM_E_NONFINITE (no tree is returned).
 * Errors: SPAMM_E_INVAL (n < 1, bad leaf, null A/out), SPAMM_E_RANGE (N > 1024),
 *         SPAMM_E_NONFINITE, SPAMM_E_NOMEM, SPAMM_E_HIP.
 */
int spamm_build_tree(const float *A, int64_t n, int32_t leaf, void *stream,
                     spamm_tree **out);

/*
 * Options of a product.
 *   tau        SpAMM tolerance (absolute), as for spamm_symbolic.
 *   precision  SPAMM_PREC_FP32, SPAMM_PREC_SPLIT_BF16, SPAMM_PREC_SPLIT_FP16 or
 *              SPAMM_PREC_SPLIT_BF16X3.  SPLIT_BF16X3 classes and rounds the
 *              LOW products as SPLIT_BF16 does and takes every HIGH product
 *              a b from the two bfloat16 parts of its entries, hi = bf16(x)
 *              and lo = bf16(x - hi) (x - hi exact in FP32), as
 *              hi_a hi_b + hi_a lo_b + lo_a hi_b on BF16 matrix units with
 *              FP32 accumulation (the three-product bfloat16 method of
 *              Henry, Tang and Heinecke, ARITH 2019): within 2^-14 |a||b|
 *              of the exact product per term, against FP32's exact products,
 *              at about a fifth of the matrix-unit time.  An entry at or
 *              above 2^128 (1 - 2^-9) in magnitude would overflow its
 *              bfloat16 part, so SPLIT_BF16X3 refuses operands whose squared
 *              Frobenius norm reaches (2^128 (1 - 2^-9))^2 with SPAMM_E_RANGE
 *              (spamm_symbolic_ex; the server reports it as the request's
 *              status, C then undefined).  It needs trees built with
 *              SPAMM_TREE_BF16, like SPLIT_BF16.
 *   low_tol    split only: a kept product A_ik B_kj is LOW iff
 *              fl64(s_A s_B) < fl64(low_tol^2) on the stored squared norms,
 *              i.e. ||A_ik||_F ||B_kj||_F < low_tol; LOW products use BF16
 *              operands (each FP32 entry rounded to nearest even) or FP16
 *              ones (each leaf times 2^e, e = 14 - ceil(p / 2) where its
 *              squared norm is S = m 2^p with 0.5 <= m < 1, so every scaled
 *              entry is below 2^14; rounded to nearest even, a result below
 *              2^-14 (a binary16 subnormal) flushed to zero; the product is
 *              scaled back by 2^-(eA + eB)) with FP32
 *              accumulation, HIGH products stay FP32.  0 = nothing is LOW
 *              (unless low_rel is set).
 *   low_rel    split only, instead of low_tol: the relative threshold theta
 *              of the precision split, LOW iff ||A_ik||_F ||B_kj||_F <
 *              theta ||A||_F ||B||_F, evaluated on the device as
 *              fl64(s_A s_B) < fl64(fl64(fl64(theta^2) s_A0) s_B0), where
 *              s_A0 and s_B0 are the FP64 roots of the two trees' own norm
 *              pyramids (so every product, every step of a squaring chain
 *              included, is split against its own operands' norms).
 *              Finite, 0 or >= 1e-150; at most one of low_tol and low_rel
 *              may be non-zero.
 */
typedef struct spamm_opts {
    double  tau;
    int32_t precision;
    double  low_tol;
    int32_t sub_cull;   /* 1: sub-leaf culling (FP32, n_b = 64, trees built with     */
                        /* SPAMM_TREE_SUBNORMS): inside every kept 64 x 64 leaf product */
                        /* the 8 products of 32 x 32 sub-blocks are tested against tau */
                        /* with their own norms and only the kept ones are multiplied  */
                        /* (the paper's conditional products inside a leaf, Alg. 2);   */
                        /* the performed set equals the cull of a tree with 32 x 32    */
                        /* leaves.  0: whole leaf products.                             */
    double  low_rel;    /* split only: relative LOW threshold theta (see above)        */
} spamm_opts;

/* As spamm_build_tree, with flags (SPAMM_TREE_BF16: also store BF16 copies of
 * every leaf, needed by SPAMM_PREC_SPLIT_BF16 products; leaf must be 32 or 64.
 * SPAMM_TREE_FP16: FP16 copies at the per-leaf scale of spamm_opts, for
 * SPAMM_PREC_SPLIT_FP16; leaf 32 or 64, not together with SPAMM_TREE_BF16.
 * SPAMM_TREE_SUBNORMS: leaf must be 64; tiers 0..d+1 of norms, tier d+1 being
 * the 32 x 32 sub-blocks, each a pairwise sum over its own row-major index,
 * and every coarser tier the (s11 + s12) + (s21 + s22) of its children). */
int spamm_build_tree_ex(const float *A, int64_t n, int32_t leaf, uint32_t flags, void *stream,
                        spamm_tree **out);

/*
 * Build the epsilon-sparsified quadtree of A (Sec. II.C, Eq. epsilon):
 * epsilon = tau / max(||A||_F, ||B||_F); a leaf is dropped (a NULL node: not
 * stored, norm 0) when its squared norm s is 0 or fl64(s * m) < fl64(tau^2),
 * with m = max(||A||_F^2, norm2_other) and ||A||_F^2 the root of A's full
 * pyramid.  Coarser tiers are rebuilt over the kept leaves ((s11 + s12) +
 * (s21 + s22)), so the tree is that of A with its dropped leaves zeroed.
 * Only the kept leaves are packed (same layout as spamm_build_tree, addressed
 * through a per-leaf slot map), so storage follows the kept leaves instead of
 * N^2.  A dropped leaf can never pass the product's test against any leaf of
 * an operand whose squared norm is at most m, so a product of sparsified
 * trees keeps the same leaf products as the dense trees and gives the same C.
 *   tau          the tolerance of the products the tree will take part in.
 *   norm2_other  ||B||_F^2 of the other operand (0 for a square A A).
 *   flags        0 or SPAMM_TREE_BF16.
 * Synchronizes `stream` once (kept-leaf count and roots).  spamm_tree_info's
 * norm2 is ||A_sparsified||_F^2.  NaN/Inf anywhere in A -> SPAMM_E_NONFINITE.
 * Errors as spamm_build_tree_ex, plus SPAMM_E_INVAL for a bad tau or
 * norm2_other (negative, NaN/Inf), SPAMM_TREE_SUBNORMS or SPAMM_TREE_FP16.
 */
int spamm_build_tree_sparse(const float *A, int64_t n, int32_t leaf, uint32_t flags, double tau,
                            double norm2_other, void *stream, spamm_tree **out);

/*
 * Build the quadtree of the product C = A B that `plan` computed, from C and
 * the plan's schedule (Sec. II.C: truncating the product space truncates
 * the result).  A leaf of C that no kept leaf product reaches is zero by
 * construction: it is not read, its norm is +0 and it is not stored.  The
 * reached leaves are read from C and packed as in spamm_build_tree_ex
 * (addressed through a per-leaf slot map, like a sparsified tree), so the
 * norms equal those of spamm_build_tree_ex on C bit for bit, and a product
 * taking this tree gives the same C as one taking the dense tree.  This is
 * the next operand of a squaring chain (X_{s+1} = X_s X_s) without a dense
 * rebuild.
 *   C      device pointer, n x n FP32 row-major, holding the plan's product
 *          on every reached leaf (spamm_numeric of this plan, ordered before
 *          on `stream`); its other leaves are never read.
 *   plan   the plan of the product; it and C stay alive until this returns.
 *   flags  0, SPAMM_TREE_BF16 or SPAMM_TREE_FP16 (16-bit copies for a split
 *          product taking the tree; leaf 32 or 64).
 * Synchronizes `stream` twice (reached-leaf count, then the root).
 * spamm_tree_storage reports the reached leaves as stored.
 * Errors: SPAMM_E_INVAL (NULL C/plan/out, bad flags, plan on another device),
 *         SPAMM_E_NONFINITE (NaN/Inf on a reached leaf), SPAMM_E_NOMEM,
 *         SPAMM_E_HIP.
 */
int spamm_build_tree_output(const float *C, const spamm_plan *plan, uint32_t flags,
                            void *stream, spamm_tree **out);

/* Storage of a tree: leaves stored (N^2 for a dense tree), N^2, and the device
 * bytes it holds (leaf copies, norm pyramid, slot map, FP16 scale exponents).
 * Outputs may be NULL. */
int spamm_tree_storage(const spamm_tree *tree, int64_t *leaves_stored, int64_t *leaves_total,
                       size_t *device_bytes);

/* Release a tree (stream-ordered on the stream it was built on; work on other
 * streams that uses the tree must be complete).  NULL is a no-op. */
int spamm_tree_free(spamm_tree *tree);

/* Shape of a tree; any output pointer may be NULL.  norm2 = ||A||_F^2 (FP64
 * root of the norm pyramid). */
int spamm_tree_info(const spamm_tree *tree, int64_t *n, int32_t *leaf,
                    int32_t *depth, double *norm2);

/* Copy tier `tier` (0..d, or 0..d+1 with SPAMM_TREE_SUBNORMS) of the
 * squared-norm pyramid to host memory as a 2^tier x 2^tier row-major FP64
 * array (len >= 4^tier, else SPAMM_E_RANGE).  Synchronizes the tree's stream. */
int spamm_tree_norms(const spamm_tree *tree, int32_t tier, double *host, size_t len);

/* Copy the zero-padded matrix held by the tree to host memory as an
 * n_p x n_p row-major FP32 array (len >= n_p^2).  The tree keeps two copies
 * of every leaf: copy 0 is read when the tree is the left operand, copy 1
 * (stored transposed) when it is the right operand; both must reproduce the
 * same matrix.  Synchronizes. */
int spamm_tree_matrix(const spamm_tree *tree, int32_t copy, float *host, size_t len);

/* Copy the 16-bit leaf copies of a tree built with SPAMM_TREE_BF16 or
 * SPAMM_TREE_FP16 (the LOW operands of split precision, Sec. VI outlook) to
 * host memory as an n_p x n_p row-major array of raw bit patterns (len >=
 * n_p^2), copy 0 or 1 as in spamm_tree_matrix.  BF16: element (i, j) is
 * x_ij rounded to bfloat16.  FP16: element (i, j) is x_ij 2^e rounded to
 * binary16 (nearest even, a result below 2^-14 flushed to zero), e the
 * exponent of its leaf; `scale` (may be NULL, else scale_len >= N^2 for N
 * leaves per dimension) receives the exponents, leaf (I, J) at I N + J.
 * SPAMM_E_INVAL when the tree has no 16-bit copies, SPAMM_E_RANGE for short
 * buffers.  Synchronizes the tree's stream. */
int spamm_tree_matrix16(const spamm_tree *tree, int32_t copy, uint16_t *host, size_t len,
                        int32_t *scale, size_t scale_len);

/* ---- symbolic / numeric multiply (Alg. 1: collect products, then multiply) -- */

/*
 * Symbolic multiply: the tier-by-tier (i,k,j) cull of Eq. product under
 * Eq. norm condition.  A triple is kept iff s_A > 0, s_B > 0 and
 * fl64(s_A * s_B) >= fl64(tau * tau) on the stored squared norms (equality
 * keeps; zero-norm nodes are never kept, at any tau).  The plan holds the
 * kept leaf triples sorted by output tile, then k.  Asynchronous on `stream`
 * (no host synchronization).  A and B may be the same tree.
 * Errors: SPAMM_E_INVAL (null, tau < 0, tau NaN/Inf, 0 < tau < 1e-150),
 *         SPAMM_E_MISMATCH (n or leaf differ), SPAMM_E_NOMEM, SPAMM_E_HIP.
 */
int spamm_symbolic(const spamm_tree *A, const spamm_tree *B, double tau,
                   void *stream, spamm_plan **out);

/*
 * Symbolic multiply with options (split precision).  With
 * SPAMM_PREC_SPLIT_BF16 or SPAMM_PREC_SPLIT_BF16X3 (SPAMM_PREC_SPLIT_FP16) each kept leaf product is
 * also classed LOW or HIGH (see spamm_opts); both trees must have been built
 * with SPAMM_TREE_BF16 (SPAMM_TREE_FP16).
 * Errors as spamm_symbolic, plus SPAMM_E_INVAL for an unknown precision, a
 * bad low_tol or low_rel (negative, NaN/Inf, 0 < x < 1e-150, both non-zero),
 * missing 16-bit copies,
 * or sub_cull with split precision, n_b != 64 or trees without sub-norms.
 * A plan refers to both trees: they must not be freed before the plan.
 */
int spamm_symbolic_ex(const spamm_tree *A, const spamm_tree *B, const spamm_opts *opts,
                      void *stream, spamm_plan **out);

/*
 * Numeric multiply: C = sum over kept k (ascending) of A_ik B_kj for every
 * output leaf, FP32 MFMA with FP32 accumulation (Eq. product; the multiply
 * phase of Alg. 1).  Split precision: the LOW products (BF16 or scaled FP16
 * operands; with FP16 each product is accumulated on its own, scaled back
 * and added) and the HIGH ones (FP32, or compensated BF16 with
 * SPAMM_PREC_SPLIT_BF16X3) are each summed over k ascending, the LOW ones
 * first, and a leaf is their sum.  C: device pointer, n x n FP32 row-major, fully overwritten (zeros
 * where no product lands; alpha = 1, beta = 0).  C must not overlap the
 * trees' storage; it may alias the matrix a tree was built from.  Enqueue on
 * the plan's stream or order streams yourself.
 */
int spamm_numeric(const spamm_plan *plan, float *C, void *stream);

/*
 * Copy the kept leaf triples to host memory as sorted uint64 keys
 * (linear_index(i, j) << 32) | k, linear_index from Eq. linear index (row
 * bits on odd positions); with split precision bit 63 is set on LOW products.
 * *count receives K.  cap < K -> SPAMM_E_RANGE (nothing copied).
 * Synchronizes the plan's stream.
 */
int spamm_plan_tasks(const spamm_plan *plan, uint64_t *host, size_t cap, size_t *count);

/*
 * Sub-leaf culling: copy the 32 x 32 sub-products performed by the last
 * spamm_numeric of the plan as sorted uint64 keys (linear_index(i, j) << 32) | k
 * over the grid of 32 x 32 sub-blocks (i, j, k < 2N), i.e. the task keys of
 * the same product on a tree with 32 x 32 leaves.  *count receives their
 * number; cap too small -> SPAMM_E_RANGE.  SPAMM_E_INVAL when the plan does
 * not cull sub-leaves.  Synchronizes the plan's stream.
 */
int spamm_plan_subtasks(const spamm_plan *plan, uint64_t *host, size_t cap, size_t *count);

/* Kept counts per tier and work totals.  Synchronizes the plan's stream. */
int spamm_plan_stats(const spamm_plan *plan, spamm_stats *out);

/* Release a plan (stream-ordered).  NULL is a no-op. */
int spamm_plan_free(spamm_plan *plan);

/* ---- one-call multiply --------------------------------------------------- */

/* C = A B under the SpAMM condition with tolerance tau: symbolic + numeric on
 * `stream`, with a temporary plan.  Asynchronous (no host synchronization). */
int spamm_multiply(const spamm_tree *A, const spamm_tree *B, double tau, float *C,
                   void *stream);

/* As spamm_multiply; when `stats` is not NULL the call also times the cull
 * and the leaf GEMM with HIP events on `stream`, synchronizes, and fills it. */
int spamm_multiply_ex(const spamm_tree *A, const spamm_tree *B, double tau, float *C,
                      void *stream, spamm_stats *stats);

/* Product with options: symbolic + numeric on `stream` with a temporary plan;
 * `stats` as for spamm_multiply_ex (NULL: no timing, no synchronization). */
int spamm_multiply_opts(const spamm_tree *A, const spamm_tree *B, const spamm_opts *opts,
                        float *C, void *stream, spamm_stats *stats);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * product of spamm_multiply_opts (symbolic + numeric on `stream`, no stats)
 * with the task arena in a fixed device block of the library instead of an
 * allocation.  The block (SPAMM_NOALLOC_SCRATCH_BYTES on every device the
 * library runs on, held until the process ends) is found once per device;
 * the call itself allocates nothing (no hipMalloc, no pool, no host heap)
 * and never synchronizes.  Trees, A, B and C are the caller's, as for
 * spamm_multiply_opts.
 * Every call on one device shares that device's block, and it keeps the
 * last call's contents: calls that overlap on one device (on different
 * streams or threads) race and must be ordered by the caller.
 * A product whose task arena exceeds the block is refused with SPAMM_E_RANGE:
 * depth d <= 8 (at most 256 leaves per dimension) fits in every precision
 * and with sub-leaf culling.  Other errors as spamm_symbolic_ex.
 */
#define SPAMM_NOALLOC_SCRATCH_BYTES (64u << 20)
int spamm_multiply_noalloc(const spamm_tree *A, const spamm_tree *B, const spamm_opts *opts,
                           float *C, void *stream);

/* ---- serving: continuous batching of products and squaring chains -------- */

/*
 * A server owns one scheduler thread, `max_slots` streams and a device-memory
 * budget on the device current at spamm_server_create.  Each slot keeps one
 * device arena for the trees and the task arena of the request it runs
 * (spamm_request_footprint bytes; C is the caller's), reused across requests
 * and grown when needed.  Requests wait in a FIFO queue; the scheduler admits
 * the head when a slot is free and its arena fits: idle arenas are released
 * to make room, and the arenas together never exceed the budget.  An
 * admitted request's trees and cull run on its slot's stream, overlapping
 * other requests' work;
 * the leaf products of every request whose cull has been enqueued are
 * gathered into one batched leaf-GEMM launch group (up to 16 requests of one
 * leaf size, uneven n and tau; the FP32, BF16-split and FP16-split requests
 * of a group get one launch per kind) on the server's
 * GEMM stream, so small products share the chip.  A squaring chain (the
 * matrix square is the central step of density-matrix purification,
 * Sec. IV.B) stays on the device: each step's product is rebuilt into a tree
 * and squared again without a host round trip.  The rebuild reads only the
 * leaves that the step's kept products reach (the others are zero, as in
 * spamm_build_tree_output), and the leaf GEMM of every step before the last
 * writes only the blocks of C that have products; the last step writes all
 * of C.
 *
 * Determinism: every output leaf is computed by one workgroup with a fixed k
 * order, so a request's C is bit-identical whether it runs alone or in a mix.
 */
typedef struct spamm_server spamm_server;

typedef struct spamm_request {
    const float *A;      /* device, n x n FP32 row-major (lda = n)                    */
    const float *B;      /* device n x n, or NULL for B = A; must be NULL or A when    */
                         /* chain_len > 0                                             */
    float *C;            /* device, n x n FP32 row-major output; may alias A          */
    int64_t n;           /* order, >= 1                                                */
    int32_t leaf;        /* n_b in {16, 32, 64} (32 or 64 for split precision)         */
    int32_t precision;   /* SPAMM_PREC_FP32, SPAMM_PREC_SPLIT_BF16, _SPLIT_FP16 or     */
                         /* _SPLIT_BF16X3                                              */
    double tau;          /* SpAMM tolerance of every product (as spamm_symbolic)      */
    double low_tol;      /* split precision: absolute LOW threshold (as spamm_opts)   */
    int32_t chain_len;   /* 0: C = A B.  L in 1..64: X_0 = A, X_{s+1} = X_s X_s under  */
                         /* tau (each X_s rebuilt into a tree), C = X_L               */
    double low_rel;      /* split precision: relative LOW threshold theta (as         */
                         /* spamm_opts), taken against each step's own roots         */
} spamm_request;

typedef struct spamm_result {
    int32_t status;      /* SPAMM_OK, or the request's error (e.g. SPAMM_E_NONFINITE    */
                         /* when an input or an intermediate square holds NaN/Inf)   */
    int32_t steps;       /* products performed (1, or chain_len)                      */
    int64_t tasks;       /* leaf products over all steps                              */
    int64_t tasks_low;   /* of which LOW                                              */
    double  flops;       /* 2 n_b^3 tasks                                             */
    double  queue_ms;    /* submit -> admission (host clock)                          */
    double  latency_ms;  /* submit -> completion seen by the scheduler (host clock)   */
} spamm_result;

/* Counters of a server since its creation (spamm_server_info). */
typedef struct spamm_server_stats {
    int64_t  admitted;           /* requests admitted                                */
    int64_t  completed;          /* requests finished (any status)                   */
    int64_t  queued;             /* requests waiting for admission now               */
    int64_t  launches;           /* batched leaf-GEMM launch groups (one launch per  */
                                 /* precision present in the group)                   */
    int64_t  launched_products;  /* products over all launch groups                  */
    int64_t  max_batch;          /* most products in one launch group                */
    int64_t  peak_active;        /* most requests admitted at once                   */
    uint64_t used;               /* bytes held by the slot arenas now                */
    uint64_t peak_used;          /* most bytes held by the slot arenas at once       */
    uint64_t budget;             /* hbm_budget                                       */
    double   sched_cpu_ms;       /* CPU time used by the scheduler thread so far     */
    double   sched_wall_ms;      /* wall time since the scheduler thread started     */
    int64_t  rounds;             /* rounds: shared launches of the tree builds and   */
                                 /* culls of several requests' steps                 */
    int64_t  round_steps;        /* request steps built and culled in rounds         */
} spamm_server_stats;

/*
 * Create a server on the current device.  hbm_budget: bytes of device memory
 * the slot arenas may hold at once (> 0).  max_slots: requests admitted
 * at once, 1..64.  Errors: SPAMM_E_INVAL, SPAMM_E_NOMEM, SPAMM_E_HIP.
 */
int spamm_server_create(size_t hbm_budget, int32_t max_slots, spamm_server **out);

/*
 * Device bytes of a request's slot arena (its trees and task arena, and for
 * a chain the keep flags, slots and scan partials of its step trees; buffers
 * at 256-byte aligned offsets); also validates the request (host only, no device call).  Errors: SPAMM_E_INVAL (null
 * pointers, n < 1, bad leaf, precision, tau, low_tol, low_rel (as
 * spamm_symbolic_ex), chain_len outside 0..64,
 * a chain with B not NULL and not A, split precision with leaf 16),
 * SPAMM_E_RANGE (more than 1024 leaves per dimension).
 */
int spamm_request_footprint(const spamm_request *req, size_t *bytes);

/*
 * Queue a request (thread-safe, non-blocking).  The caller keeps A, B and C
 * alive and unwritten-by-others until the request is done; A and B must
 * already hold their values (the server's streams do not wait on the
 * caller's).  *ticket receives a positive id.  Errors: as
 * spamm_request_footprint; SPAMM_E_NOMEM when the footprint exceeds the
 * whole budget (it could never be admitted); SPAMM_E_BUSY when 65536
 * requests are already queued; SPAMM_E_INVAL after destroy began.
 */
int spamm_submit(spamm_server *server, const spamm_request *req, uint64_t *ticket);

/*
 * Non-blocking, thread-safe.  Returns SPAMM_PENDING while the request is
 * queued or running; otherwise fills *out (may be NULL), forgets the ticket
 * and returns SPAMM_OK (the request's own status is out->status).
 * SPAMM_E_INVAL for an unknown or already collected ticket.
 */
int spamm_poll(spamm_server *server, uint64_t ticket, spamm_result *out);

/* Copy the server's counters (thread-safe). */
int spamm_server_info(spamm_server *server, spamm_server_stats *out);

/*
 * Stop the server: queued requests that were not admitted are dropped
 * (their C is not written), admitted ones run to completion, then the
 * scheduler thread, streams and memory are released.  No other call on the
 * server may run concurrently with or after this one.  NULL is a no-op.
 */
int spamm_server_destroy(spamm_server *server);

/* ---- errors --------------------------------------------------------------- */
const char *spamm_strerror(int code);
const char *spamm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SPAMM_H */
