// Internal runtime pieces shared by the one-call API (api.hip) and the
// serving loop (server.hip).  Not part of the C ABI.
#pragma once

#include <stddef.h>

#include "common.hpp"

namespace spamm {

// Error plumbing: set the calling thread's message, return code.
int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);

// Depth d and padded order n_p = n_b 2^d of an n x n operand (SPAMM_E_RANGE
// past kMaxDepth tiers).
int tree_depth(int64_t n, int32_t leaf, int32_t *d, int64_t *np);

// Current device, with the library's stream-ordered memory pool for it
// created (once per device).
int prepare_device(int *dev);

// Stream-ordered allocation on `s` from the pool of device `dev`, which
// prepare_device has created (hipErrorInvalidDevice otherwise).  Freed with
// hipFreeAsync.
hipError_t dev_alloc_async(int dev, void **ptr, size_t bytes, hipStream_t s);

// Validates and enqueues a tree build on `s` without synchronizing; the
// root squared norm is copied to *root_dst (pinned host memory, may be null)
// asynchronously.  With `arena` (device memory of tree_device_bytes bytes,
// 256-byte aligned) the tree's buffers are carved from it and never freed by
// the tree; otherwise they come from the stream-ordered pool.  On error
// nothing stays allocated.
int tree_build_async(const float *A, int64_t n, int32_t leaf, uint32_t flags, hipStream_t s,
                     double *root_dst, spamm_tree **out, void *arena = nullptr);

// Tree of the product C that plan `p` computed (only the leaves a kept
// product reaches are read and stored, leaf l at slot[l]; the others are
// zero), enqueued on `s` without synchronizing.  With `arena` (tree_device_bytes
// bytes) and `map` (output_map_bytes(depth) bytes: keep flags, slots, scan
// partials) the buffers are carved from them; otherwise one allocation of the
// tree's own.  The plan's schedule is read by the enqueued work.
int tree_build_output_async(const float *C, const spamm_plan *p, uint32_t flags, hipStream_t s,
                            spamm_tree **out, void *arena = nullptr, void *map = nullptr);
size_t output_map_bytes(int32_t depth);

// spamm_symbolic_ex on stream `s`, optionally with the plan's buffers carved
// from `arena` (plan_device_bytes bytes, 256-byte aligned).
int symbolic_async(const spamm_tree *A, const spamm_tree *B, const spamm_opts *opts,
                   hipStream_t s, void *arena, spamm_plan **out);

// Device bytes of one tree / one plan of depth d, buffers at 256-byte
// aligned offsets (the arena sizes; also admission control).
size_t tree_device_bytes(int64_t n, int32_t leaf, uint32_t flags);

// Tree flags a request of this precision needs (16-bit copies for split).
inline uint32_t tree_flags_for(int32_t precision)
{
    return precision == SPAMM_PREC_SPLIT_BF16 || precision == SPAMM_PREC_SPLIT_BF16X3
               ? SPAMM_TREE_BF16
           : precision == SPAMM_PREC_SPLIT_FP16 ? SPAMM_TREE_FP16 : 0u;
}
size_t plan_device_bytes(int depth, bool split);

// SPAMM_PREC_SPLIT_BF16X3: an entry at or above 2^128 (1 - 2^-9) rounds to
// an infinite bfloat16 part.  No entry reaches it while the operand's squared
// Frobenius norm stays below the square of that bound.
constexpr double kX3MaxRoot2 = (1.0 - 1.0 / 512) * (1.0 - 1.0 / 512) * 0x1p256;

// Leaf GEMM launches (gemm.hip): a plan's job and kind, and one batched
// launch of jobs of one kind and leaf size.
void plan_jobs(const spamm_plan *p, float *C, GemmJob &j);
GemmKind plan_kind(const spamm_plan *p);
hipError_t launch_gemm_jobs(int leaf, GemmKind kind, const GemmJobs &jobs, hipStream_t s);

// Exclusive scan of m uint32 (out[m] = total); partials: scan_partials_len(m).
hipError_t launch_scan_u32(const uint32_t *in, uint32_t m, uint32_t *out, uint32_t *partials,
                           hipStream_t s);
size_t scan_partials_len(uint32_t m);

// Epsilon-sparsified build (norms.hip): dense norms, drop, slots, pyramid;
// then the pack of the kept leaves.
hipError_t launch_sparse_norms(const float *A, int64_t n, int leaf, int depth, double *norms,
                               double tau, double other2, uint32_t *keep, uint32_t *slot,
                               uint32_t *partials, double *root_dense, hipStream_t s);
hipError_t launch_sparse_pack(const float *A, int64_t n, int leaf, int depth, float *tiles,
                              float *tilesT, uint16_t *t16, uint16_t *tT16, const uint32_t *keep,
                              const uint32_t *slot, hipStream_t s);

// ---- batched tree builds and culls of several products ----------------------
// Tables of jobs passed by value to one launch; a workgroup finds its job by
// block0 (ascending).  Used by the serving loop to build and cull the steps of
// many requests in a few launches.
constexpr int kMaxRound = 16;

template <typename J>
struct Jobs {
    int32_t njobs;
    uint32_t nblocks;      // total grid
    J job[kMaxRound];
};

template <typename J>
__device__ inline const J &job_at(const Jobs<J> &jobs, uint32_t bid)
{
    // independent tests (no chain of dependent loads)
    int j = 0;
#pragma unroll
    for (int i = 1; i < kMaxRound; ++i)
        j += (i < jobs.njobs && bid >= jobs.job[i].block0) ? 1 : 0;
    return jobs.job[j];
}

struct PackJob {           // leaf norms and packed copies of one tree
    const float *A;
    int64_t n;
    float *tiles, *tilesT;
    uint16_t *t16, *tT16;
    int32_t *scale16;
    double *leafn, *parent;
    const uint32_t *keep;  // with known_zero: the leaves not kept are zero
    uint32_t ntiles, block0;
    uint32_t cb;           // blocks of 4 leaves per workgroup (1 .. kPackChunk)
    int32_t known_zero;
    // a pack after the norms: leaf norms, the two roots and tau^2 of the
    // product the tree takes part in (leaves no product can keep are skipped)
    const double *drop_s, *rootA, *rootB;
    double T2;
};

struct KeepJob {           // output-leaf keep flags from a product's schedule
    const uint32_t *browptr, *bent, *browptr_lo, *bent_lo;
    uint32_t *keep;
    uint32_t nblocks, nleaves, block0;
};

struct PyrJob {            // one workgroup per tree
    double *norms;
    int32_t top;
    uint32_t block0;
};

struct TopJob {            // root and tiers 1..top, one workgroup per plan
    const double *nA, *nB;
    uint32_t *rowptr, *list0, *list1;
    uint64_t *leafK;
    double T2;
    int32_t top;
    uint32_t block0;
};

struct TierJob {           // one tier below the leaves of one plan
    const double *tA, *tB;
    const uint32_t *prow, *plist;
    uint32_t *counts, *crow, *clist;
    double T2;
    uint32_t np, block0;
};

struct LeafJob {           // the leaf tier of one plan
    const double *tA, *tB, *nA, *nB;
    const uint32_t *prow, *plist;
    uint32_t *counts, *browptr, *bent, *browptr_lo, *bent_lo;
    uint64_t *leafK;
    uint64_t *rout;        // 5 words: HIGH and LOW products, 0, the two roots
    double T2, L2, theta2;
    uint32_t np, block0;
    int32_t split;
};

// ---- rounds: the tree builds and culls of several products in shared
// launches (serving loop).  Trees and plans are set up on the host with
// their buffers carved (tree_prepare, plan_prepare), then built and culled
// together; depths 1..kRoundMaxDepth.
constexpr int kRoundMaxDepth = 8;

struct RoundTree {
    const spamm_tree *tree;     // carved, not yet built
    const float *src;           // the matrix (A, B, or the product of `from`)
    const spamm_plan *from;     // output tree: the plan that computed src, else null
    // tau^2 of the product the tree takes part in, and its other operand
    // (the tree itself for a square).  T2 > 0: the norms are built first and
    // only the leaves some kept product can read are packed
    double T2;
    const spamm_tree *other;
};

// Carves a tree (tree_device_bytes bytes of `arena`) without building it.
// `keep`: for an output tree, N^2 words of keep flags (leaves stay at their
// linear index, so the tree needs no slot map), else null.
int tree_prepare(int64_t n, int32_t leaf, uint32_t flags, void *arena, uint32_t *keep,
                 hipStream_t s, spamm_tree **out);
// Sets up a plan with its buffers carved from `arena`, without culling.
int plan_prepare(const spamm_tree *A, const spamm_tree *B, const spamm_opts *opts,
                 hipStream_t s, void *arena, spamm_plan **out);
hipError_t launch_build_round(const RoundTree *trees, int ntrees, hipStream_t s);
// rout: 5 words per plan (HIGH and LOW leaf products, 0, the roots' bits).
hipError_t launch_cull_round(const spamm_plan *const *plans, int nplans, uint64_t *rout,
                             hipStream_t s);

// Steady clock in microseconds (request timestamps).
double now_us();

}  // namespace spamm
