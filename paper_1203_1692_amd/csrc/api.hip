// C ABI of libspamm: argument checks, device memory (a stream-ordered pool
// of the library's own per device), launches and host-side exports.  No computation of the
// multiply happens here; every step runs in the kernels of norms.hip,
// cull.hip and gemm.hip.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <new>
#include <vector>

#include "runtime.hpp"

namespace spamm {
hipError_t launch_build(const float *A, int64_t n, int leaf, int depth, float *tiles,
                        float *tilesT, uint16_t *t16, uint16_t *tT16, int32_t *scale16,
                        double *norms, bool sub, hipStream_t s);
hipError_t launch_cull(spamm_plan *p, hipStream_t s);
hipError_t launch_gemm(const spamm_plan *p, float *C, hipStream_t s);
hipError_t launch_output_map(const uint32_t *browptr, const uint32_t *bent,
                             const uint32_t *browptr_lo, const uint32_t *bent_lo,
                             uint32_t nblocks, int depth, uint32_t *keep, uint32_t *slot,
                             uint32_t *partials, hipStream_t s);
hipError_t launch_output_pack(const float *C, int64_t n, int leaf, int depth, float *tiles,
                              float *tilesT, uint16_t *t16, uint16_t *tT16, int32_t *scale16,
                              double *norms, const uint32_t *keep, const uint32_t *slot,
                              hipStream_t s);
}  // namespace spamm

using namespace spamm;

namespace {
thread_local char g_err[512] = "";
}  // namespace

namespace spamm {

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    if (e == hipErrorOutOfMemory)
        return fail(SPAMM_E_NOMEM, "%s: out of device memory", what);
    return fail(SPAMM_E_HIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

#define HIP_TRY(expr, what)                       \
    do {                                          \
        hipError_t e_ = (expr);                   \
        if (e_ != hipSuccess)                     \
            return hip_fail(e_, what);            \
    } while (0)

// One stream-ordered memory pool per device, created on first use and owned
// by the library for the life of the process.  Its release threshold is
// unbounded so that freed blocks stay cached for the next tree or plan; the
// device's default pool, which other code in the process may use, is left as
// it is.
namespace {
hipMemPool_t g_pool[64] = {};
std::mutex g_pool_mu;
}  // namespace

int prepare_device(int *dev)
{
    HIP_TRY(hipGetDevice(dev), "hipGetDevice");
    if (*dev < 0 || *dev >= 64)
        return fail(SPAMM_E_HIP, "device ordinal %d out of range", *dev);
    std::lock_guard<std::mutex> lock(g_pool_mu);
    if (g_pool[*dev] == nullptr) {
        hipMemPoolProps props;
        memset(&props, 0, sizeof props);
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = *dev;
        hipMemPool_t pool = nullptr;
        HIP_TRY(hipMemPoolCreate(&pool, &props), "hipMemPoolCreate");
        uint64_t thr = UINT64_MAX;
        hipError_t e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        if (e != hipSuccess) {
            hipMemPoolDestroy(pool);
            return hip_fail(e, "hipMemPoolSetAttribute");
        }
        g_pool[*dev] = pool;
    }
    return SPAMM_OK;
}

hipError_t dev_alloc_async(int dev, void **ptr, size_t bytes, hipStream_t s)
{
    hipMemPool_t pool;
    {
        std::lock_guard<std::mutex> lock(g_pool_mu);
        pool = (dev >= 0 && dev < 64) ? g_pool[dev] : nullptr;
    }
    if (pool == nullptr)
        return hipErrorInvalidDevice;
    return hipMallocFromPoolAsync(ptr, bytes, pool, s);
}

double now_us()
{
    using namespace std::chrono;
    return (double)duration_cast<nanoseconds>(steady_clock::now().time_since_epoch()).count() * 1e-3;
}

int tree_depth(int64_t n, int32_t leaf, int32_t *d, int64_t *np)
{
    int32_t t = 0;
    int64_t p = leaf;
    while (p < n) {
        p *= 2;
        t += 1;
        if (t > kMaxDepth)
            return fail(SPAMM_E_RANGE, "n = %lld needs more than %d tiers at leaf %d",
                        (long long)n, kMaxDepth, leaf);
    }
    *d = t;
    *np = p;
    return SPAMM_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Device buffers of a plan of depth d (worst case: every candidate kept),
// each at a 256-byte aligned offset of one block.
struct PlanSizes {
    int64_t rp_off[kMaxDepth + 1];
    size_t rowptr, list[2], counts, partials, browptr, bent;
};

static PlanSizes plan_sizes(int d)
{
    PlanSizes z{};
    int64_t rp = 0;
    for (int t = 0; t < d; ++t) {
        z.rp_off[t] = rp;
        rp += (int64_t(1) << (2 * t)) + 1;
    }
    z.rp_off[d] = rp;
    int64_t cap_list[2] = {1, 1};
    for (int t = 0; t < d; ++t)
        cap_list[t & 1] = std::max(cap_list[t & 1], int64_t(1) << (3 * t));
    const int64_t nblocks = d == 0 ? 1 : (int64_t(1) << (2 * (d - 1)));
    const int64_t ncounts = nblocks;
    const int64_t cap_bent = d == 0 ? 1 : nblocks * (int64_t(1) << d);
    z.rowptr = sizeof(uint32_t) * (size_t)std::max<int64_t>(rp, 2);
    z.list[0] = sizeof(uint32_t) * (size_t)cap_list[0];
    z.list[1] = sizeof(uint32_t) * (size_t)cap_list[1];
    z.counts = sizeof(uint32_t) * 4 * (size_t)ncounts;
    z.partials = sizeof(uint32_t) * scan_partials_len((uint32_t)std::max<int64_t>(ncounts, 1));
    z.browptr = sizeof(uint32_t) * (size_t)(nblocks + 1);
    z.bent = sizeof(uint32_t) * (size_t)cap_bent;
    return z;
}

// The plan's buffers in allocation order (split adds the LOW schedule).
struct PlanBuf { void **dst; size_t bytes; };

static int plan_bufs(spamm_plan *p, const PlanSizes &z, bool split, bool sub, PlanBuf *out)
{
    int k = 0;
    out[k++] = {(void **)&p->rowptr, z.rowptr};
    out[k++] = {(void **)&p->list[0], z.list[0]};
    out[k++] = {(void **)&p->list[1], z.list[1]};
    out[k++] = {(void **)&p->counts, z.counts};
    out[k++] = {(void **)&p->partials, z.partials};
    out[k++] = {(void **)&p->browptr, z.browptr};
    out[k++] = {(void **)&p->bent, z.bent};
    // [0] HIGH, [1] LOW leaf products, [2] sub-products, [3]/[4] the roots
    out[k++] = {(void **)&p->leafK, 5 * sizeof(uint64_t)};
    if (split) {
        out[k++] = {(void **)&p->browptr_lo, z.browptr};
        out[k++] = {(void **)&p->bent_lo, z.bent};
    }
    if (sub)
        out[k++] = {(void **)&p->submask, z.bent};   // 4 bytes per leaf-tier entry
    return k;
}

size_t plan_device_bytes(int depth, bool split)
{
    spamm_plan dummy{};
    PlanBuf b[12];
    const int k = plan_bufs(&dummy, plan_sizes(depth), split, false, b);
    size_t total = 0;
    for (int i = 0; i < k; ++i)
        total += align256(b[i].bytes);
    return total;
}

// Tree buffers: left and right FP32 leaf copies, optional 16-bit copies
// (BF16, or FP16 with a scale exponent per leaf), the norm pyramid; 256-byte
// aligned offsets of one block.
struct TreeLayout {
    size_t tiles, tilesT, t16, tT16, scale16, norms, total;
};

static TreeLayout tree_layout(int64_t np, int32_t d, uint32_t flags)
{
    const bool copies16 = (flags & (SPAMM_TREE_BF16 | SPAMM_TREE_FP16)) != 0;
    const bool fp16 = (flags & SPAMM_TREE_FP16) != 0;
    const bool sub = (flags & SPAMM_TREE_SUBNORMS) != 0;
    TreeLayout L{};
    const size_t tile = sizeof(float) * (size_t)np * (size_t)np;
    const size_t norm = sizeof(double) * (size_t)tier_offset(d + (sub ? 2 : 1));
    size_t o = 0;
    L.tiles = o;
    o += align256(tile);
    L.tilesT = o;
    o += align256(tile);
    L.t16 = o;
    o += copies16 ? align256(tile / 2) : 0;
    L.tT16 = o;
    o += copies16 ? align256(tile / 2) : 0;
    L.scale16 = o;
    o += fp16 ? align256(sizeof(int32_t) * ((size_t)1 << (2 * d))) : 0;
    L.norms = o;
    o += align256(norm);
    L.total = o;
    return L;
}

size_t tree_device_bytes(int64_t n, int32_t leaf, uint32_t flags)
{
    int32_t d = 0;
    int64_t p = leaf;
    while (p < n) {
        p *= 2;
        d += 1;
    }
    return tree_layout(p, d, flags).total;
}

int tree_build_async(const float *A, int64_t n, int32_t leaf, uint32_t flags, hipStream_t s,
                     double *root_dst, spamm_tree **out, void *arena)
{
    if (out == nullptr)
        return fail(SPAMM_E_INVAL, "out is NULL");
    *out = nullptr;
    if (A == nullptr)
        return fail(SPAMM_E_INVAL, "A is NULL");
    if (n < 1)
        return fail(SPAMM_E_INVAL, "n = %lld < 1", (long long)n);
    if (leaf != 16 && leaf != 32 && leaf != 64)
        return fail(SPAMM_E_INVAL, "leaf = %d not in {16, 32, 64}", leaf);
    if ((flags & ~(SPAMM_TREE_BF16 | SPAMM_TREE_SUBNORMS | SPAMM_TREE_FP16)) != 0)
        return fail(SPAMM_E_INVAL, "unknown tree flags 0x%x", flags);
    const bool bf16 = (flags & SPAMM_TREE_BF16) != 0;
    const bool fp16 = (flags & SPAMM_TREE_FP16) != 0;
    const bool sub = (flags & SPAMM_TREE_SUBNORMS) != 0;
    if (bf16 && fp16)
        return fail(SPAMM_E_INVAL, "a tree keeps BF16 or FP16 leaf copies, not both");
    if ((bf16 || fp16) && leaf == 16)
        return fail(SPAMM_E_INVAL, "16-bit leaf copies need leaf 32 or 64");
    if (sub && leaf != 64)
        return fail(SPAMM_E_INVAL, "sub-block norms need leaf 64");
    int32_t d;
    int64_t np;
    int rc = tree_depth(n, leaf, &d, &np);
    if (rc)
        return rc;
    int dev;
    if ((rc = prepare_device(&dev)))
        return rc;
    const TreeLayout L = tree_layout(np, d, flags);

    spamm_tree *t = new (std::nothrow) spamm_tree();
    if (!t)
        return fail(SPAMM_E_NOMEM, "host allocation failed");
    t->device = dev;
    t->stream = s;
    t->n = n;
    t->np = np;
    t->leaf = leaf;
    t->depth = d;
    t->sub = sub;
    t->stored = int64_t(1) << (2 * d);
    // one block for every buffer: the caller's arena, else an allocation of
    // the tree's own
    hipError_t e = hipSuccess;
    char *base = (char *)arena;
    if (arena != nullptr) {
        t->borrowed = true;
    } else {
        e = dev_alloc_async(dev, &t->block, L.total, s);
        if (e != hipSuccess)
            t->block = nullptr;
        base = (char *)t->block;
    }
    if (e == hipSuccess) {
        t->tiles = (float *)(base + L.tiles);
        t->tilesT = (float *)(base + L.tilesT);
        t->tiles16 = bf16 || fp16 ? (uint16_t *)(base + L.t16) : nullptr;
        t->tilesT16 = bf16 || fp16 ? (uint16_t *)(base + L.tT16) : nullptr;
        t->fp16 = fp16;
        t->scale16 = fp16 ? (int32_t *)(base + L.scale16) : nullptr;
        t->norms = (double *)(base + L.norms);
        // the 16-bit copies (and FP16 scale exponents) come with the norm pass
        e = launch_build(A, n, leaf, d, t->tiles, t->tilesT, t->tiles16, t->tilesT16, t->scale16,
                         t->norms, sub, s);
    }
    if (e == hipSuccess && root_dst != nullptr)
        e = hipMemcpyAsync(root_dst, t->norms, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) {
        rc = hip_fail(e, "tree build");
        spamm_tree_free(t);
        return rc;
    }
    *out = t;
    return SPAMM_OK;
}

// keep flags, slots and scan partials of an output tree of depth d
struct OutputMap {
    size_t keep, slot, partials, total;
};

static OutputMap output_map(int32_t d)
{
    const uint32_t N2 = 1u << (2 * d);
    OutputMap M{};
    M.keep = 0;
    M.slot = align256(sizeof(uint32_t) * N2);
    M.partials = M.slot + align256(sizeof(uint32_t) * ((size_t)N2 + 1));
    M.total = M.partials + align256(sizeof(uint32_t) * scan_partials_len(N2));
    return M;
}

size_t output_map_bytes(int32_t depth) { return output_map(depth).total; }

static int check_output_args(const float *C, const spamm_plan *p, uint32_t flags, int *dev)
{
    if (C == nullptr || p == nullptr)
        return fail(SPAMM_E_INVAL, "C or plan is NULL");
    if ((flags & ~(SPAMM_TREE_BF16 | SPAMM_TREE_FP16)) != 0)
        return fail(SPAMM_E_INVAL, "flags 0x%x: an output tree takes SPAMM_TREE_BF16 or "
                    "SPAMM_TREE_FP16 only", flags);
    if ((flags & SPAMM_TREE_BF16) && (flags & SPAMM_TREE_FP16))
        return fail(SPAMM_E_INVAL, "a tree keeps BF16 or FP16 leaf copies, not both");
    if (flags != 0 && p->leaf == 16)
        return fail(SPAMM_E_INVAL, "16-bit leaf copies need leaf 32 or 64");
    int rc = prepare_device(dev);
    if (rc)
        return rc;
    if (*dev != p->device)
        return fail(SPAMM_E_INVAL, "the plan lives on device %d, current device is %d",
                    p->device, *dev);
    return SPAMM_OK;
}

static spamm_tree *output_tree_shell(const spamm_plan *p, int dev, hipStream_t s)
{
    spamm_tree *t = new (std::nothrow) spamm_tree();
    if (!t)
        return nullptr;
    t->device = dev;
    t->stream = s;
    t->n = p->n;
    t->np = p->A->np;
    t->leaf = p->leaf;
    t->depth = p->depth;
    return t;
}

static void output_tree_carve(spamm_tree *t, char *base, const TreeLayout &L, uint32_t flags)
{
    const bool fp16 = (flags & SPAMM_TREE_FP16) != 0, c16 = flags != 0;
    t->tiles = (float *)(base + L.tiles);
    t->tilesT = (float *)(base + L.tilesT);
    t->tiles16 = c16 ? (uint16_t *)(base + L.t16) : nullptr;
    t->tilesT16 = c16 ? (uint16_t *)(base + L.tT16) : nullptr;
    t->fp16 = fp16;
    t->scale16 = fp16 ? (int32_t *)(base + L.scale16) : nullptr;
    t->norms = (double *)(base + L.norms);
}

int tree_prepare(int64_t n, int32_t leaf, uint32_t flags, void *arena, uint32_t *keep,
                 hipStream_t s, spamm_tree **out)
{
    if (out == nullptr || arena == nullptr)
        return fail(SPAMM_E_INVAL, "out or arena is NULL");
    *out = nullptr;
    if ((flags & ~(SPAMM_TREE_BF16 | SPAMM_TREE_FP16)) != 0 ||
        ((flags & SPAMM_TREE_BF16) && (flags & SPAMM_TREE_FP16)) || (flags != 0 && leaf == 16))
        return fail(SPAMM_E_INVAL, "tree flags 0x%x at leaf %d", flags, leaf);
    int32_t d;
    int64_t np;
    int rc = tree_depth(n, leaf, &d, &np);
    if (rc)
        return rc;
    int dev;
    if ((rc = prepare_device(&dev)))
        return rc;
    spamm_tree *t = new (std::nothrow) spamm_tree();
    if (!t)
        return fail(SPAMM_E_NOMEM, "host allocation failed");
    t->device = dev;
    t->stream = s;
    t->n = n;
    t->np = np;
    t->leaf = leaf;
    t->depth = d;
    t->stored = int64_t(1) << (2 * d);
    t->borrowed = true;
    output_tree_carve(t, (char *)arena, tree_layout(np, d, flags), flags);
    t->keep = keep;
    *out = t;
    return SPAMM_OK;
}

int tree_build_output_async(const float *C, const spamm_plan *p, uint32_t flags, hipStream_t s,
                            spamm_tree **out, void *arena, void *map)
{
    if (out == nullptr)
        return fail(SPAMM_E_INVAL, "out is NULL");
    *out = nullptr;
    int dev;
    int rc = check_output_args(C, p, flags, &dev);
    if (rc)
        return rc;
    if ((arena == nullptr) != (map == nullptr))
        return fail(SPAMM_E_INVAL, "give both the tree arena and the output map, or neither");
    const int32_t d = p->depth;
    const TreeLayout L = tree_layout(p->A->np, d, flags);
    const OutputMap M = output_map(d);
    spamm_tree *t = output_tree_shell(p, dev, s);
    if (!t)
        return fail(SPAMM_E_NOMEM, "host allocation failed");
    t->stored = int64_t(1) << (2 * d);      // capacity: the reached leaves fill a prefix
    hipError_t e = hipSuccess;
    char *base = (char *)arena, *mbase = (char *)map;
    if (arena != nullptr) {
        t->borrowed = true;
    } else {
        e = dev_alloc_async(dev, &t->block, L.total + M.total, s);
        if (e != hipSuccess)
            t->block = nullptr;
        base = (char *)t->block;
        mbase = base + L.total;
    }
    if (e == hipSuccess) {
        output_tree_carve(t, base, L, flags);
        t->keep = (uint32_t *)(mbase + M.keep);
        t->slot = (uint32_t *)(mbase + M.slot);
        const bool split = p->precision != SPAMM_PREC_FP32;
        e = launch_output_map(p->browptr, p->bent, split ? p->browptr_lo : nullptr,
                              split ? p->bent_lo : nullptr, (uint32_t)p->nblocks, d, t->keep,
                              t->slot, (uint32_t *)(mbase + M.partials), s);
        if (e == hipSuccess)
            e = launch_output_pack(C, p->n, p->leaf, d, t->tiles, t->tilesT, t->tiles16,
                                   t->tilesT16, t->scale16, t->norms, t->keep, t->slot, s);
    }
    if (e != hipSuccess) {
        rc = hip_fail(e, "output tree build");
        spamm_tree_free(t);
        return rc;
    }
    *out = t;
    return SPAMM_OK;
}

static int check_tol(double v, const char *name)
{
    if (!(v >= 0.0) || isinf(v))
        return fail(SPAMM_E_INVAL, "%s = %g must be finite and >= 0", name, v);
    if (v > 0.0 && v < 1e-150)
        return fail(SPAMM_E_INVAL, "%s = %g below 1e-150 (its square would underflow)", name, v);
    return SPAMM_OK;
}

// Validates a product's operands and options against device `dev` and fills
// *p (host fields only, no allocation, no device call); *bytes receives the
// size of the plan's one device block (its buffers at 256-byte aligned
// offsets).
static int plan_setup(spamm_plan *p, const spamm_tree *A, const spamm_tree *B,
                      const spamm_opts *opts, int dev, hipStream_t s, size_t *bytes)
{
    if (A == nullptr || B == nullptr || opts == nullptr)
        return fail(SPAMM_E_INVAL, "tree or options NULL");
    int rc;
    if ((rc = check_tol(opts->tau, "tau")))
        return rc;
    if (opts->precision != SPAMM_PREC_FP32 && opts->precision != SPAMM_PREC_SPLIT_BF16 &&
        opts->precision != SPAMM_PREC_SPLIT_FP16 && opts->precision != SPAMM_PREC_SPLIT_BF16X3)
        return fail(SPAMM_E_INVAL, "unknown precision %d", opts->precision);
    const bool split = opts->precision != SPAMM_PREC_FP32;
    const bool want16 = opts->precision == SPAMM_PREC_SPLIT_FP16;
    if (split && (rc = check_tol(opts->low_tol, "low_tol")))
        return rc;
    if (split && (rc = check_tol(opts->low_rel, "low_rel")))
        return rc;
    if (split && opts->low_tol > 0.0 && opts->low_rel > 0.0)
        return fail(SPAMM_E_INVAL, "low_tol = %g and low_rel = %g: give one threshold",
                    opts->low_tol, opts->low_rel);
    if (A->n != B->n || A->leaf != B->leaf)
        return fail(SPAMM_E_MISMATCH, "A is %lld/%d, B is %lld/%d (n/leaf)", (long long)A->n,
                    A->leaf, (long long)B->n, B->leaf);
    if (split && (A->tiles16 == nullptr || B->tilesT16 == nullptr || A->fp16 != want16 ||
                  B->fp16 != want16))
        return fail(SPAMM_E_INVAL, "split precision %s needs trees built with %s",
                    want16 ? "SPLIT_FP16"
                    : opts->precision == SPAMM_PREC_SPLIT_BF16X3 ? "SPLIT_BF16X3"
                                                                 : "SPLIT_BF16",
                    want16 ? "SPAMM_TREE_FP16" : "SPAMM_TREE_BF16");
    if (opts->precision == SPAMM_PREC_SPLIT_BF16X3 &&
        (A->root >= kX3MaxRoot2 || B->root >= kX3MaxRoot2))
        return fail(SPAMM_E_RANGE,
                    "SPLIT_BF16X3: ||A||_F^2 = %g, ||B||_F^2 = %g; an entry could overflow its "
                    "bfloat16 part (squared norms must stay below %g)",
                    A->root, B->root, kX3MaxRoot2);
    if (opts->sub_cull != 0 && opts->sub_cull != 1)
        return fail(SPAMM_E_INVAL, "sub_cull = %d not in {0, 1}", opts->sub_cull);
    const bool sub = opts->sub_cull == 1;
    if (sub && (split || A->leaf != 64 || !A->sub || !B->sub))
        return fail(SPAMM_E_INVAL,
                    "sub-leaf culling needs FP32 precision and leaf-64 trees built with "
                    "SPAMM_TREE_SUBNORMS");
    if (A->device != dev || B->device != dev)
        return fail(SPAMM_E_INVAL, "trees live on device %d/%d, current device is %d", A->device,
                    B->device, dev);
    p->device = dev;
    p->stream = s;
    p->A = A;
    p->B = B;
    p->depth = A->depth;
    p->leaf = A->leaf;
    p->n = A->n;
    p->tau = opts->tau;
    p->T2 = opts->tau * opts->tau;
    p->precision = opts->precision;
    p->low_tol = split ? opts->low_tol : 0.0;
    p->L2 = p->low_tol * p->low_tol;
    p->low_rel = split ? opts->low_rel : 0.0;
    p->theta2 = p->low_rel * p->low_rel;
    p->sub = sub ? 1 : 0;
    const int d = p->depth;
    p->nblocks = d == 0 ? 1 : (int64_t(1) << (2 * (d - 1)));
    const PlanSizes z = plan_sizes(d);
    for (int t = 0; t <= d; ++t)
        p->rp_off[t] = z.rp_off[t];
    PlanBuf bufs[12];
    const int nb = plan_bufs(p, z, split, sub, bufs);
    size_t total = 0;
    for (int i = 0; i < nb; ++i)
        total += align256(bufs[i].bytes);
    *bytes = total;
    return SPAMM_OK;
}

// Points the buffers of a set-up plan into `base` (its block).
static void plan_carve(spamm_plan *p, char *base)
{
    PlanBuf bufs[12];
    const int nb = plan_bufs(p, plan_sizes(p->depth), p->precision != SPAMM_PREC_FP32,
                             p->sub != 0, bufs);
    size_t off = 0;
    for (int i = 0; i < nb; ++i) {
        *bufs[i].dst = base + off;
        off += align256(bufs[i].bytes);
    }
}

// ... and enqueues the cull on the plan's stream.
static hipError_t plan_carve_and_cull(spamm_plan *p, char *base)
{
    plan_carve(p, base);
    return launch_cull(p, p->stream);
}

int plan_prepare(const spamm_tree *A, const spamm_tree *B, const spamm_opts *opts,
                 hipStream_t s, void *arena, spamm_plan **out)
{
    if (out == nullptr || arena == nullptr)
        return fail(SPAMM_E_INVAL, "out or arena is NULL");
    *out = nullptr;
    int dev, rc;
    if ((rc = prepare_device(&dev)))
        return rc;
    spamm_plan *p = new (std::nothrow) spamm_plan();
    if (!p)
        return fail(SPAMM_E_NOMEM, "host allocation failed");
    size_t total = 0;
    if ((rc = plan_setup(p, A, B, opts, dev, s, &total))) {
        delete p;
        return rc;
    }
    plan_carve(p, (char *)arena);
    *out = p;
    return SPAMM_OK;
}

int symbolic_async(const spamm_tree *A, const spamm_tree *B, const spamm_opts *opts,
                   hipStream_t s, void *arena, spamm_plan **out)
{
    if (out == nullptr)
        return fail(SPAMM_E_INVAL, "out is NULL");
    *out = nullptr;
    if (A == nullptr || B == nullptr || opts == nullptr)
        return fail(SPAMM_E_INVAL, "tree or options NULL");
    int dev, rc;
    if ((rc = prepare_device(&dev)))
        return rc;
    spamm_plan *p = new (std::nothrow) spamm_plan();
    if (!p)
        return fail(SPAMM_E_NOMEM, "host allocation failed");
    size_t total = 0;
    if ((rc = plan_setup(p, A, B, opts, dev, s, &total))) {
        delete p;
        return rc;
    }
    // every buffer at its offset of one block: the caller's arena, else an
    // allocation of the plan's own
    char *base = (char *)arena;
    if (base == nullptr) {
        hipError_t e = dev_alloc_async(dev, (void **)&base, total, s);
        if (e != hipSuccess) {
            rc = hip_fail(e, "plan allocation");
            spamm_plan_free(p);
            return rc;
        }
        p->block = base;
    }
    hipError_t e = plan_carve_and_cull(p, base);
    if (e != hipSuccess) {
        rc = hip_fail(e, "cull launch");
        spamm_plan_free(p);
        return rc;
    }
    *out = p;
    return SPAMM_OK;
}

// ---- the product with no allocation ----------------------------------------
// The task arena of spamm_multiply_noalloc: one fixed block per device, held
// by the loaded code object until the process ends.  In host code `scratch`
// only names the symbol; its device address on each device comes from
// hipGetSymbolAddress (taken once per device, with that device current).
static __device__ __align__(256) unsigned char scratch[SPAMM_NOALLOC_SCRATCH_BYTES];

namespace {
void *g_scratch[64] = {};
std::mutex g_scratch_mu;
}  // namespace

static int scratch_address(int dev, void **out)
{
    if (dev < 0 || dev >= 64)
        return fail(SPAMM_E_HIP, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[dev] == nullptr) {
        void *ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (ptr == nullptr)
            return fail(SPAMM_E_HIP, "no device address for the scratch block on device %d", dev);
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return SPAMM_OK;
}

}  // namespace spamm

extern "C" {

const char *spamm_strerror(int code)
{
    switch (code) {
    case SPAMM_OK: return "success";
    case SPAMM_E_INVAL: return "invalid argument";
    case SPAMM_E_NONFINITE: return "non-finite value in input matrix";
    case SPAMM_E_NOMEM: return "out of device memory";
    case SPAMM_E_HIP: return "HIP runtime error";
    case SPAMM_E_RANGE: return "size out of range";
    case SPAMM_E_MISMATCH: return "operand shapes differ";
    case SPAMM_E_BUSY: return "server queue full";
    case SPAMM_PENDING: return "request pending";
    default: return "unknown status";
    }
}

const char *spamm_last_error(void) { return g_err; }

int spamm_build_tree(const float *A, int64_t n, int32_t leaf, void *stream, spamm_tree **out)
{
    return spamm_build_tree_ex(A, n, leaf, 0u, stream, out);
}

int spamm_build_tree_ex(const float *A, int64_t n, int32_t leaf, uint32_t flags, void *stream,
                        spamm_tree **out)
{
    if (out == nullptr)
        return fail(SPAMM_E_INVAL, "out is NULL");
    *out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    double root = 0.0;
    spamm_tree *t = nullptr;
    int rc = tree_build_async(A, n, leaf, flags, s, &root, &t);
    if (rc)
        return rc;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        rc = hip_fail(e, "spamm_build_tree");
        spamm_tree_free(t);
        return rc;
    }
    if (!isfinite(root)) {
        spamm_tree_free(t);
        return fail(SPAMM_E_NONFINITE, "input matrix holds NaN or Inf (||A||_F^2 = %g)", root);
    }
    t->root = root;
    t->root_dense = root;
    *out = t;
    return SPAMM_OK;
}

int spamm_build_tree_output(const float *C, const spamm_plan *plan, uint32_t flags,
                            void *stream, spamm_tree **out)
{
    if (out == nullptr)
        return fail(SPAMM_E_INVAL, "out is NULL");
    *out = nullptr;
    int dev;
    int rc = check_output_args(C, plan, flags, &dev);
    if (rc)
        return rc;
    const spamm_plan *p = plan;
    hipStream_t s = (hipStream_t)stream;
    const int32_t d = p->depth;
    const uint32_t N2 = 1u << (2 * d);
    spamm_tree *t = output_tree_shell(p, dev, s);
    if (!t)
        return fail(SPAMM_E_NOMEM, "host allocation failed");
    // pass 1: keep flags and slots (storage then follows the reached leaves)
    const size_t np_bytes = align256(sizeof(uint32_t) * scan_partials_len(N2));
    void *scratch = nullptr;
    uint32_t reached = 0;
    hipError_t e = dev_alloc_async(dev, (void **)&t->keep, sizeof(uint32_t) * N2, s);
    if (e == hipSuccess)
        e = dev_alloc_async(dev, (void **)&t->slot, sizeof(uint32_t) * ((size_t)N2 + 1), s);
    if (e == hipSuccess)
        e = dev_alloc_async(dev, &scratch, np_bytes, s);
    if (e == hipSuccess) {
        const bool split = p->precision != SPAMM_PREC_FP32;
        e = launch_output_map(p->browptr, p->bent, split ? p->browptr_lo : nullptr,
                              split ? p->bent_lo : nullptr, (uint32_t)p->nblocks, d, t->keep,
                              t->slot, (uint32_t *)scratch, s);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(&reached, t->slot + N2, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (scratch != nullptr)
        hipFreeAsync(scratch, s);
    // pass 2: the reached leaves (one buffer each, as a sparsified tree)
    const bool c16 = flags != 0, fp16 = (flags & SPAMM_TREE_FP16) != 0;
    const size_t leaf_bytes = sizeof(float) * (size_t)p->leaf * (size_t)p->leaf;
    const size_t cnt = std::max<size_t>(reached, 1);   // keep the pointers valid when empty
    t->stored = reached;
    t->fp16 = fp16;
    if (e == hipSuccess)
        e = dev_alloc_async(dev, (void **)&t->tiles, leaf_bytes * cnt, s);
    if (e == hipSuccess)
        e = dev_alloc_async(dev, (void **)&t->tilesT, leaf_bytes * cnt, s);
    if (e == hipSuccess && c16)
        e = dev_alloc_async(dev, (void **)&t->tiles16, leaf_bytes / 2 * cnt, s);
    if (e == hipSuccess && c16)
        e = dev_alloc_async(dev, (void **)&t->tilesT16, leaf_bytes / 2 * cnt, s);
    if (e == hipSuccess && fp16)
        e = dev_alloc_async(dev, (void **)&t->scale16, sizeof(int32_t) * N2, s);
    if (e == hipSuccess)
        e = dev_alloc_async(dev, (void **)&t->norms,
                            sizeof(double) * (size_t)tier_offset(d + 1), s);
    if (e == hipSuccess)
        e = launch_output_pack(C, p->n, p->leaf, d, t->tiles, t->tilesT, t->tiles16, t->tilesT16,
                               t->scale16, t->norms, t->keep, t->slot, s);
    double root = 0.0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&root, t->norms, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        rc = hip_fail(e, "spamm_build_tree_output");
        spamm_tree_free(t);
        return rc;
    }
    if (!isfinite(root)) {
        spamm_tree_free(t);
        return fail(SPAMM_E_NONFINITE, "C holds NaN or Inf on a reached leaf (||C||_F^2 = %g)",
                    root);
    }
    t->root = root;
    t->root_dense = root;
    *out = t;
    return SPAMM_OK;
}

int spamm_build_tree_sparse(const float *A, int64_t n, int32_t leaf, uint32_t flags, double tau,
                            double norm2_other, void *stream, spamm_tree **out)
{
    if (out == nullptr)
        return fail(SPAMM_E_INVAL, "out is NULL");
    *out = nullptr;
    if (A == nullptr)
        return fail(SPAMM_E_INVAL, "A is NULL");
    if (n < 1)
        return fail(SPAMM_E_INVAL, "n = %lld < 1", (long long)n);
    if (leaf != 16 && leaf != 32 && leaf != 64)
        return fail(SPAMM_E_INVAL, "leaf = %d not in {16, 32, 64}", leaf);
    if ((flags & ~SPAMM_TREE_BF16) != 0)
        return fail(SPAMM_E_INVAL, "flags 0x%x: a sparsified tree takes SPAMM_TREE_BF16 only",
                    flags);
    const bool bf16 = (flags & SPAMM_TREE_BF16) != 0;
    if (bf16 && leaf == 16)
        return fail(SPAMM_E_INVAL, "BF16 leaf copies need leaf 32 or 64");
    int rc;
    if ((rc = check_tol(tau, "tau")))
        return rc;
    if (!(norm2_other >= 0.0) || isinf(norm2_other))
        return fail(SPAMM_E_INVAL, "norm2_other = %g must be finite and >= 0", norm2_other);
    int32_t d;
    int64_t np;
    if ((rc = tree_depth(n, leaf, &d, &np)))
        return rc;
    int dev;
    if ((rc = prepare_device(&dev)))
        return rc;
    hipStream_t s = (hipStream_t)stream;
    const uint32_t N2 = 1u << (2 * d);
    spamm_tree *t = new (std::nothrow) spamm_tree();
    if (!t)
        return fail(SPAMM_E_NOMEM, "host allocation failed");
    t->device = dev;
    t->stream = s;
    t->n = n;
    t->np = np;
    t->leaf = leaf;
    t->depth = d;
    // scratch: scan partials, then the dense root (8-byte aligned)
    const size_t np_bytes = align256(sizeof(uint32_t) * scan_partials_len(N2));
    void *scratch = nullptr;
    hipError_t e = dev_alloc_async(dev, (void **)&t->norms, sizeof(double) * (size_t)tier_offset(d + 1), s);
    if (e == hipSuccess)
        e = dev_alloc_async(dev, (void **)&t->keep, sizeof(uint32_t) * N2, s);
    if (e == hipSuccess)
        e = dev_alloc_async(dev, (void **)&t->slot, sizeof(uint32_t) * ((size_t)N2 + 1), s);
    if (e == hipSuccess)
        e = dev_alloc_async(dev, &scratch, np_bytes + sizeof(double), s);
    double *root_dense_dev = (double *)((char *)scratch + np_bytes);
    if (e == hipSuccess)
        e = launch_sparse_norms(A, n, leaf, d, t->norms, tau, norm2_other, t->keep, t->slot,
                                (uint32_t *)scratch, root_dense_dev, s);
    uint32_t kept = 0;
    double roots[2] = {0.0, 0.0};
    if (e == hipSuccess)
        e = hipMemcpyAsync(&kept, t->slot + N2, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&roots[0], t->norms, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&roots[1], root_dense_dev, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (scratch != nullptr)
        hipFreeAsync(scratch, s);
    if (e != hipSuccess) {
        rc = hip_fail(e, "spamm_build_tree_sparse");
        spamm_tree_free(t);
        return rc;
    }
    if (!isfinite(roots[1])) {
        spamm_tree_free(t);
        return fail(SPAMM_E_NONFINITE, "input matrix holds NaN or Inf (||A||_F^2 = %g)", roots[1]);
    }
    const size_t leaf_bytes = sizeof(float) * (size_t)leaf * (size_t)leaf;
    const size_t cnt = std::max<size_t>(kept, 1);     // keep the pointers valid when empty
    e = dev_alloc_async(dev, (void **)&t->tiles, cnt * leaf_bytes, s);
    if (e == hipSuccess)
        e = dev_alloc_async(dev, (void **)&t->tilesT, cnt * leaf_bytes, s);
    if (e == hipSuccess && bf16)
        e = dev_alloc_async(dev, (void **)&t->tiles16, cnt * leaf_bytes / 2, s);
    if (e == hipSuccess && bf16)
        e = dev_alloc_async(dev, (void **)&t->tilesT16, cnt * leaf_bytes / 2, s);
    if (e == hipSuccess && kept > 0)
        e = launch_sparse_pack(A, n, leaf, d, t->tiles, t->tilesT, t->tiles16, t->tilesT16, t->keep,
                               t->slot, s);
    if (e != hipSuccess) {
        rc = hip_fail(e, "spamm_build_tree_sparse (pack)");
        spamm_tree_free(t);
        return rc;
    }
    t->stored = kept;
    t->root = roots[0];
    t->root_dense = roots[1];
    *out = t;
    return SPAMM_OK;
}

int spamm_tree_storage(const spamm_tree *t, int64_t *stored, int64_t *total, size_t *device_bytes)
{
    if (t == nullptr)
        return fail(SPAMM_E_INVAL, "tree is NULL");
    const int64_t N2 = int64_t(1) << (2 * t->depth);
    const size_t leaf_bytes = sizeof(float) * (size_t)t->leaf * (size_t)t->leaf;
    const size_t copies = (t->tiles16 != nullptr) ? 3 : 2;   // two FP32 + two half-size 16-bit
    size_t b = copies * leaf_bytes * (size_t)std::max<int64_t>(t->stored, t->slot ? 1 : 0) +
               sizeof(double) * (size_t)tier_offset(t->depth + (t->sub ? 2 : 1));
    if (t->slot != nullptr)
        b += sizeof(uint32_t) * (2 * (size_t)N2 + 1);
    if (t->scale16 != nullptr)
        b += sizeof(int32_t) * (size_t)N2;
    if (stored) *stored = t->stored;
    if (total) *total = N2;
    if (device_bytes) *device_bytes = b;
    return SPAMM_OK;
}

int spamm_tree_free(spamm_tree *t)
{
    if (t == nullptr)
        return SPAMM_OK;
    int dev0 = -1;
    hipGetDevice(&dev0);
    if (dev0 != t->device)
        hipSetDevice(t->device);
    hipError_t e = hipSuccess;
    if (t->block != nullptr) {
        e = hipFreeAsync(t->block, t->stream);
    } else if (!t->borrowed) {
        // sparsified and output trees: one allocation per buffer
        for (void *ptr : {(void *)t->tiles, (void *)t->tilesT, (void *)t->tiles16,
                          (void *)t->tilesT16, (void *)t->norms, (void *)t->slot, (void *)t->keep,
                          (void *)t->scale16}) {
            if (ptr == nullptr)
                continue;
            hipError_t f = hipFreeAsync(ptr, t->stream);
            if (e == hipSuccess)
                e = f;
        }
    }
    if (dev0 >= 0 && dev0 != t->device)
        hipSetDevice(dev0);
    delete t;
    return e == hipSuccess ? SPAMM_OK : hip_fail(e, "spamm_tree_free");
}

int spamm_tree_info(const spamm_tree *t, int64_t *n, int32_t *leaf, int32_t *depth, double *norm2)
{
    if (t == nullptr)
        return fail(SPAMM_E_INVAL, "tree is NULL");
    if (n) *n = t->n;
    if (leaf) *leaf = t->leaf;
    if (depth) *depth = t->depth;
    if (norm2) *norm2 = t->root;
    return SPAMM_OK;
}

int spamm_tree_norms(const spamm_tree *t, int32_t tier, double *host, size_t len)
{
    if (t == nullptr || host == nullptr)
        return fail(SPAMM_E_INVAL, "NULL argument");
    const int top = t->depth + (t->sub ? 1 : 0);
    if (tier < 0 || tier > top)
        return fail(SPAMM_E_INVAL, "tier %d outside 0..%d", tier, top);
    const int64_t Nt = int64_t(1) << tier;
    if (len < (size_t)(Nt * Nt))
        return fail(SPAMM_E_RANGE, "host buffer holds %zu < %lld values", len, (long long)(Nt * Nt));
    std::vector<double> lin((size_t)(Nt * Nt));
    HIP_TRY(hipMemcpyAsync(lin.data(), t->norms + tier_offset(tier), sizeof(double) * lin.size(),
                           hipMemcpyDeviceToHost, t->stream),
            "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(t->stream), "hipStreamSynchronize");
    for (int64_t l = 0; l < Nt * Nt; ++l)
        host[(int64_t)lin_row((uint32_t)l) * Nt + lin_col((uint32_t)l)] = lin[(size_t)l];
    return SPAMM_OK;
}

int spamm_tree_matrix(const spamm_tree *t, int32_t copy, float *host, size_t len)
{
    if (t == nullptr || host == nullptr)
        return fail(SPAMM_E_INVAL, "NULL argument");
    if (copy != 0 && copy != 1)
        return fail(SPAMM_E_INVAL, "copy = %d not in {0, 1}", copy);
    const int64_t np = t->np, b = t->leaf, N = int64_t(1) << t->depth;
    if (len < (size_t)(np * np))
        return fail(SPAMM_E_RANGE, "host buffer holds %zu < %lld values", len, (long long)(np * np));
    // a sparsified tree holds only its kept leaves (leaf l at slot[l])
    const bool sparse = t->slot != nullptr;
    std::vector<float> tiles((size_t)(t->stored * b * b));
    std::vector<uint32_t> slot(sparse ? (size_t)(N * N) : 0), keep(sparse ? (size_t)(N * N) : 0);
    if (!tiles.empty())
        HIP_TRY(hipMemcpyAsync(tiles.data(), copy == 0 ? t->tiles : t->tilesT,
                               sizeof(float) * tiles.size(), hipMemcpyDeviceToHost, t->stream),
                "hipMemcpyAsync");
    if (sparse) {
        HIP_TRY(hipMemcpyAsync(slot.data(), t->slot, sizeof(uint32_t) * slot.size(),
                               hipMemcpyDeviceToHost, t->stream),
                "hipMemcpyAsync");
        HIP_TRY(hipMemcpyAsync(keep.data(), t->keep, sizeof(uint32_t) * keep.size(),
                               hipMemcpyDeviceToHost, t->stream),
                "hipMemcpyAsync");
    }
    HIP_TRY(hipStreamSynchronize(t->stream), "hipStreamSynchronize");
    const std::vector<float> zero((size_t)(b * b), 0.0f);
    for (int64_t l = 0; l < N * N; ++l) {
        const int64_t I = lin_row((uint32_t)l), J = lin_col((uint32_t)l);
        const float *src = !sparse ? tiles.data() + l * b * b
                           : keep[(size_t)l] ? tiles.data() + (int64_t)slot[(size_t)l] * b * b
                                             : zero.data();
        for (int r = 0; r < (int)b; ++r)
            for (int c = 0; c < (int)b; ++c) {
                const float v = src[leaf_index((int)b, r, c)];
                if (copy == 0)
                    host[(I * b + r) * np + J * b + c] = v;
                else
                    host[(I * b + c) * np + J * b + r] = v;
            }
    }
    return SPAMM_OK;
}

int spamm_tree_matrix16(const spamm_tree *t, int32_t copy, uint16_t *host, size_t len,
                        int32_t *scale, size_t scale_len)
{
    if (t == nullptr || host == nullptr)
        return fail(SPAMM_E_INVAL, "NULL argument");
    if (copy != 0 && copy != 1)
        return fail(SPAMM_E_INVAL, "copy = %d not in {0, 1}", copy);
    if (t->tiles16 == nullptr)
        return fail(SPAMM_E_INVAL, "the tree holds no 16-bit leaf copies");
    const int64_t np = t->np, b = t->leaf, N = int64_t(1) << t->depth;
    if (len < (size_t)(np * np))
        return fail(SPAMM_E_RANGE, "host buffer holds %zu < %lld values", len, (long long)(np * np));
    if (scale != nullptr && t->scale16 != nullptr && scale_len < (size_t)(N * N))
        return fail(SPAMM_E_RANGE, "scale buffer holds %zu < %lld values", scale_len,
                    (long long)(N * N));
    const bool sparse = t->slot != nullptr;
    std::vector<uint16_t> tiles((size_t)(t->stored * b * b));
    std::vector<int32_t> sc(t->scale16 != nullptr ? (size_t)(N * N) : 0);
    std::vector<uint32_t> slot(sparse ? (size_t)(N * N) : 0), keep(sparse ? (size_t)(N * N) : 0);
    if (!tiles.empty())
        HIP_TRY(hipMemcpyAsync(tiles.data(), copy == 0 ? t->tiles16 : t->tilesT16,
                               sizeof(uint16_t) * tiles.size(), hipMemcpyDeviceToHost, t->stream),
                "hipMemcpyAsync");
    if (!sc.empty())
        HIP_TRY(hipMemcpyAsync(sc.data(), t->scale16, sizeof(int32_t) * sc.size(),
                               hipMemcpyDeviceToHost, t->stream),
                "hipMemcpyAsync");
    if (sparse) {
        HIP_TRY(hipMemcpyAsync(slot.data(), t->slot, sizeof(uint32_t) * slot.size(),
                               hipMemcpyDeviceToHost, t->stream),
                "hipMemcpyAsync");
        HIP_TRY(hipMemcpyAsync(keep.data(), t->keep, sizeof(uint32_t) * keep.size(),
                               hipMemcpyDeviceToHost, t->stream),
                "hipMemcpyAsync");
    }
    HIP_TRY(hipStreamSynchronize(t->stream), "hipStreamSynchronize");
    const std::vector<uint16_t> zero((size_t)(b * b), 0);
    for (int64_t l = 0; l < N * N; ++l) {
        const int64_t I = lin_row((uint32_t)l), J = lin_col((uint32_t)l);
        const uint16_t *src = !sparse ? tiles.data() + l * b * b
                              : keep[(size_t)l] ? tiles.data() + (int64_t)slot[(size_t)l] * b * b
                                                : zero.data();
        for (int r = 0; r < (int)b; ++r)
            for (int c = 0; c < (int)b; ++c) {
                const int idx = b == 32 ? Leaf16Layout<32>::index(r, c) : Leaf16Layout<64>::index(r, c);
                if (copy == 0)
                    host[(I * b + r) * np + J * b + c] = src[idx];
                else
                    host[(I * b + c) * np + J * b + r] = src[idx];
            }
        if (scale != nullptr && !sc.empty())
            scale[I * N + J] = sc[(size_t)l];
    }
    return SPAMM_OK;
}

int spamm_plan_free(spamm_plan *p)
{
    if (p == nullptr)
        return SPAMM_OK;
    int dev0 = -1;
    hipGetDevice(&dev0);
    if (dev0 != p->device)
        hipSetDevice(p->device);
    hipError_t e = p->block != nullptr ? hipFreeAsync(p->block, p->stream) : hipSuccess;
    if (dev0 >= 0 && dev0 != p->device)
        hipSetDevice(dev0);
    delete p;
    return e == hipSuccess ? SPAMM_OK : hip_fail(e, "spamm_plan_free");
}

int spamm_symbolic(const spamm_tree *A, const spamm_tree *B, double tau, void *stream,
                   spamm_plan **out)
{
    spamm_opts o{};
    o.tau = tau;
    o.precision = SPAMM_PREC_FP32;
    o.low_tol = 0.0;
    return spamm_symbolic_ex(A, B, &o, stream, out);
}

int spamm_symbolic_ex(const spamm_tree *A, const spamm_tree *B, const spamm_opts *opts,
                      void *stream, spamm_plan **out)
{
    return symbolic_async(A, B, opts, (hipStream_t)stream, nullptr, out);
}

int spamm_numeric(const spamm_plan *p, float *C, void *stream)
{
    if (p == nullptr || C == nullptr)
        return fail(SPAMM_E_INVAL, "NULL argument");
    HIP_TRY(launch_gemm(p, C, (hipStream_t)stream), "leaf GEMM launch");
    return SPAMM_OK;
}

int spamm_plan_stats(const spamm_plan *p, spamm_stats *out)
{
    if (p == nullptr || out == nullptr)
        return fail(SPAMM_E_INVAL, "NULL argument");
    memset(out, 0, sizeof *out);
    const int d = p->depth;
    out->depth = d;
    out->leaf = p->leaf;
    out->symbolic_ms = -1.0;
    out->numeric_ms = -1.0;
    std::vector<uint32_t> tot((size_t)d + 1, 0);
    for (int t = 0; t < d; ++t)
        HIP_TRY(hipMemcpyAsync(&tot[(size_t)t], p->rowptr + p->rp_off[t] + (int64_t(1) << (2 * t)),
                               sizeof(uint32_t), hipMemcpyDeviceToHost, p->stream),
                "hipMemcpyAsync");
    const bool split = p->precision != SPAMM_PREC_FP32;
    uint64_t K[3] = {0, 0, 0};
    uint32_t entries[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(K, p->leafK, (p->sub ? 3 : split ? 2 : 1) * sizeof(uint64_t),
                           hipMemcpyDeviceToHost, p->stream),
            "hipMemcpyAsync");
    // the FP32 cull writes only the HIGH count; the LOW slot is not initialized
    HIP_TRY(hipMemcpyAsync(&entries[0], p->browptr + p->nblocks, sizeof(uint32_t),
                           hipMemcpyDeviceToHost, p->stream),
            "hipMemcpyAsync");
    if (split)
        HIP_TRY(hipMemcpyAsync(&entries[1], p->browptr_lo + p->nblocks, sizeof(uint32_t),
                               hipMemcpyDeviceToHost, p->stream),
                "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
    if (!split)
        K[1] = 0;
    const int64_t all = (int64_t)(K[0] + K[1]);
    for (int t = 0; t < d; ++t)
        out->kept[t] = tot[(size_t)t];
    out->kept[d] = all;
    out->tasks = all;
    out->tasks_low = (int64_t)K[1];
    out->block_entries = entries[0];
    out->block_entries_low = entries[1];
    out->flops = 2.0 * (double)p->leaf * p->leaf * p->leaf * (double)all;
    if (p->sub) {
        const double h = p->leaf / 2;
        out->subtasks = (int64_t)K[2];
        out->flops = 2.0 * h * h * h * (double)K[2];
    }
    return SPAMM_OK;
}

// Copies one class's block schedule (row pointers + entries) to the host.
static int fetch_schedule(const spamm_plan *p, const uint32_t *drp, const uint32_t *dent,
                          std::vector<uint32_t> &rp, std::vector<uint32_t> &ent)
{
    const size_t nb = (size_t)p->nblocks;
    rp.assign(nb + 1, 0);
    HIP_TRY(hipMemcpyAsync(rp.data(), drp, sizeof(uint32_t) * (nb + 1), hipMemcpyDeviceToHost,
                           p->stream),
            "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
    ent.assign(rp[nb], 0);
    if (!ent.empty()) {
        HIP_TRY(hipMemcpyAsync(ent.data(), dent, sizeof(uint32_t) * ent.size(),
                               hipMemcpyDeviceToHost, p->stream),
                "hipMemcpyAsync");
        HIP_TRY(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
    }
    return SPAMM_OK;
}

int spamm_plan_tasks(const spamm_plan *p, uint64_t *host, size_t cap, size_t *count)
{
    if (p == nullptr || count == nullptr)
        return fail(SPAMM_E_INVAL, "NULL argument");
    const bool split = p->precision != SPAMM_PREC_FP32;
    uint64_t K[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(K, p->leafK, (split ? 2 : 1) * sizeof(uint64_t), hipMemcpyDeviceToHost,
                           p->stream),
            "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
    const uint64_t total = K[0] + K[1];
    *count = (size_t)total;
    if (host == nullptr || cap < total)
        return host == nullptr && cap == 0 ? SPAMM_OK
                                           : fail(SPAMM_E_RANGE, "cap %zu < K = %llu", cap,
                                                  (unsigned long long)total);
    std::vector<uint32_t> rp[2], ent[2];
    int rc = fetch_schedule(p, p->browptr, p->bent, rp[0], ent[0]);
    if (rc == SPAMM_OK && split)
        rc = fetch_schedule(p, p->browptr_lo, p->bent_lo, rp[1], ent[1]);
    if (rc != SPAMM_OK)
        return rc;
    // Expand block entries to leaf keys in (output leaf, k) order: leaf
    // 4 P + q of block P takes the entries whose mask has bit q; within a
    // leaf the two classes are merged by k (each list is ascending).
    const size_t nb = (size_t)p->nblocks;
    size_t o = 0;
    for (size_t P = 0; P < nb; ++P)
        for (uint32_t q = 0; q < 4; ++q) {
            const uint64_t lc = p->depth == 0 ? 0 : 4 * (uint64_t)P + q;
            uint32_t e[2] = {rp[0][P], split ? rp[1][P] : 0u};
            const uint32_t end[2] = {rp[0][P + 1], split ? rp[1][P + 1] : 0u};
            for (;;) {
                for (int c = 0; c < 2; ++c)
                    while (e[c] < end[c] && !((ent[c][e[c]] >> (16 + q)) & 1u))
                        ++e[c];
                const bool has0 = e[0] < end[0], has1 = e[1] < end[1];
                if (!has0 && !has1)
                    break;
                const int c = !has1 ? 0 : !has0 ? 1
                                     : ((ent[0][e[0]] & 0xFFFFu) < (ent[1][e[1]] & 0xFFFFu) ? 0 : 1);
                if (o >= cap)
                    return fail(SPAMM_E_RANGE, "inconsistent task count");
                host[o++] = (lc << 32) | (ent[c][e[c]] & 0xFFFFu) | ((uint64_t)c << 63);
                ++e[c];
            }
        }
    if (o != total)
        return fail(SPAMM_E_HIP, "task count mismatch: %zu expanded vs %llu counted", o,
                    (unsigned long long)total);
    return SPAMM_OK;
}

int spamm_plan_subtasks(const spamm_plan *p, uint64_t *host, size_t cap, size_t *count)
{
    if (p == nullptr || count == nullptr)
        return fail(SPAMM_E_INVAL, "NULL argument");
    if (!p->sub)
        return fail(SPAMM_E_INVAL, "the plan does not cull sub-leaves");
    uint64_t K[3] = {0, 0, 0};
    HIP_TRY(hipMemcpyAsync(K, p->leafK, 3 * sizeof(uint64_t), hipMemcpyDeviceToHost, p->stream),
            "hipMemcpyAsync");
    HIP_TRY(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
    *count = (size_t)K[2];
    if (host == nullptr || cap < K[2])
        return host == nullptr && cap == 0 ? SPAMM_OK
                                           : fail(SPAMM_E_RANGE, "cap %zu < %llu sub-products", cap,
                                                  (unsigned long long)K[2]);
    std::vector<uint32_t> rp, ent;
    int rc = fetch_schedule(p, p->browptr, p->bent, rp, ent);
    if (rc != SPAMM_OK)
        return rc;
    std::vector<uint8_t> mask(4 * ent.size());
    if (!mask.empty()) {
        HIP_TRY(hipMemcpyAsync(mask.data(), p->submask, mask.size(), hipMemcpyDeviceToHost,
                               p->stream),
                "hipMemcpyAsync");
        HIP_TRY(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
    }
    // leaf (I, J) = child q of block P; its sub-leaf (a, b) has linear index
    // 4 lin(I, J) + 2a + b on the 32 x 32 grid and takes sub-product (k, c) as
    // k32 = 2k + c: leaves, then sub-leaves, then k, then c ascending is the
    // sorted order.
    const size_t nb = (size_t)p->nblocks;
    size_t o = 0;
    for (size_t P = 0; P < nb; ++P)
        for (uint32_t q = 0; q < 4; ++q) {
            const uint64_t lc = p->depth == 0 ? 0 : 4 * (uint64_t)P + q;
            for (uint32_t ab = 0; ab < 4; ++ab)
                for (uint32_t e = rp[P]; e < rp[P + 1]; ++e) {
                    const uint32_t m = mask[4 * (size_t)e + q];
                    const uint64_t k = ent[e] & 0xFFFFu;
                    for (uint32_t c = 0; c < 2; ++c) {
                        if (!((m >> (2 * ab + c)) & 1u))
                            continue;
                        if (o >= cap)
                            return fail(SPAMM_E_RANGE, "inconsistent sub-product count");
                        host[o++] = ((4 * lc + ab) << 32) | (2 * k + c);
                    }
                }
        }
    if (o != K[2])
        return fail(SPAMM_E_HIP, "sub-product count mismatch: %zu expanded vs %llu counted", o,
                    (unsigned long long)K[2]);
    return SPAMM_OK;
}

int spamm_multiply_opts(const spamm_tree *A, const spamm_tree *B, const spamm_opts *opts,
                        float *C, void *stream, spamm_stats *stats)
{
    if (C == nullptr)
        return fail(SPAMM_E_INVAL, "C is NULL");
    hipStream_t s = (hipStream_t)stream;
    // the timing events are destroyed on every exit path
    struct Events {
        hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
        ~Events()
        {
            for (hipEvent_t x : ev)
                if (x)
                    hipEventDestroy(x);
        }
    } events;
    hipEvent_t *ev = events.ev;
    if (stats) {
        for (int i = 0; i < 3; ++i)
            HIP_TRY(hipEventCreate(&ev[i]), "hipEventCreate");
        HIP_TRY(hipEventRecord(ev[0], s), "hipEventRecord");
    }
    spamm_plan *p = nullptr;
    int rc = spamm_symbolic_ex(A, B, opts, stream, &p);
    if (rc == SPAMM_OK && stats) {
        hipError_t e = hipEventRecord(ev[1], s);
        if (e != hipSuccess)
            rc = hip_fail(e, "hipEventRecord");
    }
    if (rc == SPAMM_OK)
        rc = spamm_numeric(p, C, stream);
    if (rc == SPAMM_OK && stats) {
        hipError_t e = hipEventRecord(ev[2], s);
        if (e != hipSuccess)
            rc = hip_fail(e, "hipEventRecord");
        if (rc == SPAMM_OK)
            rc = spamm_plan_stats(p, stats);   // synchronizes
        float ms = 0.f;
        if (rc == SPAMM_OK && hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess)
            stats->symbolic_ms = ms;
        if (rc == SPAMM_OK && hipEventElapsedTime(&ms, ev[1], ev[2]) == hipSuccess)
            stats->numeric_ms = ms;
    }
    int rc2 = spamm_plan_free(p);
    return rc != SPAMM_OK ? rc : rc2;
}

int spamm_multiply_ex(const spamm_tree *A, const spamm_tree *B, double tau, float *C, void *stream,
                      spamm_stats *stats)
{
    spamm_opts o{};
    o.tau = tau;
    o.precision = SPAMM_PREC_FP32;
    o.low_tol = 0.0;
    return spamm_multiply_opts(A, B, &o, C, stream, stats);
}

int spamm_multiply(const spamm_tree *A, const spamm_tree *B, double tau, float *C, void *stream)
{
    return spamm_multiply_ex(A, B, tau, C, stream, nullptr);
}

int spamm_multiply_noalloc(const spamm_tree *A, const spamm_tree *B, const spamm_opts *opts,
                           float *C, void *stream)
{
    if (C == nullptr)
        return fail(SPAMM_E_INVAL, "C is NULL");
    if (A == nullptr || B == nullptr || opts == nullptr)
        return fail(SPAMM_E_INVAL, "tree or options NULL");
    int dev;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    void *base = nullptr;
    int rc = scratch_address(dev, &base);
    if (rc)
        return rc;
    // the plan lives on this stack frame; its buffers in the scratch block
    spamm_plan p{};
    size_t bytes = 0;
    if ((rc = plan_setup(&p, A, B, opts, dev, (hipStream_t)stream, &bytes)))
        return rc;
    if (bytes > (size_t)SPAMM_NOALLOC_SCRATCH_BYTES)
        return fail(SPAMM_E_RANGE,
                    "the task arena of this product needs %zu bytes, the no-allocation "
                    "scratch block holds %zu (depth %d; at most 8 fits)",
                    bytes, (size_t)SPAMM_NOALLOC_SCRATCH_BYTES, p.depth);
    hipError_t e = plan_carve_and_cull(&p, (char *)base);
    if (e == hipSuccess)
        e = launch_gemm(&p, C, (hipStream_t)stream);
    if (e != hipSuccess)
        return hip_fail(e, "spamm_multiply_noalloc");
    return SPAMM_OK;
}

}  // extern "C"
