// Shared device helpers and internal structures of libspamm (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spamm.h"

namespace spamm {

constexpr int kWave = 64;
constexpr int kMaxDepth = 10;        // N = 2^d <= 1024 tiles per dimension

// ---- linear (Morton) index, Eq. linear index: row bits on odd positions ----
__host__ __device__ inline uint32_t spread_bits(uint32_t x)
{
    x &= 0xFFFFu;
    x = (x | (x << 8)) & 0x00FF00FFu;
    x = (x | (x << 4)) & 0x0F0F0F0Fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}

__host__ __device__ inline uint32_t compact_bits(uint32_t x)
{
    x &= 0x55555555u;
    x = (x | (x >> 1)) & 0x33333333u;
    x = (x | (x >> 2)) & 0x0F0F0F0Fu;
    x = (x | (x >> 4)) & 0x00FF00FFu;
    x = (x | (x >> 8)) & 0x0000FFFFu;
    return x;
}

__host__ __device__ inline uint32_t lin_index(uint32_t i, uint32_t j)
{
    return (spread_bits(i) << 1) | spread_bits(j);
}

__host__ __device__ inline uint32_t lin_row(uint32_t l) { return compact_bits(l >> 1); }
__host__ __device__ inline uint32_t lin_col(uint32_t l) { return compact_bits(l); }

// Offset of tier t inside the norm pyramid: tiers 0..d stored back to back,
// tier t holds 4^t values in linear-index order.
__host__ __device__ inline int64_t tier_offset(int t) { return ((int64_t(1) << (2 * t)) - 1) / 3; }

// Storage of one packed n_b x n_b leaf, designed for the leaf GEMM: the
// columns (the k of a left operand) are cut into panels of kKS = min(n_b, 32)
// columns stored one after the other, each panel row-major with rows of kKS
// floats.  Inside a panel row the 16-byte granules (4 floats) are permuted by
// an XOR with a function of the row, so that the 16 rows read at one logical
// column by a ds_read_b128 hit 16 distinct groups of LDS banks.  A panel is
// the unit the GEMM copies to LDS (verbatim, with direct-to-LDS loads).
// Element (r, c) of the leaf lives at index(r, c).
template <int B>
struct LeafLayout {
    static constexpr int kKS = B < 32 ? B : 32;                  // panel width
    static constexpr int kPanels = B / kKS;
    static constexpr int kPanel = B * kKS;                       // floats per panel
    static constexpr int kGran = kKS / 4;                        // granules per panel row
    // 16 consecutive rows cover 16 / kGran bank offsets; the XOR separates
    // the rows that share one
    static constexpr int kShift = kGran == 8 ? 1 : (kGran == 4 ? 2 : 3);
    __host__ __device__ static constexpr int pindex(int r, int cc)   // inside a panel
    {
        return r * kKS + 4 * ((cc >> 2) ^ ((r >> kShift) & (kGran - 1))) + (cc & 3);
    }
    __host__ __device__ static constexpr int index(int r, int c)
    {
        return (c / kKS) * kPanel + pindex(r, c % kKS);
    }
};

__host__ __device__ inline int leaf_index(int B, int r, int c)
{
    switch (B) {
    case 16: return LeafLayout<16>::index(r, c);
    case 32: return LeafLayout<32>::index(r, c);
    default: return LeafLayout<64>::index(r, c);
    }
}

// 16-bit copy of a leaf (split precision, n_b in {32, 64}): the columns (the k
// of a left operand) cut into panels of 32 stored one after the other (one
// panel at n_b = 32, two at 64), each panel row-major with rows of 32 values
// (64 bytes: four 16-byte granules of 8 values); the granules of a row are
// XOR-permuted by (r >> 2) & 3, so that 16 rows read at one logical column by
// a ds_read_b128 hit 16 distinct groups of banks.  The wide LOW kernel stages
// whole leaves (both panels, 8 KB at n_b = 64).
template <int B>
struct Leaf16Layout {
    static constexpr int kKS = 32;                               // panel width
    static constexpr int kPanel = B * kKS;                       // values per panel
    __host__ __device__ static constexpr int index(int r, int c)
    {
        return (c >> 5) * kPanel + r * kKS + 8 * (((c & 31) >> 3) ^ ((r >> 2) & 3)) + (c & 7);
    }
};

// FP32 -> BF16 with round-to-nearest-even on the bit pattern (inputs are
// finite: non-finite matrices are rejected when the tree is built).
__host__ __device__ inline uint16_t to_bf16(float x)
{
    uint32_t u;
    __builtin_memcpy(&u, &x, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// The SpAMM keep decision on stored squared norms (both FP64):
// zero norm -> NULL link, never kept; otherwise kept unless s_A s_B < tau^2.
__device__ inline bool keep_pair(double sa, double sb, double T2)
{
    return (sa > 0.0) & (sb > 0.0) & !(sa * sb < T2);
}

// Split precision: a kept product is LOW (16-bit operands) iff s_A s_B < L2,
// L2 = fl64(low_tol^2); L2 = 0 makes every product HIGH (FP32).
__device__ inline bool low_pair(double sa, double sb, double L2) { return sa * sb < L2; }

// The LOW bound of a product: with a relative threshold (theta2 =
// fl64(theta^2) > 0) it is (theta2 s_A0) s_B0 from the roots of the two
// trees' own pyramids, i.e. norm product < theta ||A||_F ||B||_F; else the
// absolute L2.
__device__ inline double low_bound(double L2, double theta2, const double *__restrict__ rootA,
                                   const double *__restrict__ rootB)
{
    return theta2 > 0.0 ? (theta2 * rootA[0]) * rootB[0] : L2;
}

__device__ inline int lane_id() { return __lane_id(); }

__device__ inline uint64_t lanes_below() { return (uint64_t(1) << lane_id()) - 1; }

// One product in a (possibly batched) leaf-GEMM launch: grid blocks
// [block0, block0 + nblocks) work on this job (blocks of 2 x 2 output leaves,
// or of 4 x 4 for the wide split kernel).  tA / tBT point to the FP32
// leaves (LeafLayout), tA16 / tBT16 to the 16-bit ones (Leaf16Layout: BF16,
// or FP16 at the per-leaf scale exponents escA / escB).
struct GemmJob {
    const void *tA;
    const void *tBT;
    const uint32_t *browptr;
    const uint32_t *bent;
    float *C;
    int64_t n;
    uint32_t nblocks, block0;
    uint32_t nleaf;        // leaves per dimension, N = 2^d
    int32_t single;        // depth 0: one leaf
    int32_t skip_empty;    // blocks without products write nothing (their C
                           // leaves keep what they held), else they write zeros
    // split precision: BF16 leaf copies and the LOW schedule (tA/tBT,
    // browptr/bent then hold the FP32 copies and the HIGH schedule), else null
    const void *tA16;
    const void *tBT16;
    const uint32_t *browptr_lo;
    const uint32_t *bent_lo;
    // sub-leaf culling (n_b = 64, 32 x 32 sub-blocks), else null
    const double *subA;    // tier d+1 norms of A: 4 per leaf, child 2a + c
    const double *subB;    // tier d+1 norms of B
    double T2;             // tau^2
    uint8_t *submask;      // per (entry, wave): performed sub-products, bit 2(2a+b)+c
    unsigned long long *subK;  // count of performed sub-products
    // sparsified trees: storage slot of each leaf (linear index), else null
    const uint32_t *slotA;
    const uint32_t *slotB;
    // FP16 split: scale exponent of every leaf (linear index), else null
    const int32_t *escA;
    const int32_t *escB;
};

// Storage position of leaf `l` of a tree: its slot when the tree is
// sparsified (only kept leaves stored), else l itself.
__device__ inline int64_t leaf_slot(const uint32_t *slot, uint32_t l)
{
    return slot != nullptr ? (int64_t)slot[l] : (int64_t)l;
}

constexpr int kMaxJobs = 16;

// Leaf-GEMM kernels of a launch: whole FP32 leaf products, split precision
// (LOW on BF16 or scaled FP16, HIGH on FP32, one kernel), FP32 with sub-leaf
// culling.
enum class GemmKind { Fp32, Split, SplitF16, Sub, SplitWide, Wide32, SubWide, SplitX3,
                      SplitWideX3 };

struct GemmJobs {          // passed by value as a kernel argument
    int32_t njobs;
    uint32_t nblocks;      // total grid
    GemmJob job[kMaxJobs];
};

}  // namespace spamm

// ---- internal handles ------------------------------------------------------
struct spamm_tree {
    int device;
    hipStream_t stream;     // stream the tree was built on (frees are ordered there)
    int64_t n, np;
    int32_t leaf, depth;
    float *tiles;           // N^2 leaves (left-operand copy), linear-index order, LeafLayout
    float *tilesT;          // the same leaves transposed (right-operand copy), LeafLayout
    uint16_t *tiles16;      // 16-bit left-operand copy (Leaf16Layout), or null
    uint16_t *tilesT16;     // 16-bit right-operand (transposed) copy, or null
    bool fp16;              // the 16-bit copies are FP16 at scale16, else BF16
    int32_t *scale16;       // FP16 copies: scale exponent e of every leaf, else null
    double *norms;          // tiers 0..d (0..d+1 with sub-norms), tier_offset layout
    double root;            // ||A||_F^2
    bool borrowed;          // buffers carved from a caller's arena (not freed here)
    void *block;            // dense trees: the one allocation holding every buffer
    bool sub;               // tier d+1 holds the norms of the 32 x 32 sub-blocks (n_b = 64)
    // epsilon-sparsified tree: only the kept leaves are stored, leaf l at
    // slot[l] (dropped leaves have norm 0 and are never read); else null
    uint32_t *slot;
    uint32_t *keep;         // 1 per stored leaf (linear index), sparsified trees
    int64_t stored;         // leaves held in tiles (N^2 for a dense tree)
    double root_dense;      // ||A||_F^2 before dropping (== root for a dense tree)
};

struct spamm_plan {
    int device;
    hipStream_t stream;
    const spamm_tree *A, *B;
    int32_t depth, leaf;
    int64_t n;
    double tau, T2;
    int32_t precision;      // SPAMM_PREC_*
    double low_tol, L2;     // split: LOW iff s_A s_B < L2 = low_tol^2 (absolute)
    double low_rel, theta2; // split, relative: L2 = (theta2 s_A0) s_B0 on the device,
                            // theta2 = low_rel^2 (0 when the threshold is absolute)
    // tier lists for t < d: CSR over the 4^t tier-t output tiles (linear
    // index), entries = kept k at that tier, ascending
    uint32_t *rowptr;       // all tiers t = 0..d-1, offset rp_off[t], 4^t + 1 each
    int64_t rp_off[spamm::kMaxDepth + 1];
    uint32_t *list[2];      // ping-pong tier lists
    uint32_t *counts;       // per-child-tile counts of the tier being built
    uint32_t *partials;     // scan block sums
    // leaf-tier schedule: CSR over the GEMM blocks (tier d-1 tiles, or the
    // single leaf when d = 0); entry = k | (quadrant mask << 16)
    uint32_t *browptr;      // HIGH (FP32) products
    uint32_t *bent;
    uint32_t *browptr_lo;   // LOW (BF16) products, split precision only
    uint32_t *bent_lo;
    uint64_t *leafK;        // [0] HIGH, [1] LOW kept leaf products, [2] sub-products done,
                            // [3], [4] ||A||_F^2, ||B||_F^2 (FP64 bits, written by the cull)
    uint8_t *submask;       // sub-leaf culling: 4 bytes per leaf-tier entry, else null
    int32_t sub;            // sub-leaf culling in the numeric multiply
    int64_t nblocks;
    void *block;            // the plan's one allocation (all buffers), or null in an arena
};
