// Symbolic multiply: tier-by-tier cull of the (i,k,j) product space
// (Eq. product under Eq. norm condition), emitting the kept leaf triples
// grouped by output tile and sorted by k.
//
// Tier t holds, for every output tile of that tier (linear index l, Eq.
// linear index), the ascending list of kept inner indices k (CSR).  The
// candidates of tier t are the 8 children (2i+a, 2k+c, 2j+b) of the kept tier
// t-1 triples.  One wave owns one parent output tile P; a lane owns one parent
// k and tests its 8 children on the stored FP64 squared norms.  Since tiers
// are stored in linear-index order, the four children of node (i,k) are the
// contiguous values 4 l(i,k) + {0,1,2,3}, so a lane needs two 32-byte loads.
// Children of P land in tiles 4P + q (q = 2a + b); within one such tile the
// order (parent k ascending, c) is exactly child k ascending, so a wave-local
// ballot prefix gives every output position and no sort is needed.
//
// Each tier is count -> exclusive scan -> emit.  The grid of every launch
// depends only on t, so the whole cull is asynchronous; list capacities are
// the worst case (8^t entries), which never overflows.
//
// Leaf tier: the GEMM works on blocks of 2 x 2 output leaves (the children of
// one tier-(d-1) tile), so the last tier emits per block the union of kept k
// with a 4-bit mask of the leaves (q) that take the product.  With split
// precision each kept leaf product is also classed LOW (s_A s_B < low_tol^2,
// or < (theta^2 s_A0) s_B0 for a relative threshold; 16-bit operands) or
// HIGH (FP32), and the two classes get separate lists.
#include <algorithm>
#include <vector>

#include "runtime.hpp"

namespace spamm {

// Root triple (0,0,0) at tier 0.
__global__ void cull_root(const double *__restrict__ nA, const double *__restrict__ nB, double T2,
                          double L2, double theta2, uint32_t *__restrict__ rowptr0,
                          uint32_t *__restrict__ list0,
                          uint32_t *__restrict__ browptr, uint32_t *__restrict__ bent,
                          uint32_t *__restrict__ browptr_lo, uint32_t *__restrict__ bent_lo,
                          uint64_t *__restrict__ leafK, int last)
{
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    const uint32_t kept = keep_pair(nA[0], nB[0], T2) ? 1u : 0u;
    reinterpret_cast<double *>(leafK)[3] = nA[0];
    reinterpret_cast<double *>(leafK)[4] = nB[0];
    if (last) {
        // d = 0: the root is the only leaf
        const uint32_t low =
            (kept && low_pair(nA[0], nB[0], low_bound(L2, theta2, nA, nB))) ? 1u : 0u;
        browptr[0] = 0;
        browptr[1] = kept & ~low;
        if (kept & ~low)
            bent[0] = 0u | (1u << 16);
        leafK[0] = kept & ~low;
        leafK[1] = 0;
        if (browptr_lo != nullptr) {
            browptr_lo[0] = 0;
            browptr_lo[1] = low;
            if (low)
                bent_lo[0] = 0u | (1u << 16);
            leafK[1] = low;
        }
    } else {
        rowptr0[0] = 0;
        rowptr0[1] = kept;
        list0[0] = 0;
        leafK[0] = leafK[1] = 0;
    }
}

// The 8 keep flags of parent triple (I, kp, J) at child tier t.
// Bit (2q + c) = child (2I+a, 2kp+c, 2J+b), q = 2a + b.
__device__ inline uint32_t child_flags(const double *__restrict__ nA, const double *__restrict__ nB,
                                       double T2, uint32_t I, uint32_t kp, uint32_t J)
{
    const double2 *pa = reinterpret_cast<const double2 *>(nA + 4 * (int64_t)lin_index(I, kp));
    const double2 *pb = reinterpret_cast<const double2 *>(nB + 4 * (int64_t)lin_index(kp, J));
    const double2 a01 = pa[0], a23 = pa[1];   // A children 2a + c
    const double2 b01 = pb[0], b23 = pb[1];   // B children 2c + b
    const double a[4] = {a01.x, a01.y, a23.x, a23.y};
    const double b[4] = {b01.x, b01.y, b23.x, b23.y};
    uint32_t f = 0;
#pragma unroll
    for (int qa = 0; qa < 2; ++qa)
#pragma unroll
        for (int qb = 0; qb < 2; ++qb)
#pragma unroll
            for (int c = 0; c < 2; ++c)
                f |= (keep_pair(a[2 * qa + c], b[2 * c + qb], T2) ? 1u : 0u)
                     << (2 * (2 * qa + qb) + c);
    return f;
}

// The 8 LOW flags (split precision) of the same children, among kept ones.
__device__ inline uint32_t child_low(const double *__restrict__ nA, const double *__restrict__ nB,
                                     double L2, uint32_t I, uint32_t kp, uint32_t J, uint32_t kept)
{
    const double2 *pa = reinterpret_cast<const double2 *>(nA + 4 * (int64_t)lin_index(I, kp));
    const double2 *pb = reinterpret_cast<const double2 *>(nB + 4 * (int64_t)lin_index(kp, J));
    const double2 a01 = pa[0], a23 = pa[1];
    const double2 b01 = pb[0], b23 = pb[1];
    const double a[4] = {a01.x, a01.y, a23.x, a23.y};
    const double b[4] = {b01.x, b01.y, b23.x, b23.y};
    uint32_t f = 0;
#pragma unroll
    for (int qa = 0; qa < 2; ++qa)
#pragma unroll
        for (int qb = 0; qb < 2; ++qb)
#pragma unroll
            for (int c = 0; c < 2; ++c)
                f |= (low_pair(a[2 * qa + c], b[2 * c + qb], L2) ? 1u : 0u) << (2 * (2 * qa + qb) + c);
    return f & kept;
}

// Leaf-tier quadrant mask of inner child c from the 8 flags.
__device__ inline uint32_t mask_of(uint32_t f, int c)
{
    return ((f >> c) & 1u) | (((f >> (2 + c)) & 1u) << 1) | (((f >> (4 + c)) & 1u) << 2) |
           (((f >> (6 + c)) & 1u) << 3);
}

// Tiers below the leaves: per parent output tile P (one wave), the number of
// kept children in each child tile 4P + q.
__device__ inline void count_tile(const double *__restrict__ nA, const double *__restrict__ nB,
                                  double T2, const uint32_t *__restrict__ prow,
                                  const uint32_t *__restrict__ plist, uint32_t P,
                                  uint32_t *__restrict__ counts, int lane)
{
    const uint32_t I = lin_row(P), J = lin_col(P);
    const uint32_t beg = prow[P], end = prow[P + 1];
    uint32_t tot[4] = {0, 0, 0, 0};
    for (uint32_t base = beg; base < end; base += kWave) {
        const uint32_t idx = base + lane;
        uint32_t f = 0;
        if (idx < end)
            f = child_flags(nA, nB, T2, I, plist[idx], J);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            tot[q] += __popcll(__ballot((f >> (2 * q)) & 1u)) +
                      __popcll(__ballot((f >> (2 * q + 1)) & 1u));
    }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            counts[4 * P + q] = tot[q];
    }
}

__global__ __launch_bounds__(256) void cull_count(const double *__restrict__ nA,
                                                  const double *__restrict__ nB, double T2,
                                                  const uint32_t *__restrict__ prow,
                                                  const uint32_t *__restrict__ plist,
                                                  uint32_t nparents, uint32_t *__restrict__ counts)
{
    const uint32_t P = blockIdx.x * 4u + (threadIdx.x >> 6);
    if (P < nparents)
        count_tile(nA, nB, T2, prow, plist, P, counts, threadIdx.x & 63);
}

// Leaf tier: per GEMM block P (a tier-(d-1) tile), the number of schedule
// entries (distinct k with at least one product) and of leaf products, for the
// HIGH list and, when SPLIT, the LOW list.  counts layout (np = nparents):
// [0,np) HIGH entries, [np,2np) HIGH products, [2np,3np) LOW entries,
// [3np,4np) LOW products.
template <bool SPLIT>
__device__ inline void count_leaf_tile(const double *__restrict__ nA,
                                       const double *__restrict__ nB, double T2, double L2,
                                       const uint32_t *__restrict__ prow,
                                       const uint32_t *__restrict__ plist, uint32_t nparents,
                                       uint32_t *__restrict__ counts, uint32_t P, int lane)
{
    const uint32_t I = lin_row(P), J = lin_col(P);
    const uint32_t beg = prow[P], end = prow[P + 1];
    uint32_t ent_hi = 0, ent_lo = 0, tasks_hi = 0, tasks_lo = 0;
    for (uint32_t base = beg; base < end; base += kWave) {
        const uint32_t idx = base + lane;
        uint32_t f = 0, lo = 0;
        if (idx < end) {
            const uint32_t kp = plist[idx];
            f = child_flags(nA, nB, T2, I, kp, J);
            if constexpr (SPLIT)
                lo = child_low(nA, nB, L2, I, kp, J, f);
        }
        const uint32_t hi = f & ~lo;
        ent_hi += __popcll(__ballot(mask_of(hi, 0) != 0)) + __popcll(__ballot(mask_of(hi, 1) != 0));
        tasks_hi += __popc(hi);
        if constexpr (SPLIT) {
            ent_lo += __popcll(__ballot(mask_of(lo, 0) != 0)) + __popcll(__ballot(mask_of(lo, 1) != 0));
            tasks_lo += __popc(lo);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        tasks_hi += __shfl_xor(tasks_hi, o);
        if constexpr (SPLIT)
            tasks_lo += __shfl_xor(tasks_lo, o);
    }
    if (lane == 0) {
        counts[P] = ent_hi;
        counts[nparents + P] = tasks_hi;
        if constexpr (SPLIT) {
            counts[2 * nparents + P] = ent_lo;
            counts[3 * nparents + P] = tasks_lo;
        }
    }
}

template <bool SPLIT>
__global__ __launch_bounds__(256) void cull_count_leaf(const double *__restrict__ nA,
                                                       const double *__restrict__ nB, double T2,
                                                       double L2a, double theta2,
                                                       const double *__restrict__ rootA,
                                                       const double *__restrict__ rootB,
                                                       const uint32_t *__restrict__ prow,
                                                       const uint32_t *__restrict__ plist,
                                                       uint32_t nparents,
                                                       uint32_t *__restrict__ counts)
{
    const uint32_t P = blockIdx.x * 4u + (threadIdx.x >> 6);
    if (P >= nparents)
        return;
    const double L2 = SPLIT ? low_bound(L2a, theta2, rootA, rootB) : 0.0;
    count_leaf_tile<SPLIT>(nA, nB, T2, L2, prow, plist, nparents, counts, P, threadIdx.x & 63);
}

// Writes the kept children of parent output tile P (one wave) into the
// child lists at the positions given by the scanned counts.
__device__ inline void emit_tile(const double *__restrict__ nA, const double *__restrict__ nB,
                                 double T2, const uint32_t *__restrict__ prow,
                                 const uint32_t *__restrict__ plist, uint32_t P,
                                 const uint32_t *__restrict__ crow, uint32_t *__restrict__ clist,
                                 int lane)
{
    const uint64_t below = lanes_below();
    const uint32_t I = lin_row(P), J = lin_col(P);
    const uint32_t beg = prow[P], end = prow[P + 1];
    uint32_t run[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        run[q] = crow[4 * P + q];
    for (uint32_t base = beg; base < end; base += kWave) {
        const uint32_t idx = base + lane;
        uint32_t f = 0, kp = 0;
        if (idx < end) {
            kp = plist[idx];
            f = child_flags(nA, nB, T2, I, kp, J);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t f0 = (f >> (2 * q)) & 1u, f1 = (f >> (2 * q + 1)) & 1u;
            const uint64_t b0 = __ballot(f0), b1 = __ballot(f1);
            const uint32_t pos = run[q] + __popcll(b0 & below) + __popcll(b1 & below);
            if (f0)
                clist[pos] = 2 * kp;
            if (f1)
                clist[pos + f0] = 2 * kp + 1;
            run[q] += __popcll(b0) + __popcll(b1);
        }
    }
}

__global__ __launch_bounds__(256) void cull_emit(const double *__restrict__ nA,
                                                 const double *__restrict__ nB, double T2,
                                                 const uint32_t *__restrict__ prow,
                                                 const uint32_t *__restrict__ plist,
                                                 uint32_t nparents,
                                                 const uint32_t *__restrict__ crow,
                                                 uint32_t *__restrict__ clist)
{
    const uint32_t P = blockIdx.x * 4u + (threadIdx.x >> 6);
    if (P < nparents)
        emit_tile(nA, nB, T2, prow, plist, P, crow, clist, threadIdx.x & 63);
}

// Writes the (k | mask << 16) entries of the flags `fl` of one chunk.
__device__ inline void emit_entries(uint32_t fl, uint32_t kp, uint64_t below, uint32_t &run,
                                    uint32_t *__restrict__ clist)
{
    const uint32_t m0 = mask_of(fl, 0), m1 = mask_of(fl, 1);
    const uint64_t b0 = __ballot(m0 != 0), b1 = __ballot(m1 != 0);
    const uint32_t pos = run + __popcll(b0 & below) + __popcll(b1 & below);
    if (m0)
        clist[pos] = (2 * kp) | (m0 << 16);
    if (m1)
        clist[pos + (m0 ? 1 : 0)] = (2 * kp + 1) | (m1 << 16);
    run += __popcll(b0) + __popcll(b1);
}

template <bool SPLIT>
__device__ inline void emit_leaf_tile(const double *__restrict__ nA,
                                      const double *__restrict__ nB, double T2, double L2,
                                      const uint32_t *__restrict__ prow,
                                      const uint32_t *__restrict__ plist,
                                      const uint32_t *__restrict__ rp_hi,
                                      uint32_t *__restrict__ ent_hi,
                                      const uint32_t *__restrict__ rp_lo,
                                      uint32_t *__restrict__ ent_lo, uint32_t P, int lane)
{
    const uint64_t below = lanes_below();
    const uint32_t I = lin_row(P), J = lin_col(P);
    const uint32_t beg = prow[P], end = prow[P + 1];
    uint32_t run_hi = rp_hi[P], run_lo = 0;
    if constexpr (SPLIT)
        run_lo = rp_lo[P];
    for (uint32_t base = beg; base < end; base += kWave) {
        const uint32_t idx = base + lane;
        uint32_t f = 0, lo = 0, kp = 0;
        if (idx < end) {
            kp = plist[idx];
            f = child_flags(nA, nB, T2, I, kp, J);
            if constexpr (SPLIT)
                lo = child_low(nA, nB, L2, I, kp, J, f);
        }
        emit_entries(f & ~lo, kp, below, run_hi, ent_hi);
        if constexpr (SPLIT)
            emit_entries(lo, kp, below, run_lo, ent_lo);
    }
}

template <bool SPLIT>
__global__ __launch_bounds__(256) void cull_emit_leaf(const double *__restrict__ nA,
                                                      const double *__restrict__ nB, double T2,
                                                      double L2a, double theta2,
                                                      const double *__restrict__ rootA,
                                                      const double *__restrict__ rootB,
                                                      const uint32_t *__restrict__ prow,
                                                      const uint32_t *__restrict__ plist,
                                                      uint32_t nparents,
                                                      const uint32_t *__restrict__ rp_hi,
                                                      uint32_t *__restrict__ ent_hi,
                                                      const uint32_t *__restrict__ rp_lo,
                                                      uint32_t *__restrict__ ent_lo)
{
    const uint32_t P = blockIdx.x * 4u + (threadIdx.x >> 6);
    if (P >= nparents)
        return;
    const double L2 = SPLIT ? low_bound(L2a, theta2, rootA, rootB) : 0.0;
    emit_leaf_tile<SPLIT>(nA, nB, T2, L2, prow, plist, rp_hi, ent_hi, rp_lo, ent_lo, P,
                          threadIdx.x & 63);
}

// ---- exclusive scan of uint32 counts: out[0..m) prefix, out[m] = total -------
constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;
constexpr int kScanChunk = kScanThreads * kScanItems;

// Block-wide exclusive scan of 4 consecutive items per thread; returns the
// thread's prefix and writes the block total to *total (all threads).
__device__ inline uint32_t block_scan4(const uint32_t v[kScanItems], uint32_t *total)
{
    __shared__ uint32_t wsum[kScanThreads / kWave];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t t = v[0] + v[1] + v[2] + v[3];
    uint32_t inc = t;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o);
        if (lane >= o)
            inc += y;
    }
    if (lane == 63)
        wsum[w] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int i = 0; i < kScanThreads / kWave; ++i) {
        const uint32_t x = wsum[i];
        before += (i < w) ? x : 0u;
        all += x;
    }
    __syncthreads();   // wsum may be reused by the caller's next call
    *total = all;
    return before + inc - t;
}

__global__ __launch_bounds__(kScanThreads) void scan_chunk_sums(const uint32_t *__restrict__ in,
                                                                uint32_t m,
                                                                uint32_t *__restrict__ partials)
{
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        v[i] = (base + i < m) ? in[base + i] : 0u;
    uint32_t total;
    block_scan4(v, &total);
    if (threadIdx.x == 0)
        partials[blockIdx.x] = total;
}

// Single workgroup: exclusive scan of in[0..m) (m <= kScanChunk per pass, loops
// otherwise) into out; out[m] = total.
__device__ inline void block_exclusive_scan(const uint32_t *__restrict__ in, uint32_t m,
                                            uint32_t *__restrict__ out)
{
    uint32_t carry = 0;
    for (int64_t c0 = 0; c0 < m; c0 += kScanChunk) {
        const int64_t base = c0 + threadIdx.x * kScanItems;
        uint32_t v[kScanItems];
#pragma unroll
        for (int i = 0; i < kScanItems; ++i)
            v[i] = (base + i < m) ? in[base + i] : 0u;
        uint32_t total;
        uint32_t p = block_scan4(v, &total) + carry;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            if (base + i < m)
                out[base + i] = p;
            p += v[i];
        }
        carry += total;
    }
    if (threadIdx.x == 0)
        out[m] = carry;
}

__global__ __launch_bounds__(kScanThreads) void scan_single(const uint32_t *__restrict__ in, uint32_t m,
                                                            uint32_t *__restrict__ out)
{
    block_exclusive_scan(in, m, out);
}

// Single workgroup: sum of in[0..m) (returned to thread 0).
__device__ inline uint64_t block_sum(const uint32_t *__restrict__ in, uint32_t m)
{
    __shared__ uint64_t part[kScanThreads / kWave];
    uint64_t s = 0;
    for (uint32_t i = threadIdx.x; i < m; i += blockDim.x)
        s += in[i];
    for (int o = 32; o > 0; o >>= 1)
        s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0)
        part[threadIdx.x >> 6] = s;
    __syncthreads();
    uint64_t t = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i)
            t += part[i];
    __syncthreads();   // part may be reused by the caller's next call
    return t;
}

// Leaf tier with few parent tiles (np <= 4 kScanChunk), one workgroup: the
// block row pointers from the HIGH (and, with browptr_lo, LOW) entry counts
// of cull_count_leaf, and the kept leaf products of each class into leafK.
// Replaces two to four launches of the general path for small products.
__global__ __launch_bounds__(kScanThreads) void leaf_scan_totals(const uint32_t *__restrict__ counts,
                                                                 uint32_t np,
                                                                 uint32_t *__restrict__ browptr,
                                                                 uint32_t *__restrict__ browptr_lo,
                                                                 uint64_t *__restrict__ leafK)
{
    block_exclusive_scan(counts, np, browptr);
    const uint64_t hi = block_sum(counts + np, np);
    uint64_t lo = 0;
    if (browptr_lo != nullptr) {
        block_exclusive_scan(counts + 2 * (size_t)np, np, browptr_lo);
        lo = block_sum(counts + 3 * (size_t)np, np);
    }
    if (threadIdx.x == 0) {
        leafK[0] = hi;
        leafK[1] = lo;
    }
}

__global__ __launch_bounds__(kScanThreads) void scan_chunks(const uint32_t *__restrict__ in, uint32_t m,
                                                            const uint32_t *__restrict__ offs,
                                                            uint32_t *__restrict__ out)
{
    const int64_t base = (int64_t)blockIdx.x * kScanChunk + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        v[i] = (base + i < m) ? in[base + i] : 0u;
    uint32_t total;
    uint32_t p = block_scan4(v, &total) + offs[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < m)
            out[base + i] = p;
        p += v[i];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
        out[m] = offs[gridDim.x];   // grand total
}

// Row pointers of tier t start at tier_offset(t) + t (tier u holds 4^u + 1).
__device__ inline int64_t rowptr_offset(int t) { return tier_offset(t) + t; }

// The root and tiers 1..top in one workgroup (top <= kTopTiers): the small
// upper tiers cost one launch instead of three each.  Same count -> scan ->
// emit per tier as the per-tier kernels (the same tests, and the same order
// with four parents per wave), so the lists are identical; barriers separate
// the phases.  Everything the tiers read
// stays in LDS: both pyramids' tiers 1..top, the row pointers, the lists of
// tiers below `top` and the counts, so a tier costs LDS round trips rather
// than dependent global loads.  The row pointers of every tier (the plan's
// kept counts) and the list of tier `top` (read by the next tier's kernels)
// are also written to global memory.
constexpr int kTopTiers = 5;
// offset of tier t (1 <= t <= kTopTiers) in cull_top's LDS copy: tiers 1..t-1
// back to back (4^u values each, a multiple of 4, so every tier starts 32-byte
// aligned)
__host__ __device__ constexpr int top_offset(int t) { return int(((int64_t(1) << (2 * t)) - 4) / 3); }
constexpr int kTopNorms = top_offset(kTopTiers + 1);
// row pointers of tiers 0..kTopTiers back to back (4^t + 1 each)
__host__ __device__ constexpr int top_row_offset(int t) { return int(((int64_t(1) << (2 * t)) - 1) / 3) + t; }
constexpr int kTopRows = top_row_offset(kTopTiers + 1);
// lists of the tiers below the top one: even tiers <= 8^(kTopTiers - 1)
// entries, odd tiers <= 8^(kTopTiers - 2)
constexpr int kTopListEven = 1 << (3 * (kTopTiers - 1));
constexpr int kTopListOdd = 1 << (3 * (kTopTiers - 2));
static_assert(kTopTiers % 2 == 1, "tier kTopTiers - 1 is even");

// The top tiers' parents (tiers 0..4) hold at most 16 values of k, so a wave
// takes four parents at once, one per group of 16 lanes; counts and write
// positions come from the group's bits of each ballot, in the same order as
// the one-parent-per-wave code (parent k ascending, then c).
static_assert(kTopTiers <= 5, "a top-tier parent list fits 16 lanes");

__device__ inline void count_tile16(const double *__restrict__ nA, const double *__restrict__ nB,
                                    double T2, const uint32_t *__restrict__ prow,
                                    const uint32_t *__restrict__ plist, uint32_t P, bool active,
                                    uint32_t *__restrict__ counts, int lane)
{
    const int gl = lane & 15;
    const uint64_t gmask = 0xFFFFull << (lane & 48);
    uint32_t f = 0;
    if (active) {
        const uint32_t beg = prow[P], end = prow[P + 1];
        if (beg + gl < end)
            f = child_flags(nA, nB, T2, lin_row(P), plist[beg + gl], lin_col(P));
    }
    uint32_t tot[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        tot[q] = __popcll(__ballot((f >> (2 * q)) & 1u) & gmask) +
                 __popcll(__ballot((f >> (2 * q + 1)) & 1u) & gmask);
    if (active && gl == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            counts[4 * P + q] = tot[q];
    }
}

__device__ inline void emit_tile16(const double *__restrict__ nA, const double *__restrict__ nB,
                                   double T2, const uint32_t *__restrict__ prow,
                                   const uint32_t *__restrict__ plist, uint32_t P, bool active,
                                   const uint32_t *__restrict__ crow, uint32_t *__restrict__ clist,
                                   int lane)
{
    const int gl = lane & 15;
    const uint64_t gmask = 0xFFFFull << (lane & 48);
    const uint64_t below = lanes_below() & gmask;
    uint32_t f = 0, kp = 0;
    if (active) {
        const uint32_t beg = prow[P], end = prow[P + 1];
        if (beg + gl < end) {
            kp = plist[beg + gl];
            f = child_flags(nA, nB, T2, lin_row(P), kp, lin_col(P));
        }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t f0 = (f >> (2 * q)) & 1u, f1 = (f >> (2 * q + 1)) & 1u;
        const uint64_t b0 = __ballot(f0), b1 = __ballot(f1);
        if (f0 | f1) {
            const uint32_t pos = crow[4 * P + q] + __popcll(b0 & below) + __popcll(b1 & below);
            if (f0)
                clist[pos] = 2 * kp;
            if (f1)
                clist[pos + f0] = 2 * kp + 1;
        }
    }
}

__device__ inline void top_tiers(const double *__restrict__ nA, const double *__restrict__ nB,
                                 double T2, uint32_t *__restrict__ rowptr,
                                 uint32_t *__restrict__ list0, uint32_t *__restrict__ list1,
                                 uint64_t *__restrict__ leafK, int top)
{
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    constexpr int NW = kScanThreads / kWave;
    // tiers 1..top of both pyramids, each tier at a 16-byte aligned offset
    // (the children of a node are read as two 16-byte pairs)
    __shared__ __align__(16) double sA[kTopNorms], sB[kTopNorms];
    __shared__ uint32_t sRow[kTopRows];
    __shared__ uint32_t sList0[kTopListEven], sList1[kTopListOdd];
    __shared__ uint32_t sCnt[4 << (2 * (kTopTiers - 1))];
    for (int t = 1; t <= top; ++t) {
        const int64_t cnt = int64_t(1) << (2 * t);
        for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) {
            sA[top_offset(t) + i] = nA[tier_offset(t) + i];
            sB[top_offset(t) + i] = nB[tier_offset(t) + i];
        }
    }
    if (threadIdx.x == 0) {
        const uint32_t kept = keep_pair(nA[0], nB[0], T2) ? 1u : 0u;
        sRow[0] = 0;
        sRow[1] = kept;
        sList0[0] = 0;
        rowptr[0] = 0;
        rowptr[1] = kept;
        if (top == 0)
            list0[0] = 0;
        leafK[0] = leafK[1] = 0;
        reinterpret_cast<double *>(leafK)[3] = nA[0];
        reinterpret_cast<double *>(leafK)[4] = nB[0];
    }
    __syncthreads();
    for (int t = 1; t <= top; ++t) {
        const uint32_t np = 1u << (2 * (t - 1));
        const double *tA = sA + top_offset(t), *tB = sB + top_offset(t);
        const uint32_t *prow = sRow + top_row_offset(t - 1);
        uint32_t *crow = sRow + top_row_offset(t);
        const uint32_t *plist = (t - 1) & 1 ? sList1 : sList0;
        for (uint32_t P0 = 4 * w; P0 < np; P0 += 4 * NW)
            count_tile16(tA, tB, T2, prow, plist, P0 + (lane >> 4), P0 + (lane >> 4) < np, sCnt,
                         lane);
        __syncthreads();
        // exclusive scan of the counts (4 np <= kScanChunk: one pass) into
        // crow, crow[4 np] = total, in LDS and in the plan's row pointers
        const uint32_t m = 4 * np;
        uint32_t *grow = rowptr + rowptr_offset(t);
        {
            const uint32_t base = threadIdx.x * kScanItems;
            uint32_t v[kScanItems];
#pragma unroll
            for (int i = 0; i < kScanItems; ++i)
                v[i] = (base + i < m) ? sCnt[base + i] : 0u;
            uint32_t total;
            uint32_t pfx = block_scan4(v, &total);
#pragma unroll
            for (int i = 0; i < kScanItems; ++i) {
                if (base + i < m) {
                    crow[base + i] = pfx;
                    grow[base + i] = pfx;
                }
                pfx += v[i];
            }
            if (threadIdx.x == 0) {
                crow[m] = total;
                grow[m] = total;
            }
        }
        __syncthreads();
        // the top tier's list goes to the plan (the next tier reads it)
        uint32_t *clist = t == top ? (t & 1 ? list1 : list0) : (t & 1 ? sList1 : sList0);
        for (uint32_t P0 = 4 * w; P0 < np; P0 += 4 * NW)
            emit_tile16(tA, tB, T2, prow, plist, P0 + (lane >> 4), P0 + (lane >> 4) < np, crow,
                        clist, lane);
        __syncthreads();
    }
}

__global__ __launch_bounds__(kScanThreads) void cull_top(const double *__restrict__ nA,
                                                         const double *__restrict__ nB, double T2,
                                                         uint32_t *__restrict__ rowptr,
                                                         uint32_t *__restrict__ list0,
                                                         uint32_t *__restrict__ list1,
                                                         uint64_t *__restrict__ leafK, int top)
{
    top_tiers(nA, nB, T2, rowptr, list0, list1, leafK, top);
}

// partials needs ceil(m / kScanChunk) + 1 entries.
hipError_t launch_scan_u32(const uint32_t *in, uint32_t m, uint32_t *out, uint32_t *partials,
                           hipStream_t s)
{
    if (m <= (uint32_t)kScanChunk * 4) {
        hipLaunchKernelGGL(scan_single, dim3(1), dim3(kScanThreads), 0, s, in, m, out);
        return hipGetLastError();
    }
    const uint32_t nb = (m + kScanChunk - 1) / kScanChunk;
    hipLaunchKernelGGL(scan_chunk_sums, dim3(nb), dim3(kScanThreads), 0, s, in, m, partials);
    // exclusive scan of the chunk sums in place (partials[nb] = total)
    hipLaunchKernelGGL(scan_single, dim3(1), dim3(kScanThreads), 0, s, partials, nb, partials);
    hipLaunchKernelGGL(scan_chunks, dim3(nb), dim3(kScanThreads), 0, s, in, m, partials, out);
    return hipGetLastError();
}

size_t scan_partials_len(uint32_t m) { return (m + kScanChunk - 1) / kScanChunk + 1; }

// Sum of m uint32 values into one uint64 (single workgroup).
__global__ __launch_bounds__(kScanThreads) void reduce_tasks(const uint32_t *__restrict__ in,
                                                             uint32_t m, uint64_t *__restrict__ out)
{
    const uint64_t t = block_sum(in, m);
    if (threadIdx.x == 0)
        *out = t;
}

hipError_t launch_cull(spamm_plan *p, hipStream_t s)
{
    const int d = p->depth;
    const bool split = p->precision != SPAMM_PREC_FP32;
    const double *nA = p->A->norms, *nB = p->B->norms;
    hipError_t e;
    if (d == 0) {
        hipLaunchKernelGGL(cull_root, dim3(1), dim3(64), 0, s, nA, nB, p->T2, split ? p->L2 : 0.0,
                           split ? p->theta2 : 0.0, p->rowptr + p->rp_off[0], p->list[0], p->browptr, p->bent,
                           p->browptr_lo, p->bent_lo, p->leafK, 1);
        return hipGetLastError();
    }
    // root and the upper tiers in one workgroup, the rest tier by tier
    const int top = d - 1 < kTopTiers ? d - 1 : kTopTiers;
    hipLaunchKernelGGL(cull_top, dim3(1), dim3(kScanThreads), 0, s, nA, nB, p->T2, p->rowptr,
                       p->list[0], p->list[1], p->leafK, top);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    for (int t = top + 1; t <= d; ++t) {
        const uint32_t np = 1u << (2 * (t - 1));
        const double *tA = nA + tier_offset(t), *tB = nB + tier_offset(t);
        const uint32_t *prow = p->rowptr + p->rp_off[t - 1];
        const uint32_t *plist = p->list[(t - 1) & 1];
        const dim3 grid((np + 3) / 4), block(256);
        if (t < d) {
            uint32_t *crow = p->rowptr + p->rp_off[t];
            hipLaunchKernelGGL(cull_count, grid, block, 0, s, tA, tB, p->T2, prow, plist, np, p->counts);
            if ((e = hipGetLastError()) != hipSuccess)
                return e;
            if ((e = launch_scan_u32(p->counts, 4 * np, crow, p->partials, s)) != hipSuccess)
                return e;
            hipLaunchKernelGGL(cull_emit, grid, block, 0, s, tA, tB, p->T2, prow, plist, np,
                               (const uint32_t *)crow, p->list[t & 1]);
        } else {
            if (split)
                hipLaunchKernelGGL(cull_count_leaf<true>, grid, block, 0, s, tA, tB, p->T2, p->L2,
                                   p->theta2, nA, nB, prow, plist, np, p->counts);
            else
                hipLaunchKernelGGL(cull_count_leaf<false>, grid, block, 0, s, tA, tB, p->T2, 0.0,
                                   0.0, nA, nB, prow, plist, np, p->counts);
            if ((e = hipGetLastError()) != hipSuccess)
                return e;
            if (np <= (uint32_t)kScanChunk * 4) {
                // row pointers and totals in one workgroup
                hipLaunchKernelGGL(leaf_scan_totals, dim3(1), dim3(kScanThreads), 0, s, p->counts,
                                   np, p->browptr, split ? p->browptr_lo : (uint32_t *)nullptr,
                                   p->leafK);
                if ((e = hipGetLastError()) != hipSuccess)
                    return e;
            } else {
                hipLaunchKernelGGL(reduce_tasks, dim3(1), dim3(kScanThreads), 0, s, p->counts + np,
                                   np, p->leafK);
                if (split)
                    hipLaunchKernelGGL(reduce_tasks, dim3(1), dim3(kScanThreads), 0, s,
                                       p->counts + 3 * (size_t)np, np, p->leafK + 1);
                if ((e = hipGetLastError()) != hipSuccess)
                    return e;
                if ((e = launch_scan_u32(p->counts, np, p->browptr, p->partials, s)) != hipSuccess)
                    return e;
                if (split && (e = launch_scan_u32(p->counts + 2 * (size_t)np, np, p->browptr_lo,
                                                  p->partials, s)) != hipSuccess)
                    return e;
            }
            if (split)
                hipLaunchKernelGGL(cull_emit_leaf<true>, grid, block, 0, s, tA, tB, p->T2, p->L2,
                                   p->theta2, nA, nB, prow, plist, np,
                                   (const uint32_t *)p->browptr, p->bent,
                                   (const uint32_t *)p->browptr_lo, p->bent_lo);
            else
                hipLaunchKernelGGL(cull_emit_leaf<false>, grid, block, 0, s, tA, tB, p->T2, 0.0,
                                   0.0, nA, nB, prow, plist, np, (const uint32_t *)p->browptr, p->bent,
                                   (const uint32_t *)nullptr, (uint32_t *)nullptr);
        }
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    // leafK[0] = HIGH leaf products, leafK[1] = LOW ones (0 without split),
    // leafK[3], leafK[4] = the roots ||A||_F^2, ||B||_F^2 (FP64 bit patterns)
    return hipSuccess;
}

// ---- rounds: the culls of several plans in shared launches -----------------
// The same per-wave code as the per-plan kernels above, so every plan's
// lists are the ones its own cull would give; plans of depth 1..8.
__global__ __launch_bounds__(kScanThreads) void cull_top_jobs(const Jobs<TopJob> jobs)
{
    const TopJob &j = jobs.job[blockIdx.x];
    top_tiers(j.nA, j.nB, j.T2, j.rowptr, j.list0, j.list1, j.leafK, j.top);
}

__global__ __launch_bounds__(256) void cull_count_jobs(const Jobs<TierJob> jobs)
{
    const TierJob &j = job_at(jobs, blockIdx.x);
    const uint32_t P = (blockIdx.x - j.block0) * 4u + (threadIdx.x >> 6);
    if (P < j.np)
        count_tile(j.tA, j.tB, j.T2, j.prow, j.plist, P, j.counts, threadIdx.x & 63);
}

// exclusive scan of one plan's 4 np child counts into its row pointers
__global__ __launch_bounds__(kScanThreads) void cull_scan_jobs(const Jobs<TierJob> jobs)
{
    const TierJob &j = jobs.job[blockIdx.x];
    block_exclusive_scan(j.counts, 4 * j.np, j.crow);
}

__global__ __launch_bounds__(256) void cull_emit_jobs(const Jobs<TierJob> jobs)
{
    const TierJob &j = job_at(jobs, blockIdx.x);
    const uint32_t P = (blockIdx.x - j.block0) * 4u + (threadIdx.x >> 6);
    if (P < j.np)
        emit_tile(j.tA, j.tB, j.T2, j.prow, j.plist, P, j.crow, j.clist, threadIdx.x & 63);
}

__global__ __launch_bounds__(256) void cull_count_leaf_jobs(const Jobs<LeafJob> jobs)
{
    const LeafJob &j = job_at(jobs, blockIdx.x);
    const uint32_t P = (blockIdx.x - j.block0) * 4u + (threadIdx.x >> 6);
    if (P >= j.np)
        return;
    if (j.split)
        count_leaf_tile<true>(j.tA, j.tB, j.T2, low_bound(j.L2, j.theta2, j.nA, j.nB), j.prow,
                              j.plist, j.np, j.counts, P, threadIdx.x & 63);
    else
        count_leaf_tile<false>(j.tA, j.tB, j.T2, 0.0, j.prow, j.plist, j.np, j.counts, P,
                               threadIdx.x & 63);
}

// One workgroup per plan: block row pointers of both classes, the kept leaf
// products into leafK, and the plan's readback words, in one pass over the
// four count arrays (every chunk's loads in flight together, where separate
// scans and sums would each wait for their own).
__global__ __launch_bounds__(kScanThreads) void leaf_totals_jobs(const Jobs<LeafJob> jobs)
{
    const LeafJob &j = jobs.job[blockIdx.x];
    __shared__ uint64_t tsum[kScanThreads / kWave][2];
    const uint32_t np = j.np;
    const uint32_t *ch = j.counts, *cth = j.counts + np;
    const uint32_t *cl = j.counts + 2 * (size_t)np, *ctl = j.counts + 3 * (size_t)np;
    uint32_t carry_h = 0, carry_l = 0;
    uint64_t task_h = 0, task_l = 0;
    for (uint32_t c0 = 0; c0 < np; c0 += kScanChunk) {
        const uint32_t base = c0 + threadIdx.x * kScanItems;
        uint32_t vh[kScanItems], vl[kScanItems];
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            const bool in = base + i < np;
            vh[i] = in ? ch[base + i] : 0u;
            vl[i] = in && j.split ? cl[base + i] : 0u;
            task_h += in ? cth[base + i] : 0u;
            task_l += in && j.split ? ctl[base + i] : 0u;
        }
        uint32_t th, tl;
        uint32_t ph = block_scan4(vh, &th) + carry_h;
        uint32_t pl = block_scan4(vl, &tl) + carry_l;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            if (base + i < np) {
                j.browptr[base + i] = ph;
                if (j.split)
                    j.browptr_lo[base + i] = pl;
            }
            ph += vh[i];
            pl += vl[i];
        }
        carry_h += th;
        carry_l += tl;
    }
    if (threadIdx.x == 0) {
        j.browptr[np] = carry_h;
        if (j.split)
            j.browptr_lo[np] = carry_l;
    }
    for (int o = 32; o > 0; o >>= 1) {
        task_h += __shfl_xor(task_h, o);
        task_l += __shfl_xor(task_l, o);
    }
    if ((threadIdx.x & 63) == 0) {
        tsum[threadIdx.x >> 6][0] = task_h;
        tsum[threadIdx.x >> 6][1] = task_l;
    }
    __syncthreads();
    uint64_t hi = 0, lo = 0;
    for (int i = 0; i < kScanThreads / kWave; ++i) {
        hi += tsum[i][0];
        lo += tsum[i][1];
    }
    if (threadIdx.x == 0) {
        j.leafK[0] = hi;
        j.leafK[1] = lo;
        j.rout[0] = hi;
        j.rout[1] = lo;
        j.rout[2] = 0;
        j.rout[3] = (uint64_t)__double_as_longlong(j.nA[0]);
        j.rout[4] = (uint64_t)__double_as_longlong(j.nB[0]);
    }
}

__global__ __launch_bounds__(256) void cull_emit_leaf_jobs(const Jobs<LeafJob> jobs)
{
    const LeafJob &j = job_at(jobs, blockIdx.x);
    const uint32_t P = (blockIdx.x - j.block0) * 4u + (threadIdx.x >> 6);
    if (P >= j.np)
        return;
    if (j.split)
        emit_leaf_tile<true>(j.tA, j.tB, j.T2, low_bound(j.L2, j.theta2, j.nA, j.nB), j.prow,
                             j.plist, j.browptr, j.bent, j.browptr_lo, j.bent_lo, P,
                             threadIdx.x & 63);
    else
        emit_leaf_tile<false>(j.tA, j.tB, j.T2, 0.0, j.prow, j.plist, j.browptr, j.bent,
                              nullptr, nullptr, P, threadIdx.x & 63);
}

template <typename J>
static hipError_t launch_jobs_chunked(const std::vector<J> &all, bool per_block,
                                      void (*kernel)(const Jobs<J>), int threads,
                                      uint32_t (*blocks_of)(const J &), hipStream_t s)
{
    for (size_t i0 = 0; i0 < all.size(); i0 += kMaxRound) {
        Jobs<J> t{};
        for (size_t i = i0; i < all.size() && t.njobs < kMaxRound; ++i) {
            J j = all[i];
            j.block0 = per_block ? (uint32_t)t.njobs : t.nblocks;
            t.nblocks += per_block ? 1u : blocks_of(j);
            t.job[t.njobs++] = j;
        }
        hipLaunchKernelGGL(kernel, dim3(t.nblocks), dim3(threads), 0, s, t);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

static uint32_t tier_blocks(const TierJob &j) { return (j.np + 3) / 4; }
static uint32_t leaf_blocks(const LeafJob &j) { return (j.np + 3) / 4; }
static uint32_t one_block(const TopJob &) { return 1; }

// The culls of `nplans` plans (depth 1..8, buffers carved): the upper tiers
// of all in one launch, then each deeper tier's count -> scan -> emit over
// the plans that have it, then the leaf tier of all.
hipError_t launch_cull_round(const spamm_plan *const *plans, int nplans, uint64_t *rout,
                             hipStream_t s)
{
    std::vector<TopJob> tops;
    int dmax = 0;
    for (int i = 0; i < nplans; ++i) {
        const spamm_plan *p = plans[i];
        if (p->depth < 1 || p->depth > 8)
            return hipErrorInvalidValue;
        TopJob t{};
        t.nA = p->A->norms;
        t.nB = p->B->norms;
        t.rowptr = p->rowptr;
        t.list0 = p->list[0];
        t.list1 = p->list[1];
        t.leafK = p->leafK;
        t.T2 = p->T2;
        t.top = p->depth - 1 < kTopTiers ? p->depth - 1 : kTopTiers;
        tops.push_back(t);
        dmax = std::max(dmax, (int)p->depth);
    }
    hipError_t e = launch_jobs_chunked(tops, true, cull_top_jobs, kScanThreads, one_block, s);
    for (int t = kTopTiers + 1; t < dmax && e == hipSuccess; ++t) {
        std::vector<TierJob> tiers;
        for (int i = 0; i < nplans; ++i) {
            const spamm_plan *p = plans[i];
            if (t >= p->depth)
                continue;
            TierJob j{};
            j.tA = p->A->norms + tier_offset(t);
            j.tB = p->B->norms + tier_offset(t);
            j.prow = p->rowptr + p->rp_off[t - 1];
            j.plist = p->list[(t - 1) & 1];
            j.counts = p->counts;
            j.crow = p->rowptr + p->rp_off[t];
            j.clist = p->list[t & 1];
            j.T2 = p->T2;
            j.np = 1u << (2 * (t - 1));
            tiers.push_back(j);
        }
        e = launch_jobs_chunked(tiers, false, cull_count_jobs, 256, tier_blocks, s);
        if (e == hipSuccess)
            e = launch_jobs_chunked(tiers, true, cull_scan_jobs, kScanThreads, tier_blocks, s);
        if (e == hipSuccess)
            e = launch_jobs_chunked(tiers, false, cull_emit_jobs, 256, tier_blocks, s);
    }
    std::vector<LeafJob> leaves;
    for (int i = 0; i < nplans; ++i) {
        const spamm_plan *p = plans[i];
        const int d = p->depth;
        const bool split = p->precision != SPAMM_PREC_FP32;
        LeafJob j{};
        j.tA = p->A->norms + tier_offset(d);
        j.tB = p->B->norms + tier_offset(d);
        j.nA = p->A->norms;
        j.nB = p->B->norms;
        j.prow = p->rowptr + p->rp_off[d - 1];
        j.plist = p->list[(d - 1) & 1];
        j.counts = p->counts;
        j.browptr = p->browptr;
        j.bent = p->bent;
        j.browptr_lo = split ? p->browptr_lo : nullptr;
        j.bent_lo = split ? p->bent_lo : nullptr;
        j.leafK = p->leafK;
        j.rout = rout + 5 * (size_t)i;
        j.T2 = p->T2;
        j.L2 = split ? p->L2 : 0.0;
        j.theta2 = split ? p->theta2 : 0.0;
        j.np = 1u << (2 * (d - 1));
        j.split = split ? 1 : 0;
        leaves.push_back(j);
    }
    if (e == hipSuccess)
        e = launch_jobs_chunked(leaves, false, cull_count_leaf_jobs, 256, leaf_blocks, s);
    if (e == hipSuccess)
        e = launch_jobs_chunked(leaves, true, leaf_totals_jobs, kScanThreads, leaf_blocks, s);
    if (e == hipSuccess)
        e = launch_jobs_chunked(leaves, false, cull_emit_leaf_jobs, 256, leaf_blocks, s);
    return e;
}

}  // namespace spamm
