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
// with a 4-bit mask of the leaves (q) that take the product.
#include "common.hpp"

namespace spamm {

// Root triple (0,0,0) at tier 0.
__global__ void cull_root(const double *__restrict__ nA, const double *__restrict__ nB, double T2,
                          uint32_t *__restrict__ rowptr0, uint32_t *__restrict__ list0,
                          uint32_t *__restrict__ browptr, uint32_t *__restrict__ bent,
                          uint64_t *__restrict__ leafK, int last)
{
    if (threadIdx.x != 0 || blockIdx.x != 0)
        return;
    const uint32_t kept = keep_pair(nA[0], nB[0], T2) ? 1u : 0u;
    if (last) {
        browptr[0] = 0;
        browptr[1] = kept;
        if (kept)
            bent[0] = 0u | (1u << 16);
        *leafK = kept;
    } else {
        rowptr0[0] = 0;
        rowptr0[1] = kept;
        list0[0] = 0;
        *leafK = 0;
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

// Leaf-tier quadrant mask of inner child c from the 8 flags.
__device__ inline uint32_t mask_of(uint32_t f, int c)
{
    return ((f >> c) & 1u) | (((f >> (2 + c)) & 1u) << 1) | (((f >> (4 + c)) & 1u) << 2) |
           (((f >> (6 + c)) & 1u) << 3);
}

template <bool LAST>
__global__ __launch_bounds__(256) void cull_count(const double *__restrict__ nA,
                                                  const double *__restrict__ nB, double T2,
                                                  const uint32_t *__restrict__ prow,
                                                  const uint32_t *__restrict__ plist,
                                                  uint32_t nparents, uint32_t *__restrict__ counts)
{
    const uint32_t P = blockIdx.x * 4u + (threadIdx.x >> 6);
    if (P >= nparents)
        return;
    const int lane = threadIdx.x & 63;
    const uint32_t I = lin_row(P), J = lin_col(P);
    const uint32_t beg = prow[P], end = prow[P + 1];
    uint32_t tot[4] = {0, 0, 0, 0};
    uint32_t entries = 0, tasks = 0;
    for (uint32_t base = beg; base < end; base += kWave) {
        const uint32_t idx = base + lane;
        uint32_t f = 0;
        if (idx < end)
            f = child_flags(nA, nB, T2, I, plist[idx], J);
        if constexpr (LAST) {
            const uint32_t m0 = mask_of(f, 0), m1 = mask_of(f, 1);
            entries += __popcll(__ballot(m0 != 0)) + __popcll(__ballot(m1 != 0));
            tasks += __popc(f);
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                tot[q] += __popcll(__ballot((f >> (2 * q)) & 1u)) +
                          __popcll(__ballot((f >> (2 * q + 1)) & 1u));
        }
    }
    if constexpr (LAST) {
        // entries per block for the GEMM schedule; leaf products per block
        // (counts[nparents + P]) are summed by reduce_tasks
        for (int o = 32; o > 0; o >>= 1)
            tasks += __shfl_xor(tasks, o);
        if (lane == 0) {
            counts[P] = entries;
            counts[nparents + P] = tasks;
        }
    } else {
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                counts[4 * P + q] = tot[q];
        }
    }
}

template <bool LAST>
__global__ __launch_bounds__(256) void cull_emit(const double *__restrict__ nA,
                                                 const double *__restrict__ nB, double T2,
                                                 const uint32_t *__restrict__ prow,
                                                 const uint32_t *__restrict__ plist,
                                                 uint32_t nparents,
                                                 const uint32_t *__restrict__ crow,
                                                 uint32_t *__restrict__ clist)
{
    const uint32_t P = blockIdx.x * 4u + (threadIdx.x >> 6);
    if (P >= nparents)
        return;
    const int lane = threadIdx.x & 63;
    const uint64_t below = lanes_below();
    const uint32_t I = lin_row(P), J = lin_col(P);
    const uint32_t beg = prow[P], end = prow[P + 1];
    uint32_t run[4];
    if constexpr (LAST) {
        run[0] = crow[P];
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            run[q] = crow[4 * P + q];
    }
    for (uint32_t base = beg; base < end; base += kWave) {
        const uint32_t idx = base + lane;
        uint32_t f = 0, kp = 0;
        if (idx < end) {
            kp = plist[idx];
            f = child_flags(nA, nB, T2, I, kp, J);
        }
        if constexpr (LAST) {
            const uint32_t m0 = mask_of(f, 0), m1 = mask_of(f, 1);
            const uint64_t b0 = __ballot(m0 != 0), b1 = __ballot(m1 != 0);
            const uint32_t pos = run[0] + __popcll(b0 & below) + __popcll(b1 & below);
            if (m0)
                clist[pos] = (2 * kp) | (m0 << 16);
            if (m1)
                clist[pos + (m0 ? 1 : 0)] = (2 * kp + 1) | (m1 << 16);
            run[0] += __popcll(b0) + __popcll(b1);
        } else {
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
}

// Sum of m uint32 values into one uint64 (single workgroup).
__global__ __launch_bounds__(1024) void reduce_tasks(const uint32_t *__restrict__ in, uint32_t m,
                                                     uint64_t *__restrict__ out)
{
    __shared__ uint64_t part[1024 / kWave];
    uint64_t s = 0;
    for (uint32_t i = threadIdx.x; i < m; i += blockDim.x)
        s += in[i];
    for (int o = 32; o > 0; o >>= 1)
        s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0)
        part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i)
            t += part[i];
        *out = t;
    }
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
__global__ __launch_bounds__(kScanThreads) void scan_single(const uint32_t *__restrict__ in, uint32_t m,
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

// partials needs ceil(m / kScanChunk) + 1 entries.
static hipError_t launch_scan(const uint32_t *in, uint32_t m, uint32_t *out, uint32_t *partials,
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

hipError_t launch_cull(spamm_plan *p, hipStream_t s)
{
    const int d = p->depth;
    const double *nA = p->A->norms, *nB = p->B->norms;
    hipLaunchKernelGGL(cull_root, dim3(1), dim3(64), 0, s, nA, nB, p->T2, p->rowptr + p->rp_off[0],
                       p->list[0], p->browptr, p->bent, p->leafK, d == 0 ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || d == 0)
        return e;
    for (int t = 1; t <= d; ++t) {
        const uint32_t np = 1u << (2 * (t - 1));
        const double *tA = nA + tier_offset(t), *tB = nB + tier_offset(t);
        const uint32_t *prow = p->rowptr + p->rp_off[t - 1];
        const uint32_t *plist = p->list[(t - 1) & 1];
        const dim3 grid((np + 3) / 4), block(256);
        if (t < d) {
            uint32_t *crow = p->rowptr + p->rp_off[t];
            hipLaunchKernelGGL(cull_count<false>, grid, block, 0, s, tA, tB, p->T2, prow, plist, np,
                               p->counts);
            if ((e = hipGetLastError()) != hipSuccess)
                return e;
            if ((e = launch_scan(p->counts, 4 * np, crow, p->partials, s)) != hipSuccess)
                return e;
            hipLaunchKernelGGL(cull_emit<false>, grid, block, 0, s, tA, tB, p->T2, prow, plist, np,
                               (const uint32_t *)crow, p->list[t & 1]);
        } else {
            hipLaunchKernelGGL(cull_count<true>, grid, block, 0, s, tA, tB, p->T2, prow, plist, np,
                               p->counts);
            hipLaunchKernelGGL(reduce_tasks, dim3(1), dim3(1024), 0, s, p->counts + np, np, p->leafK);
            if ((e = hipGetLastError()) != hipSuccess)
                return e;
            if ((e = launch_scan(p->counts, np, p->browptr, p->partials, s)) != hipSuccess)
                return e;
            hipLaunchKernelGGL(cull_emit<true>, grid, block, 0, s, tA, tB, p->T2, prow, plist, np,
                               (const uint32_t *)p->browptr, p->bent);
        }
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace spamm
