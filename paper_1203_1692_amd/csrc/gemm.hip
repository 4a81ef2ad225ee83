// Numeric multiply: C_ij = sum over kept k (ascending) of A_ik B_kj
// (Eq. product; the multiply phase of Alg. 1) on FP32 MFMA with FP32
// accumulation; with split precision the LOW products run on BF16 or FP16
// MFMA in the same kernel.
//
// Ownership.  A workgroup of 4 waves owns one block of 2 x 2 output leaves
// (the children of one tier-(d-1) tile); wave q = 2a + b owns leaf
// (2I+a, 2J+b) and is its only writer, so no atomics touch C.  The block walks
// the union of its leaves' kept k (entries k | mask << 16 from the cull); for
// each entry the needed A_(2I+a, k) (left-operand copy) and B_(k, 2J+b)
// (right-operand copy, stored transposed) go to LDS once and every wave whose
// mask bit is set multiplies from there.  Every output leaf is written once,
// with zeros where nothing was kept, cropped to n.
//
// Pipeline.  The unit of staging is one k-panel of the four operand leaves
// (LeafLayout: n_b x 32 floats each, 32 KB for all four at n_b = 64).  Wave w
// copies operand leaf w's panel with direct-to-LDS loads (global_load_lds,
// 1 KB per instruction, no registers), into one of two LDS buffers: the copy
// of stage t+1 is in flight while stage t is multiplied.  One barrier per
// stage.  The block's entry list is copied to LDS first.  Two workgroups per
// CU (68 KB LDS each at n_b = 64).
//
// Operand feed.  In a panel, lane l reads 4 consecutive k of its row with one
// conflict-free ds_read_b128.  v_mfma_f32_32x32x2_f32: A operand of lane l is
// A[l%32][k0 + l/32], B operand B[k0 + l/32][l%32]; MFMA step s of a 32-wide
// panel pairs the inner indices {s, 16 + s} (lane half h = l/32 supplies
// k = 16 h + s), so one 16-byte read feeds 4 steps.  16x16x4 (n_b = 16,
// one 16-wide panel): lane l supplies k = 4 (l/16) + s, s < 4.  The sum over k
// inside a leaf is the same; only the FP32 summation order inside it differs
// from a plain loop.  Result register v of lane l: D[8(v/4) + 4(l/32) + v%4]
// [l%32] (32x32), D[4(l/16) + v][l%16] (16x16).
#include "common.hpp"

namespace spamm {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void global_void_t;

template <int B>
struct GemmShape {
    using L = LeafLayout<B>;
    static constexpr int kStage = 4 * L::kPanel;                     // floats per stage
    // double-buffered stages, then the block's entry list
    static constexpr size_t kLds = sizeof(float) * 2 * kStage + sizeof(uint32_t) * (1 << kMaxDepth);
};

// Split kernel: the 16-bit stages (four whole leaves, double buffered) and
// the FP32 stages share one area, followed by the entry list and, with FP16
// LOW operands, each entry's four scale exponents (rows 2I, 2I+1, columns
// 2J, 2J+1).
template <int B, bool F16>
struct SplitShape {
    static constexpr size_t kBf16 = sizeof(uint16_t) * 2 * 4 * B * B;
    static constexpr size_t kFp32 = sizeof(float) * 2 * GemmShape<B>::kStage;
    static constexpr size_t kStages = kBf16 > kFp32 ? kBf16 : kFp32;
    static constexpr size_t kEnts = sizeof(uint32_t) * (1 << kMaxDepth);
    static constexpr size_t kLds = kStages + kEnts + (F16 ? 4 * sizeof(int16_t) * (1 << kMaxDepth) : 0);
};

// A block's schedule holds at most one entry per k (N <= 2^kMaxDepth); it is
// copied to LDS once, so a stage reads its entry from there instead of
// waiting on a global load.
constexpr int kMaxEnt = 1 << kMaxDepth;

__device__ inline void load_entries(const uint32_t *__restrict__ bent, uint32_t e0, uint32_t e1,
                                    uint32_t *ents)
{
    for (uint32_t i = threadIdx.x; i < e1 - e0; i += blockDim.x)
        ents[i] = bent[e0 + i];
    __syncthreads();
}

// Workgroups are dispatched round-robin over the 8 XCDs (bid mod 8).  Deal
// the blocks out in chunks of kChunk consecutive ones (linear-index order: a
// square or 2:1 patch of blocks), one chunk of each group of 8 to every XCD,
// each XCD taking its chunks in order: neighbours share an XCD's L2, and
// every XCD samples the whole matrix.  The 2 x 2-block kernels take chunks of
// 16 (their FP16 split product is bound by HBM, and smaller chunks raised
// its traffic by 8 %), the 4 x 4-block ones chunks of 4, which balance the
// heavy diagonal blocks better (301.5 against 305.1 ms for the FP32 product
// and 20.9 against 21.6 ms for the BF16 split one at n = 32768; chunks of 32
// and 64 were slower still).  The chunk an XCD takes from group g is
// rotated by g: chunk c mod 8 is three bits of the linear index, and on the
// diagonal (i = j) two of them are equal, so a fixed c mod 8 gave the
// diagonal's heavy blocks to half of the XCDs (rotated: 305.5 against 314.8
// ms for the FP32 product at n = 32768, tau = 1e-8).  (Contiguous eighths of
// the linear index put the two off-diagonal quadrants, where decaying
// products are few, on half of the XCDs: with split precision the busiest
// XCD then held 1.2x its share of the LOW products and 1.8x of the HIGH ones.)
template <uint32_t kChunk>
__device__ inline uint32_t xcd_block(uint32_t bid, uint32_t nblocks)
{
    if (nblocks % (8u * kChunk) != 0u)
        return bid;
    const uint32_t x = bid % 8u, s = bid / 8u, g = s / kChunk;
    return (g * 8u + ((x + g) & 7u)) * kChunk + s % kChunk;
}
constexpr uint32_t kChunk2 = 16, kChunk4 = 4;    // 2 x 2 and 4 x 4 blocks

// Wave w copies panel p of operand leaf w (0: A_2I, 1: A_2I+1, 2: B_2J,
// 3: B_2J+1) of entry `ent` into LDS at dst, if the entry's mask needs it.
template <int B>
__device__ inline void stage_issue(uint32_t ent, int p, const float *__restrict__ tA,
                                   const float *__restrict__ tBT, const uint32_t *slotA,
                                   const uint32_t *slotB, uint32_t I0, uint32_t J0, float *dst,
                                   int w, int lane)
{
    using L = LeafLayout<B>;
    // leaves that use operand w: A_2I -> q 0,1; A_2I+1 -> q 2,3; B_2J -> q 0,2;
    // B_2J+1 -> q 1,3
    const uint32_t users = w < 2 ? (0x3u << (2 * w)) : (0x5u << (w - 2));
    const uint32_t k = ent & 0xFFFFu, mask = ent >> 16;
    if ((mask & users) == 0)
        return;
    const float *leaf = w < 2 ? tA + leaf_slot(slotA, lin_index(I0 + w, k)) * (B * B)
                              : tBT + leaf_slot(slotB, lin_index(k, J0 + (w - 2))) * (B * B);
    const float *src = leaf + p * L::kPanel + 4 * lane;
    float *d = dst + w * L::kPanel;
#pragma unroll
    for (int i = 0; i < L::kPanel / 256; ++i)
        __builtin_amdgcn_global_load_lds((global_void_t *)(src + 256 * i), (lds_void_t *)(d + 256 * i),
                                         16, 0, 0);
}

// acc += A_panel * B_panel for a 64- or 32-row leaf (MB = B/32 blocks of
// 32x32 per dimension).  Ap: rows i, 32 columns k; Bp: rows j, 32 columns k.
template <int B>
__device__ inline void panel_mfma32(const float *__restrict__ Ap, const float *__restrict__ Bp,
                                    floatx16 (&acc)[B / 32][B / 32], int lane)
{
    using L = LeafLayout<B>;
    constexpr int MB = B / 32;
    constexpr int NG = L::kKS / 8;     // groups of 4 MFMA steps per lane half
    const int r = lane & 31, h = lane >> 5;
    floatx4 av[2][MB], bv[2][MB];
    auto load = [&](int buf, int g) {
        const int c = (L::kKS / 2) * h + 4 * g;
#pragma unroll
        for (int i = 0; i < MB; ++i)
            av[buf][i] = *reinterpret_cast<const floatx4 *>(Ap + L::pindex(i * 32 + r, c));
#pragma unroll
        for (int j = 0; j < MB; ++j)
            bv[buf][j] = *reinterpret_cast<const floatx4 *>(Bp + L::pindex(j * 32 + r, c));
    };
    load(0, 0);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        if (g + 1 < NG)
            load((g + 1) & 1, g + 1);
        // scheduling fence: the reads issued above stay ahead of this group's
        // MFMAs in registers of their own, rather than being sunk behind them
        // into the same registers (0.3-0.6 % faster, same code otherwise)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int i = 0; i < MB; ++i)
#pragma unroll
                for (int j = 0; j < MB; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[g & 1][i][s], bv[g & 1][j][s],
                                                                     acc[i][j], 0, 0, 0);
    }
}

// As panel_mfma32, with the sub-leaf culling mask of this panel: accumulator
// (i, j) takes the panel only if bit 2 i + j of `pm` is set (wave-uniform).
template <int B>
__device__ inline void panel_mfma32_sub(const float *__restrict__ Ap, const float *__restrict__ Bp,
                                        floatx16 (&acc)[B / 32][B / 32], int lane, uint32_t pm)
{
    using L = LeafLayout<B>;
    constexpr int MB = B / 32;
    constexpr int NG = L::kKS / 8;
    const int r = lane & 31, h = lane >> 5;
    floatx4 av[2][MB], bv[2][MB];
    auto load = [&](int buf, int g) {
        const int c = (L::kKS / 2) * h + 4 * g;
#pragma unroll
        for (int i = 0; i < MB; ++i)
            av[buf][i] = *reinterpret_cast<const floatx4 *>(Ap + L::pindex(i * 32 + r, c));
#pragma unroll
        for (int j = 0; j < MB; ++j)
            bv[buf][j] = *reinterpret_cast<const floatx4 *>(Bp + L::pindex(j * 32 + r, c));
    };
    load(0, 0);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        if (g + 1 < NG)
            load((g + 1) & 1, g + 1);
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int j = 0; j < MB; ++j)
                if ((pm >> (i * MB + j)) & 1u) {
#pragma unroll
                    for (int s = 0; s < 4; ++s)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                            av[g & 1][i][s], bv[g & 1][j][s], acc[i][j], 0, 0, 0);
                }
    }
}

__device__ inline void panel_mfma16(const float *__restrict__ Ap, const float *__restrict__ Bp,
                                    floatx4 &acc, int lane)
{
    using L = LeafLayout<16>;
    const int r = lane & 15, h = lane >> 4;
    const floatx4 av = *reinterpret_cast<const floatx4 *>(Ap + L::pindex(r, 4 * h));
    const floatx4 bv = *reinterpret_cast<const floatx4 *>(Bp + L::pindex(r, 4 * h));
#pragma unroll
    for (int s = 0; s < 4; ++s)
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s], bv[s], acc, 0, 0, 0);
}

// Store (or add to) one output leaf held in MFMA result layout, cropped to n.
template <int B>
__device__ inline void write_leaf32(const floatx16 (&acc)[B / 32][B / 32], int64_t row0,
                                    int64_t col0, int64_t n, float *__restrict__ C, int lane)
{
#pragma unroll
    for (int i = 0; i < B / 32; ++i)
#pragma unroll
        for (int j = 0; j < B / 32; ++j)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int64_t row = row0 + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const int64_t col = col0 + j * 32 + (lane & 31);
                if (row < n && col < n)
                    C[row * n + col] = acc[i][j][v];
            }
}

__device__ inline void write_leaf16(const floatx4 &acc, int64_t row0, int64_t col0, int64_t n,
                                    float *__restrict__ C, int lane)
{
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int64_t row = row0 + 4 * (lane >> 4) + v;
        const int64_t col = col0 + (lane & 15);
        if (row < n && col < n)
            C[row * n + col] = acc[v];
    }
}

// Compensated HIGH products (split precision SPAMM_PREC_SPLIT_BF16X3): the
// FP32 k-panels of panel_mfma32, each entry x taken as its two bfloat16
// parts hi = bf16(x) and lo = bf16(x - hi) (x - hi is exact in FP32), and a
// product a b as hi_a hi_b + hi_a lo_b + lo_a hi_b on the BF16 matrix units
// with FP32 accumulation -- the three-product bfloat16 method of Henry, Tang
// and Heinecke (ARITH 2019), within 2^-14 |a||b| of the exact product per
// term (the dropped lo_a lo_b and the parts below lo: about 3 2^-16) where
// FP32 MFMA is exact; three 32x32x16 BF16 MFMAs replace eight 32x32x2 FP32
// ones.  A lane takes 8 consecutive k of its row (two 16-byte
// reads): lane half h of slice g covers k in [16 h + 8 g, 16 h + 8 g + 8), the
// same for both operands, so each MFMA sums 16 distinct k of the panel.
__device__ inline void bf16_parts4(floatx4 x, uint32_t *hi, uint32_t *lo)
{
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const floatx2 v = {x[2 * p], x[2 * p + 1]};
        const bf16x2 h = __builtin_convertvector(v, bf16x2);        // round to nearest even
        const floatx2 hf = __builtin_convertvector(h, floatx2);      // exact
        const floatx2 r = {v[0] - hf[0], v[1] - hf[1]};               // exact
        hi[p] = __builtin_bit_cast(uint32_t, h);
        lo[p] = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, bf16x2));
    }
}

template <int B>
__device__ inline void panel_mfma_x3(const float *__restrict__ Ap, const float *__restrict__ Bp,
                                     floatx16 (&acc)[B / 32][B / 32], int lane)
{
    using L = LeafLayout<B>;
    static_assert(L::kKS == 32, "two slices of 16 per k-panel");
    constexpr int MB = B / 32;
    const int r = lane & 31, h = lane >> 5;
#pragma unroll
    for (int g = 0; g < 2; ++g) {
        const int c = 16 * h + 8 * g;
        uint32_t ah[MB][4], al[MB][4], bh[MB][4], bl[MB][4];
#pragma unroll
        for (int i = 0; i < MB; ++i) {
            bf16_parts4(*reinterpret_cast<const floatx4 *>(Ap + L::pindex(i * 32 + r, c)), ah[i],
                        al[i]);
            bf16_parts4(*reinterpret_cast<const floatx4 *>(Ap + L::pindex(i * 32 + r, c + 4)),
                        ah[i] + 2, al[i] + 2);
        }
#pragma unroll
        for (int j = 0; j < MB; ++j) {
            bf16_parts4(*reinterpret_cast<const floatx4 *>(Bp + L::pindex(j * 32 + r, c)), bh[j],
                        bl[j]);
            bf16_parts4(*reinterpret_cast<const floatx4 *>(Bp + L::pindex(j * 32 + r, c + 4)),
                        bh[j] + 2, bl[j] + 2);
        }
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int j = 0; j < MB; ++j) {
                const bf16x8 Ah = __builtin_bit_cast(bf16x8, ah[i]);
                const bf16x8 Al = __builtin_bit_cast(bf16x8, al[i]);
                const bf16x8 Bh = __builtin_bit_cast(bf16x8, bh[j]);
                const bf16x8 Bl = __builtin_bit_cast(bf16x8, bl[j]);
                // the two small terms first
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Al, Bh, acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah, Bl, acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(Ah, Bh, acc[i][j], 0, 0, 0);
            }
    }
}

// The HIGH panel routine of a kernel: FP32 MFMA, or compensated BF16.
template <int B, bool X3>
__device__ inline void panel_high(const float *__restrict__ Ap, const float *__restrict__ Bp,
                                  floatx16 (&acc)[B / 32][B / 32], int lane)
{
    if constexpr (X3)
        panel_mfma_x3<B>(Ap, Bp, acc, lane);
    else
        panel_mfma32<B>(Ap, Bp, acc, lane);
}

// FP32 products of one block, n_b >= 32: its entries [e0, e1) of `bent`,
// staged by k-panels (see the pipeline note above), into acc (X3: as
// compensated BF16 products).
template <int B, bool X3 = false>
__device__ inline void fp32_products(const float *__restrict__ tA, const float *__restrict__ tBT,
                                     const uint32_t *slotA, const uint32_t *slotB,
                                     const uint32_t *__restrict__ bent, uint32_t e0, uint32_t e1,
                                     uint32_t I0, uint32_t J0, float *smem, uint32_t *ents, int w,
                                     int lane, floatx16 (&acc)[B / 32][B / 32])
{
    using L = LeafLayout<B>;
    using S = GemmShape<B>;
    constexpr int NP = L::kPanels;
    const int qa = w >> 1, qb = w & 1;
    load_entries(bent, e0, e1, ents);
    const uint32_t T = (e1 - e0) * NP;                  // stages of this block
    if (T > 0)
        stage_issue<B>(ents[0], 0, tA, tBT, slotA, slotB, I0, J0, smem, w, lane);
    for (uint32_t t = 0; t < T; ++t) {
        const uint32_t ent = ents[t / NP];
        // this wave's copies of stage t have landed; after the barrier every
        // wave's have, and every wave is done reading the other buffer
        __builtin_amdgcn_s_waitcnt(0x0F70);             // vmcnt(0)
        __syncthreads();
        if (t + 1 < T)
            stage_issue<B>(ents[(t + 1) / NP], (int)((t + 1) % NP), tA, tBT, slotA, slotB,
                           I0, J0, smem + ((t + 1) & 1) * S::kStage, w, lane);
        if ((ent >> (16 + w)) & 1u) {
            const float *buf = smem + (t & 1) * S::kStage;
            panel_high<B, X3>(buf + qa * L::kPanel, buf + (2 + qb) * L::kPanel, acc, lane);
        }
    }
}

// The job of grid block `bid` (jobs sorted by block0; at most kMaxJobs).
__device__ inline int job_of(const GemmJobs &jobs, uint32_t bid)
{
    int j = 0;
#pragma unroll
    for (int i = 1; i < kMaxJobs; ++i)
        j += (i < jobs.njobs && bid >= jobs.job[i].block0) ? 1 : 0;
    return j;
}

template <int B>
__global__ __launch_bounds__(256) void leaf_gemm(const GemmJobs jobs)
{
    using L = LeafLayout<B>;
    using S = GemmShape<B>;
    constexpr int NP = L::kPanels;
    extern __shared__ float smem[];       // 2 stages x {A_2I, A_2I+1, B_2J, B_2J+1} panels, entries
    const GemmJob &job = jobs.job[job_of(jobs, blockIdx.x)];
    const float *__restrict__ tA = (const float *)job.tA;
    const float *__restrict__ tBT = (const float *)job.tBT;
    const uint32_t *__restrict__ browptr = job.browptr;
    const uint32_t *__restrict__ bent = job.bent;
    float *__restrict__ C = job.C;
    const int64_t n = job.n;
    const int single = job.single;
    const uint32_t blk = xcd_block<kChunk2>(blockIdx.x - job.block0, job.nblocks);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int qa = w >> 1, qb = w & 1;
    uint32_t I0 = 0, J0 = 0;
    if (!single) {
        I0 = 2 * lin_row(blk);
        J0 = 2 * lin_col(blk);
    }

    constexpr int MB = B >= 32 ? B / 32 : 1;
    floatx16 acc[MB][MB];
    floatx4 acc16;
    if constexpr (B >= 32) {
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int j = 0; j < MB; ++j)
                acc[i][j] = floatx16{0};
    } else {
        acc16 = floatx4{0};
    }

    const uint32_t e0 = browptr[blk], e1 = browptr[blk + 1];
    if (job.skip_empty && e0 == e1)
        return;                                          // the same for every wave
    if constexpr (B >= 32) {
        fp32_products<B>(tA, tBT, job.slotA, job.slotB, bent, e0, e1, I0, J0, smem,
                         (uint32_t *)(smem + 2 * S::kStage), w, lane, acc);
        if (single && w != 0)
            return;
        write_leaf32<B>(acc, (int64_t)(I0 + qa) * B, (int64_t)(J0 + qb) * B, n, C, lane);
        return;
    }
    uint32_t *ents = (uint32_t *)(smem + 2 * S::kStage);
    load_entries(bent, e0, e1, ents);
    const uint32_t T = (e1 - e0) * NP;                  // stages of this block
    if (T > 0)
        stage_issue<B>(ents[0], 0, tA, tBT, job.slotA, job.slotB, I0, J0, smem, w, lane);
    for (uint32_t t = 0; t < T; ++t) {
        const uint32_t ent = ents[t / NP];
        // this wave's copies of stage t have landed; after the barrier every
        // wave's have, and every wave is done reading the other buffer
        __builtin_amdgcn_s_waitcnt(0x0F70);             // vmcnt(0)
        __syncthreads();
        if (t + 1 < T)
            stage_issue<B>(ents[(t + 1) / NP], (int)((t + 1) % NP), tA, tBT, job.slotA,
                           job.slotB, I0, J0, smem + ((t + 1) & 1) * S::kStage, w, lane);
        if ((ent >> (16 + w)) & 1u) {
            const float *buf = smem + (t & 1) * S::kStage;
            panel_mfma16(buf + qa * L::kPanel, buf + (2 + qb) * L::kPanel, acc16, lane);
        }
    }
    if (single && w != 0)
        return;
    write_leaf16(acc16, (int64_t)(I0 + qa) * B, (int64_t)(J0 + qb) * B, n, C, lane);
}

// Sub-leaf culling (n_b = 64, 32 x 32 sub-blocks).  For its leaf product
// A_(2I+a', k) B_(k, 2J+b') wave q = 2a' + b' keeps sub-product (a, c, b),
// A_(a, c) B_(c, b), unless its stored sub-block norms fail the test against
// tau, and runs accumulator (a, b) on k-panel c only for the kept ones.
// Before its first copy the block works out every entry's kept sub-products
// (one byte per entry and wave, also written to submask and counted in subK)
// and compacts its stages to the (entry, panel) pairs some wave needs: a
// panel no wave takes is neither copied nor waited for, and an operand leaf's
// panel is copied only if one of its two user waves takes it.  The MFMAs each
// accumulator runs, and their order, are those of the uncompacted loop.
template <int B>
struct SubShape {
    static constexpr size_t kStages = sizeof(float) * 2 * GemmShape<B>::kStage;
    static constexpr size_t kEnts = sizeof(uint32_t) * kMaxEnt;
    static constexpr size_t kMasks = 4 * kMaxEnt;                       // uint8 per entry, wave
    static constexpr size_t kList = sizeof(uint16_t) * 2 * kMaxEnt;     // entry << 1 | panel
    static constexpr size_t kLds = kStages + kEnts + kMasks + kList;
};

template <int B>
__global__ __launch_bounds__(256) void leaf_gemm_sub(const GemmJobs jobs)
{
    static_assert(B == 64, "sub-blocks are the 32 x 32 quadrants of 64 x 64 leaves");
    using L = LeafLayout<B>;
    using S = GemmShape<B>;
    using Z = SubShape<B>;
    constexpr int MB = B / 32;
    static_assert(L::kPanels == 2, "one k-panel per sub-block column");
    static_assert(kMaxEnt == 4 * 256, "four entries per thread cover a block's list");
    extern __shared__ float smem[];
    __shared__ uint32_t wtot[4];
    const GemmJob &job = jobs.job[job_of(jobs, blockIdx.x)];
    const float *__restrict__ tA = (const float *)job.tA;
    const float *__restrict__ tBT = (const float *)job.tBT;
    const int single = job.single;
    const uint32_t blk = xcd_block<kChunk2>(blockIdx.x - job.block0, job.nblocks);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int qa = w >> 1, qb = w & 1;
    uint32_t I0 = 0, J0 = 0;
    if (!single) {
        I0 = 2 * lin_row(blk);
        J0 = 2 * lin_col(blk);
    }
    char *lds = (char *)smem;
    uint32_t *ents = (uint32_t *)(lds + Z::kStages);
    uint8_t *smk = (uint8_t *)(lds + Z::kStages + Z::kEnts);
    uint16_t *list = (uint16_t *)(lds + Z::kStages + Z::kEnts + Z::kMasks);
    const uint32_t e0 = job.browptr[blk], e1 = job.browptr[blk + 1];
    const uint32_t E = e1 - e0;
    load_entries(job.bent, e0, e1, ents);

    // kept sub-products of entries 4 tid .. 4 tid + 3 for all four waves,
    // and the panels each entry needs
    uint32_t need = 0, cnt = 0, subs = 0;            // need: 2 bits per entry
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t i = 4 * threadIdx.x + j;
        if (i >= E)
            break;
        const uint32_t ent = ents[i], k = ent & 0xFFFFu;
        uint32_t word = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint32_t m = 0;
            if ((ent >> (16 + q)) & 1u) {
                const double *sa = job.subA + 4 * (int64_t)lin_index(I0 + (q >> 1), k);
                const double *sb = job.subB + 4 * (int64_t)lin_index(k, J0 + (q & 1));
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
#pragma unroll
                        for (int c = 0; c < 2; ++c)
                            m |= keep_pair(sa[2 * a + c], sb[2 * c + b], job.T2)
                                     ? 1u << (2 * (2 * a + b) + c) : 0u;
            }
            word |= m << (8 * q);
            subs += __builtin_popcount(m);
        }
        *reinterpret_cast<uint32_t *>(smk + 4 * i) = word;
        *reinterpret_cast<uint32_t *>(job.submask + 4 * (int64_t)(e0 + i)) = word;
        const uint32_t nb = ((word & 0x55555555u) ? 1u : 0u) | ((word & 0xAAAAAAAAu) ? 2u : 0u);
        need |= nb << (2 * j);
        cnt += __builtin_popcount(nb);
    }
    // exclusive scan of the per-thread stage counts: stage list in entry order
    uint32_t inc = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o);
        if (lane >= o)
            inc += y;
    }
    if (lane == 63)
        wtot[w] = inc;
    for (int o = 32; o > 0; o >>= 1)
        subs += __shfl_xor(subs, o);
    if (lane == 0 && subs != 0)
        atomicAdd(job.subK, (unsigned long long)subs);
    __syncthreads();
    uint32_t pos = inc - cnt, T = 0;
    for (int v = 0; v < 4; ++v) {
        pos += v < w ? wtot[v] : 0u;
        T += wtot[v];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int c = 0; c < 2; ++c)
            if ((need >> (2 * j + c)) & 1u)
                list[pos++] = (uint16_t)(((4 * threadIdx.x + j) << 1) | c);
    __syncthreads();

    // waves that take panel c of entry i: bit q set
    auto takers = [&](uint32_t st) {
        const uint32_t word = *reinterpret_cast<const uint32_t *>(smk + 4 * (st >> 1));
        const uint32_t m = (word >> (st & 1u)) & 0x55555555u;
        return ((m & 0xFFu) ? 1u : 0u) | ((m & 0xFF00u) ? 2u : 0u) |
               ((m & 0xFF0000u) ? 4u : 0u) | ((m & 0xFF000000u) ? 8u : 0u);
    };
    floatx16 acc[MB][MB];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < MB; ++j)
            acc[i][j] = floatx16{0};
    if (T > 0) {
        const uint32_t st = list[0];
        stage_issue<B>((ents[st >> 1] & 0xFFFFu) | (takers(st) << 16), (int)(st & 1u), tA, tBT,
                       job.slotA, job.slotB, I0, J0, smem, w, lane);
    }
    for (uint32_t t = 0; t < T; ++t) {
        const uint32_t st = list[t];
        __builtin_amdgcn_s_waitcnt(0x0F70);             // vmcnt(0)
        __syncthreads();
        if (t + 1 < T) {
            const uint32_t nx = list[t + 1];
            stage_issue<B>((ents[nx >> 1] & 0xFFFFu) | (takers(nx) << 16), (int)(nx & 1u), tA, tBT,
                           job.slotA, job.slotB, I0, J0, smem + ((t + 1) & 1) * S::kStage, w, lane);
        }
        // accumulator (a, b) of this wave on panel c
        const uint32_t c = st & 1u;
        const uint32_t sm = smk[4 * (st >> 1) + w];
        const uint32_t pm = ((sm >> c) & 1u) | ((sm >> (1 + c)) & 2u) | ((sm >> (2 + c)) & 4u) |
                            ((sm >> (3 + c)) & 8u);
        if (pm != 0u) {
            const float *buf = smem + (t & 1) * S::kStage;
            panel_mfma32_sub<B>(buf + qa * L::kPanel, buf + (2 + qb) * L::kPanel, acc, lane, pm);
        }
    }
    if (single && w != 0)
        return;
    write_leaf32<B>(acc, (int64_t)(I0 + qa) * B, (int64_t)(J0 + qb) * B, job.n, job.C, lane);
}

// ---------------------------------------------------------------------------
// LOW products (split precision): 16-bit operands, FP32 accumulation, on
// v_mfma_f32_32x32x16_bf16 / _f16 (A operand of lane l: A[l%32][k0 + 8(l/32) + i],
// i < 8; B operand B[k0 + 8(l/32) + i][l%32]).  Same ownership and
// double-buffered direct-to-LDS staging as the FP32 loop; a stage is the four
// whole 16-bit leaves of one entry (Leaf16Layout, 8 KB each at n_b = 64).
// F16: the leaves hold x 2^e (e per leaf, escA / escB), so each product is
// accumulated on its own from zero and added as tmp 2^-(eA + eB): one FMA
// with the exact power of two when that is a normal float, else an exact
// ldexp and an add.  The block's exponents are copied to LDS (`eexp`, four
// per entry) before its first stage.
template <int B, bool F16>
__device__ inline void low_products(const uint16_t *__restrict__ tA16,
                                     const uint16_t *__restrict__ tBT16, const uint32_t *slotA,
                                     const uint32_t *slotB, const uint32_t *__restrict__ bent,
                                     uint32_t e0, uint32_t e1, uint32_t I0, uint32_t J0,
                                     uint16_t *smem16, uint32_t *ents, int16_t *eexp, int w,
                                     int lane, const int32_t *escA, const int32_t *escB,
                                     floatx16 (&acc)[B / 32][B / 32])
{
    using L = Leaf16Layout<B>;
    constexpr int LEAF = B * B;            // 16-bit values per leaf
    constexpr int MB = B / 32;
    const int qa = w >> 1, qb = w & 1;
    auto issue = [&](uint32_t ent, uint16_t *dst) {
        const uint32_t users = w < 2 ? (0x3u << (2 * w)) : (0x5u << (w - 2));
        const uint32_t k = ent & 0xFFFFu, mask = ent >> 16;
        if ((mask & users) == 0)
            return;
        const uint16_t *leaf = w < 2 ? tA16 + leaf_slot(slotA, lin_index(I0 + w, k)) * LEAF
                                     : tBT16 + leaf_slot(slotB, lin_index(k, J0 + (w - 2))) * LEAF;
        const uint16_t *src = leaf + 8 * lane;
        uint16_t *d = dst + w * LEAF;
#pragma unroll
        for (int i = 0; i < LEAF / 512; ++i)
            __builtin_amdgcn_global_load_lds((global_void_t *)(src + 512 * i), (lds_void_t *)(d + 512 * i),
                                             16, 0, 0);
    };
    load_entries(bent, e0, e1, ents);
    const uint32_t T = e1 - e0;
    if (T > 0)
        issue(ents[0], smem16);
    if constexpr (F16) {
        // operand o of entry i: rows I0, I0+1 of A (o = 0, 1), columns J0, J0+1
        // of B (o = 2, 3); only the operands the entry's mask uses exist (a
        // single-leaf product has no row I0+1).  Visible after the first
        // stage's barrier.
        for (uint32_t x = threadIdx.x; x < 4 * T; x += blockDim.x) {
            const uint32_t ent = ents[x >> 2], o = x & 3u, k = ent & 0xFFFFu, mask = ent >> 16;
            const uint32_t users = o < 2 ? (0x3u << (2 * o)) : (0x5u << (o - 2));
            int e = 0;
            if (mask & users)
                e = o < 2 ? escA[lin_index(I0 + o, k)] : escB[lin_index(k, J0 + (o - 2))];
            eexp[x] = (int16_t)e;
        }
    }
    const int r = lane & 31, h = lane >> 5;
    for (uint32_t t = 0; t < T; ++t) {
        const uint32_t ent = ents[t];
        __builtin_amdgcn_s_waitcnt(0x0F70);             // vmcnt(0)
        __syncthreads();
        if (t + 1 < T)
            issue(ents[t + 1], smem16 + ((t + 1) & 1) * (4 * LEAF));
        if ((ent >> (16 + w)) & 1u) {
            const uint16_t *buf = smem16 + (t & 1) * (4 * LEAF);
            const uint16_t *Ap = buf + qa * LEAF;
            const uint16_t *Bp = buf + (2 + qb) * LEAF;
            bf16x8 av[B / 16][MB], bv[B / 16][MB];
#pragma unroll
            for (int st = 0; st < B / 16; ++st) {
                const int c = 16 * st + 8 * h;
#pragma unroll
                for (int i = 0; i < MB; ++i)
                    av[st][i] = *reinterpret_cast<const bf16x8 *>(Ap + L::index(i * 32 + r, c));
#pragma unroll
                for (int j = 0; j < MB; ++j)
                    bv[st][j] = *reinterpret_cast<const bf16x8 *>(Bp + L::index(j * 32 + r, c));
            }
            if constexpr (F16) {
                const int esum = (int)eexp[4 * t + qa] + (int)eexp[4 * t + 2 + qb];
                floatx16 tmp[MB][MB];
#pragma unroll
                for (int i = 0; i < MB; ++i)
#pragma unroll
                    for (int j = 0; j < MB; ++j)
                        tmp[i][j] = floatx16{0};
#pragma unroll
                for (int st = 0; st < B / 16; ++st)
#pragma unroll
                    for (int i = 0; i < MB; ++i)
#pragma unroll
                        for (int j = 0; j < MB; ++j)
                            tmp[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                                __builtin_bit_cast(f16x8, av[st][i]),
                                __builtin_bit_cast(f16x8, bv[st][j]), tmp[i][j], 0, 0, 0);
                if (esum >= -126 && esum <= 126) {
                    const float sc = __uint_as_float((uint32_t)(127 - esum) << 23);   // 2^-esum
#pragma unroll
                    for (int i = 0; i < MB; ++i)
#pragma unroll
                        for (int j = 0; j < MB; ++j)
#pragma unroll
                            for (int v = 0; v < 16; ++v)
                                acc[i][j][v] = fmaf(tmp[i][j][v], sc, acc[i][j][v]);
                } else {
#pragma unroll
                    for (int i = 0; i < MB; ++i)
#pragma unroll
                        for (int j = 0; j < MB; ++j)
#pragma unroll
                            for (int v = 0; v < 16; ++v)
                                acc[i][j][v] += ldexpf(tmp[i][j][v], -esum);
                }
            } else {
#pragma unroll
                for (int st = 0; st < B / 16; ++st)
#pragma unroll
                    for (int i = 0; i < MB; ++i)
#pragma unroll
                        for (int j = 0; j < MB; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                av[st][i], bv[st][j], acc[i][j], 0, 0, 0);
            }
        }
    }
}

// Split precision in one launch: every block runs its LOW list (BF16 or
// scaled FP16) and then its HIGH list (FP32), so the few blocks with many HIGH products (the
// large leaves near the diagonal) overlap the LOW work of the others instead
// of forming a second launch of their own.  The classes keep separate
// accumulators (the MFMA result layouts are the same): a leaf is written as
// its LOW sum, plus its HIGH sum in one FP32 addition when the block has HIGH
// entries -- the sums of the paper's product split by class, each over k
// ascending.  X3: the HIGH products as compensated BF16 products of the
// same FP32 stages (panel_mfma_x3).
template <int B, bool F16, bool X3 = false>
__global__ __launch_bounds__(256) void leaf_gemm_split(const GemmJobs jobs)
{
    static_assert(!(F16 && X3), "compensated HIGH products go with BF16 LOW operands");
    constexpr int MB = B / 32;
    extern __shared__ float smem[];        // the 16-bit stages, then the FP32 stages
    const GemmJob &job = jobs.job[job_of(jobs, blockIdx.x)];
    const int single = job.single;
    const uint32_t blk = xcd_block<kChunk2>(blockIdx.x - job.block0, job.nblocks);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int qa = w >> 1, qb = w & 1;
    uint32_t I0 = 0, J0 = 0;
    if (!single) {
        I0 = 2 * lin_row(blk);
        J0 = 2 * lin_col(blk);
    }
    using SS = SplitShape<B, F16>;
    uint32_t *ents = (uint32_t *)((char *)smem + SS::kStages);
    int16_t *eexp = (int16_t *)((char *)smem + SS::kStages + SS::kEnts);
    if (job.skip_empty && job.browptr_lo[blk] == job.browptr_lo[blk + 1] &&
        job.browptr[blk] == job.browptr[blk + 1])
        return;                                          // the same for every wave
    floatx16 lo[MB][MB], hi[MB][MB];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < MB; ++j) {
            lo[i][j] = floatx16{0};
            hi[i][j] = floatx16{0};
        }
    low_products<B, F16>((const uint16_t *)job.tA16, (const uint16_t *)job.tBT16, job.slotA,
                          job.slotB,
                     job.bent_lo, job.browptr_lo[blk], job.browptr_lo[blk + 1], I0, J0,
                     (uint16_t *)smem, ents, eexp, w, lane, job.escA, job.escB, lo);
    __syncthreads();                       // every wave is done with the 16-bit stages
    const uint32_t h0 = job.browptr[blk], h1 = job.browptr[blk + 1];
    fp32_products<B, X3>((const float *)job.tA, (const float *)job.tBT, job.slotA, job.slotB, job.bent,
                     h0, h1, I0, J0, smem, ents, w, lane, hi);
    if (single && w != 0)
        return;
    if (h0 != h1) {
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int j = 0; j < MB; ++j)
                lo[i][j] += hi[i][j];
    }
    write_leaf32<B>(lo, (int64_t)(I0 + qa) * B, (int64_t)(J0 + qb) * B, job.n, job.C, lane);
}

// ---------------------------------------------------------------------------
// Wide split kernel (BF16 LOW operands, n_b = 64, depth >= 2).  A LOW product
// is cheap on the matrix units and its 8 KB operands dominate: with blocks of
// 2 x 2 output leaves every staged leaf feeds at most 2 products (3.1 per
// entry of 4 leaves at the benchmark's matched-error point), and the kernel
// is bound by HBM.  Here a workgroup of 16 waves owns a block of 4 x 4 output
// leaves (a tier-(d-2) node; wave w = 4r + c owns leaf (4I + r, 4J + c) and is
// its only writer), so a staged A leaf feeds up to 4 products and the bytes
// per product fall by about 1.7x.  The schedules come from the cull as the
// four 2 x 2 children's lists; the block merges them in LDS into one list
// per class of (k | 16-bit mask << 16), k ascending.
//
// A stage is the whole 16-bit leaves (8 KB, both k-panels of Leaf16Layout) of
// the up to 4 A leaves (rows) and 4 B leaves (columns) an entry needs: 64 KB
// in a 2-deep LDS ring, the next entry's copies in flight while one is
// multiplied.  A wave waits by vmcnt for its own copies, then the barrier makes
// every wave's copies visible.  (Half leaves in a 4-deep ring, three stages in
// flight, were 8 % slower: the LOW phase is bound by each stage's fixed cost
// -- the barrier, the LDS latency before the first MFMA -- against the MFMA
// work of the busiest SIMD, small when an entry holds few products, not by
// the copies' latency.)  Then the block's HIGH products (few, and
// concentrated in the blocks along the diagonal) on FP32 MFMA: stages of the
// FP32 k-panels (8 KB each, 64 KB per stage) in a 2-deep ring over the same
// LDS.  One running FP32 sum per leaf: its LOW products over k ascending,
// then its HIGH products over k ascending.  (A second launch for the HIGH
// products alone, adding to the LOW sums in C, was 14 % slower: they could
// no longer overlap the LOW work of other blocks.)  X3: the HIGH products as
// compensated BF16 products of the same FP32 stages (at n = 32768 the HIGH
// phase alone 4.4 against 9.6 ms for 1.34 M products).
constexpr int kWideWaves = 16;

// Workgroup barrier without the memory fence of __syncthreads (whose release
// half would wait for every outstanding copy, the prefetched stages
// included): the caller has already waited, by vmcnt, for its own
// direct-to-LDS copies that must be visible, and its LDS reads of the
// buffer about to be refilled were consumed before it got here.  The empty
// asm statements keep the compiler from moving memory accesses across.
__device__ inline void barrier_no_fence()
{
    __asm__ volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    __asm__ volatile("" ::: "memory");
}

constexpr int kWideStage16 = 8 * 64 * 64;                   // 16-bit values per LOW stage
constexpr int kWideStage32 = 8 * LeafLayout<64>::kPanel;     // floats per HIGH stage

struct WideShape {
    static constexpr size_t kRing = sizeof(uint16_t) * 2 * kWideStage16;   // 128 KB
    static_assert(kRing == sizeof(float) * 2 * kWideStage32, "the HIGH ring reuses the LOW one");
    static constexpr size_t kMask = sizeof(uint32_t) * kMaxEnt;
    static constexpr size_t kList = sizeof(uint32_t) * kMaxEnt;
    static constexpr size_t kLds = kRing + kMask + kList + sizeof(uint32_t) * kWideWaves;
};

// Merges the schedules of the four 2 x 2 children of 4 x 4 block P4 into
// list[0..count): k ascending, entry k | mask << 16, mask bit 4 r + c for leaf
// (r, c) of the block.  kmask: kMaxEnt words of scratch; wsum: one word per
// wave.  Returns the count (every thread).
__device__ inline uint32_t merge_children(const uint32_t *__restrict__ rp,
                                          const uint32_t *__restrict__ ent, uint32_t P4,
                                          uint32_t N, uint32_t *kmask, uint32_t *list,
                                          uint32_t *wsum)
{
    for (uint32_t i = threadIdx.x; i < N; i += blockDim.x)
        kmask[i] = 0u;
    __syncthreads();
#pragma unroll
    for (uint32_t ch = 0; ch < 4; ++ch) {
        // child ch = 2a + b holds leaves (2a + a', 2b + b'), its bit q = 2a' + b'
        const uint32_t P2 = 4u * P4 + ch, a = ch >> 1, b = ch & 1u;
        const uint32_t e0 = rp[P2], e1 = rp[P2 + 1];
        for (uint32_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
            const uint32_t x = ent[e], k = x & 0xFFFFu, m = x >> 16;
            uint32_t bits = 0;
#pragma unroll
            for (uint32_t q = 0; q < 4; ++q)
                if ((m >> q) & 1u)
                    bits |= 1u << (4 * (2 * a + (q >> 1)) + 2 * b + (q & 1u));
            atomicOr(&kmask[k], bits);
        }
    }
    __syncthreads();
    // compaction in k order: one slot per thread per round
    uint32_t base = 0;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (uint32_t r0 = 0; r0 < N; r0 += blockDim.x) {
        const uint32_t k = r0 + threadIdx.x;
        const uint32_t m = k < N ? kmask[k] : 0u;
        const uint64_t bal = __ballot(m != 0u);
        if (lane == 0)
            wsum[w] = (uint32_t)__popcll(bal);
        __syncthreads();
        uint32_t before = 0, total = 0;
        for (int i = 0; i < kWideWaves; ++i) {
            const uint32_t c = wsum[i];
            before += i < w ? c : 0u;
            total += c;
        }
        if (m != 0u)
            list[base + before + (uint32_t)__popcll(bal & lanes_below())] = k | (m << 16);
        base += total;
        __syncthreads();                     // wsum is rewritten by the next pass
    }
    return base;
}

// FP32 products of 4 x 4 block P4 (merged list of its children's HIGH, or
// only, schedules): FP32 k-panels (8 KB), 64 KB stages in a 2-deep ring over
// the workgroup's LDS; wave (r, c) adds its leaf's products into acc, k
// ascending (X3: as compensated BF16 products).
template <bool X3 = false>
__device__ inline void wide_fp32_products(const GemmJob &job, uint32_t P4, uint32_t I0,
                                          uint32_t J0, uint32_t NK, int w, int r, int c,
                                          int bit, int lane, float *smem, uint32_t *kmask,
                                          uint32_t *list, uint32_t *wsum, floatx16 (&acc)[2][2])
{
    constexpr int B = 64;
    const int pan = w >> 1, part = w & 1;
    constexpr int P32 = LeafLayout<B>::kPanel;
    float *ring32 = smem;
    const float *__restrict__ tA = (const float *)job.tA;
    const float *__restrict__ tBT = (const float *)job.tBT;
    const uint32_t nhi = merge_children(job.browptr, job.bent, P4, NK, kmask, list, wsum);
    // wave w copies half (w & 1) of FP32 panel w >> 1: four 1 KB copies
    auto issue_hi = [&](uint32_t st) {
        const uint32_t ent = list[st >> 1], k = ent & 0xFFFFu, m = ent >> 16;
        const uint32_t need = pan < 4 ? (m >> (4 * pan)) & 0xFu : (m >> (pan - 4)) & 0x1111u;
        if (need == 0u)
            return;
        const float *leaf = pan < 4
                                ? tA + leaf_slot(job.slotA, lin_index(I0 + pan, k)) * (B * B)
                                : tBT + leaf_slot(job.slotB, lin_index(k, J0 + (pan - 4))) * (B * B);
        const float *src = leaf + (st & 1u) * P32 + part * (P32 / 2) + 4 * lane;
        float *dst = ring32 + (st & 1u) * kWideStage32 + pan * P32 + part * (P32 / 2);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            __builtin_amdgcn_global_load_lds((global_void_t *)(src + 256 * i),
                                             (lds_void_t *)(dst + 256 * i), 16, 0, 0);
    };
    const uint32_t T = 2 * nhi;
    if (T > 0)
        issue_hi(0);
    for (uint32_t t = 0; t < T; ++t) {
        __builtin_amdgcn_s_waitcnt(0x0F70);             // vmcnt(0)
        __syncthreads();
        if (t + 1 < T)
            issue_hi(t + 1);
        const uint32_t ent = list[t >> 1];
        if ((ent >> (16 + bit)) & 1u) {
            const float *buf = ring32 + (t & 1u) * kWideStage32;
            panel_high<B, X3>(buf + r * P32, buf + (4 + c) * P32, acc, lane);
        }
    }
}

template <bool X3>
__global__ __launch_bounds__(1024) void leaf_gemm_split_wide(const GemmJobs jobs)
{
    constexpr int B = 64, MB = 2;
    constexpr int P16 = Leaf16Layout<B>::kPanel;       // 2048 values: one 16-bit k-panel
    extern __shared__ float smem[];
    uint16_t *ring16 = (uint16_t *)smem;
    uint32_t *kmask = (uint32_t *)((char *)smem + WideShape::kRing);
    uint32_t *list = kmask + kMaxEnt;
    uint32_t *wsum = list + kMaxEnt;
    const GemmJob &job = jobs.job[job_of(jobs, blockIdx.x)];
    const uint32_t P4 = xcd_block<kChunk4>(blockIdx.x - job.block0, job.nblocks);
    const uint32_t I0 = 4 * lin_row(P4), J0 = 4 * lin_col(P4);
    // the wave index in a scalar register: every per-wave decision below
    // (copies, waits, the mask test) is then a scalar branch.  The waves of
    // one SIMD (w mod 4 = s) own the leaves (i, (i + s) mod 4): an entry's
    // mask is close to the outer product of a set of rows and a set of
    // columns, and this Latin square spreads such a product set over the four
    // SIMDs rather than piling a whole column onto one.
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int r = w >> 2, c = (r + (w & 3)) & 3;
    const int bit = 4 * r + c;
    const uint32_t NK = job.nleaf;                     // k ranges over [0, N)
    if (job.skip_empty && job.browptr_lo[4 * P4] == job.browptr_lo[4 * P4 + 4] &&
        job.browptr[4 * P4] == job.browptr[4 * P4 + 4])
        return;                                          // none of the 4 children has products
    const uint16_t *__restrict__ tA16 = (const uint16_t *)job.tA16;
    const uint16_t *__restrict__ tBT16 = (const uint16_t *)job.tBT16;

    floatx16 acc[MB][MB];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < MB; ++j)
            acc[i][j] = floatx16{0};

    // ---- LOW products: whole 16-bit leaves, 2-deep ring ------------------------
    const uint32_t nlo = merge_children(job.browptr_lo, job.bent_lo, P4, NK, kmask, list, wsum);
    // wave w copies rows 32 (w & 1) .. +31 of both k-panels of operand leaf
    // w >> 1 (0..3: A rows, 4..7: B columns): four 1 KB direct-to-LDS copies,
    // or none if no leaf of the entry needs it
    const int pan = w >> 1, part = w & 1;
    auto issue_lo = [&](uint32_t st) {
        const uint32_t ent = list[st], k = ent & 0xFFFFu, m = ent >> 16;
        const uint32_t need = pan < 4 ? (m >> (4 * pan)) & 0xFu : (m >> (pan - 4)) & 0x1111u;
        if (need == 0u)
            return;
        const uint16_t *leaf =
            pan < 4 ? tA16 + leaf_slot(job.slotA, lin_index(I0 + pan, k)) * (B * B)
                    : tBT16 + leaf_slot(job.slotB, lin_index(k, J0 + (pan - 4))) * (B * B);
        uint16_t *dst = ring16 + (st & 1u) * kWideStage16 + pan * (B * B) + part * (P16 / 2);
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int i = 0; i < 2; ++i)
                __builtin_amdgcn_global_load_lds(
                    (global_void_t *)(leaf + p * P16 + part * (P16 / 2) + 512 * i + 8 * lane),
                    (lds_void_t *)(dst + p * P16 + 512 * i), 16, 0, 0);
    };
    if (nlo > 0)
        issue_lo(0);
    const int row = lane & 31, h = lane >> 5;
    for (uint32_t t = 0; t < nlo; ++t) {
        __builtin_amdgcn_s_waitcnt(0x0F70);             // vmcnt(0): this wave's copies of t
        barrier_no_fence();
        // entry t+1 goes to the buffer every wave finished reading at t-1
        if (t + 1 < nlo)
            issue_lo(t + 1);
        const uint32_t ent = list[t];
        if ((ent >> (16 + bit)) & 1u) {
            const uint16_t *buf = ring16 + (t & 1u) * kWideStage16;
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const uint16_t *Ap = buf + r * (B * B) + p * P16;
                const uint16_t *Bp = buf + (4 + c) * (B * B) + p * P16;
                bf16x8 av[2][MB], bv[2][MB];
#pragma unroll
                for (int st = 0; st < 2; ++st) {
                    const int col = 16 * st + 8 * h;
#pragma unroll
                    for (int i = 0; i < MB; ++i)
                        av[st][i] = *reinterpret_cast<const bf16x8 *>(
                            Ap + Leaf16Layout<B>::index(i * 32 + row, col));
#pragma unroll
                    for (int j = 0; j < MB; ++j)
                        bv[st][j] = *reinterpret_cast<const bf16x8 *>(
                            Bp + Leaf16Layout<B>::index(j * 32 + row, col));
                }
#pragma unroll
                for (int st = 0; st < 2; ++st)
#pragma unroll
                    for (int i = 0; i < MB; ++i)
#pragma unroll
                        for (int j = 0; j < MB; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                av[st][i], bv[st][j], acc[i][j], 0, 0, 0);
            }
        }
    }
    __syncthreads();                      // every wave is done with the LOW ring and list

    // ---- HIGH products ------------------------------------------------------------
    wide_fp32_products<X3>(job, P4, I0, J0, NK, w, r, c, bit, lane, smem, kmask, list, wsum, acc);
    write_leaf32<B>(acc, (int64_t)(I0 + r) * B, (int64_t)(J0 + c) * B, job.n, job.C, lane);
}

// FP32 products on 4 x 4 blocks of 64 x 64 leaves (depth >= 2): the FP32
// phase of the wide split kernel alone, so a staged panel feeds up to 4 leaf
// products instead of 2.  Every leaf sums its products over k ascending, one
// k-panel at a time, as in the 2 x 2 kernel: the same bits.
__global__ __launch_bounds__(1024) void leaf_gemm_wide32(const GemmJobs jobs)
{
    constexpr int B = 64, MB = 2;
    extern __shared__ float smem[];
    uint32_t *kmask = (uint32_t *)((char *)smem + WideShape::kRing);
    uint32_t *list = kmask + kMaxEnt;
    uint32_t *wsum = list + kMaxEnt;
    const GemmJob &job = jobs.job[job_of(jobs, blockIdx.x)];
    const uint32_t P4 = xcd_block<kChunk4>(blockIdx.x - job.block0, job.nblocks);
    const uint32_t I0 = 4 * lin_row(P4), J0 = 4 * lin_col(P4);
    // waves of one SIMD own the leaves (i, (i + s) mod 4), as in the split kernel
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int r = w >> 2, c = (r + (w & 3)) & 3;
    if (job.skip_empty && job.browptr[4 * P4] == job.browptr[4 * P4 + 4])
        return;                                          // none of the 4 children has products
    floatx16 acc[MB][MB];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < MB; ++j)
            acc[i][j] = floatx16{0};
    wide_fp32_products(job, P4, I0, J0, job.nleaf, w, r, c, 4 * r + c, lane, smem, kmask, list,
                       wsum, acc);
    write_leaf32<B>(acc, (int64_t)(I0 + r) * B, (int64_t)(J0 + c) * B, job.n, job.C, lane);
}

// Sub-leaf culling on 4 x 4 blocks of 64 x 64 leaves (depth >= 2): the
// sub-products of the 2 x 2 kernel above, staged as in leaf_gemm_wide32.
// First every child entry's kept sub-products are worked out (one byte per
// leaf: bit 2 (2a + b) + c for sub-product (a, c, b)), exported to submask in
// the 2 x 2 layout (one word per child entry) and scattered into a table by
// (k, leaf of the block).  The stages are then the (k, k-panel) pairs some
// leaf needs, in k and panel order; a stage copies only the operand panels
// of the rows and columns whose leaves take it, and wave (r, c) runs, on
// panel c', the accumulators (a, b) of its leaf with sub-product (a, c', b)
// kept.  Each accumulator runs the same MFMAs in the same order as in the
// 2 x 2 kernel: the same C.
struct SubWideShape {
    static constexpr size_t kRing = WideShape::kRing;                        // 2 x 64 KB
    static constexpr size_t kMasks = 16 * (size_t)kMaxEnt;                   // byte per (k, leaf)
    static constexpr size_t kList = sizeof(uint32_t) * 2 * kMaxEnt;          // k << 17 | c << 16 | takers
    static constexpr size_t kLds = kRing + kMasks + kList + sizeof(uint32_t) * kWideWaves;
};

__global__ __launch_bounds__(1024) void leaf_gemm_sub_wide(const GemmJobs jobs)
{
    constexpr int B = 64, MB = 2;
    constexpr int P32 = LeafLayout<B>::kPanel;
    extern __shared__ float smem[];
    float *ring32 = smem;
    uint8_t *subm = (uint8_t *)((char *)smem + SubWideShape::kRing);
    uint32_t *stl = (uint32_t *)((char *)subm + SubWideShape::kMasks);
    uint32_t *wsum = stl + 2 * kMaxEnt;
    const GemmJob &job = jobs.job[job_of(jobs, blockIdx.x)];
    const uint32_t P4 = xcd_block<kChunk4>(blockIdx.x - job.block0, job.nblocks);
    const uint32_t I0 = 4 * lin_row(P4), J0 = 4 * lin_col(P4);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int r = w >> 2, c = (r + (w & 3)) & 3;
    const int bit = 4 * r + c;
    const uint32_t NK = job.nleaf;
    const uint32_t *__restrict__ rp = job.browptr;
    const uint32_t *__restrict__ bent = job.bent;
    const uint32_t ea = rp[4 * P4], eb = rp[4 * P4 + 4];
    if (job.skip_empty && ea == eb)
        return;

    // ---- kept sub-products of every child entry ----------------------------
    for (uint32_t i = threadIdx.x; i < NK; i += blockDim.x)
        reinterpret_cast<uint4 *>(subm)[i] = make_uint4(0u, 0u, 0u, 0u);
    __syncthreads();
    uint32_t subs = 0;
    const uint32_t b1 = rp[4 * P4 + 1], b2 = rp[4 * P4 + 2], b3 = rp[4 * P4 + 3];
    for (uint32_t e = ea + threadIdx.x; e < eb; e += blockDim.x) {
        const uint32_t ch = (e >= b1 ? 1u : 0u) + (e >= b2 ? 1u : 0u) + (e >= b3 ? 1u : 0u);
        const uint32_t ca = ch >> 1, cb = ch & 1u;          // child rows 2 ca.., columns 2 cb..
        const uint32_t ent = bent[e], k = ent & 0xFFFFu;
        uint32_t word = 0;
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
            if (!((ent >> (16 + q)) & 1u))
                continue;
            const uint32_t lr = 2 * ca + (q >> 1), lc = 2 * cb + (q & 1u);
            const double *sa = job.subA + 4 * (int64_t)lin_index(I0 + lr, k);
            const double *sb = job.subB + 4 * (int64_t)lin_index(k, J0 + lc);
            uint32_t m = 0;
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int cc = 0; cc < 2; ++cc)
                        m |= keep_pair(sa[2 * a + cc], sb[2 * cc + b], job.T2)
                                 ? 1u << (2 * (2 * a + b) + cc) : 0u;
            subm[16 * k + 4 * lr + lc] = (uint8_t)m;
            word |= m << (8 * q);
            subs += __builtin_popcount(m);
        }
        *reinterpret_cast<uint32_t *>(job.submask + 4 * (int64_t)e) = word;
    }
    for (int o = 32; o > 0; o >>= 1)
        subs += __shfl_xor(subs, o);
    if (lane == 0 && subs != 0)
        atomicAdd(job.subK, (unsigned long long)subs);
    __syncthreads();

    // ---- the stages: (k, panel) pairs some leaf takes, in order ---------------
    // takers: bit 4 r' + c' when leaf (r', c') keeps a sub-product on the panel
    uint32_t T = 0;
    for (uint32_t r0 = 0; r0 < 2 * NK; r0 += blockDim.x) {
        const uint32_t idx = r0 + threadIdx.x;
        uint32_t tk = 0;
        if (idx < 2 * NK) {
            const uint32_t k = idx >> 1, cp = idx & 1u;
            const uint4 v = reinterpret_cast<const uint4 *>(subm)[k];
            const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int j = 0; j < 16; ++j)
                tk |= (((wv[j >> 2] >> (8 * (j & 3))) & (0x55u << cp)) != 0u ? 1u : 0u) << j;
        }
        const uint64_t bal = __ballot(tk != 0u);
        if (lane == 0)
            wsum[w] = (uint32_t)__popcll(bal);
        __syncthreads();
        uint32_t before = 0, total = 0;
        for (int i = 0; i < kWideWaves; ++i) {
            const uint32_t x = wsum[i];
            before += i < w ? x : 0u;
            total += x;
        }
        if (tk != 0u)
            stl[T + before + (uint32_t)__popcll(bal & lanes_below())] = (idx << 16) | tk;
        T += total;
        __syncthreads();                       // wsum is rewritten by the next pass
    }

    // ---- staged sub-products: FP32 k-panels, 64 KB stages, 2-deep ring ---------
    const float *__restrict__ tA = (const float *)job.tA;
    const float *__restrict__ tBT = (const float *)job.tBT;
    const int pan = w >> 1, part = w & 1;
    auto issue = [&](uint32_t st) {
        const uint32_t x = stl[st], k = x >> 17, cp = (x >> 16) & 1u, tk = x & 0xFFFFu;
        const uint32_t need = pan < 4 ? (tk >> (4 * pan)) & 0xFu : (tk >> (pan - 4)) & 0x1111u;
        if (need == 0u)
            return;
        const float *leaf = pan < 4
                                ? tA + leaf_slot(job.slotA, lin_index(I0 + pan, k)) * (B * B)
                                : tBT + leaf_slot(job.slotB, lin_index(k, J0 + (pan - 4))) * (B * B);
        const float *src = leaf + cp * P32 + part * (P32 / 2) + 4 * lane;
        float *dst = ring32 + (st & 1u) * kWideStage32 + pan * P32 + part * (P32 / 2);
#pragma unroll
        for (int i = 0; i < 4; ++i)
            __builtin_amdgcn_global_load_lds((global_void_t *)(src + 256 * i),
                                             (lds_void_t *)(dst + 256 * i), 16, 0, 0);
    };
    floatx16 acc[MB][MB];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < MB; ++j)
            acc[i][j] = floatx16{0};
    if (T > 0)
        issue(0);
    for (uint32_t t = 0; t < T; ++t) {
        __builtin_amdgcn_s_waitcnt(0x0F70);             // vmcnt(0)
        __syncthreads();
        if (t + 1 < T)
            issue(t + 1);
        const uint32_t x = stl[t], k = x >> 17, cp = (x >> 16) & 1u;
        const uint32_t sm = subm[16 * k + bit];
        // accumulator (a, b) on panel cp: sub-product bit 2 (2a + b) + cp
        const uint32_t pm = ((sm >> cp) & 1u) | ((sm >> (1 + cp)) & 2u) |
                            ((sm >> (2 + cp)) & 4u) | ((sm >> (3 + cp)) & 8u);
        if (pm != 0u) {
            const float *buf = ring32 + (t & 1u) * kWideStage32;
            panel_mfma32_sub<B>(buf + r * P32, buf + (4 + c) * P32, acc, lane, pm);
        }
    }
    write_leaf32<B>(acc, (int64_t)(I0 + r) * B, (int64_t)(J0 + c) * B, job.n, job.C, lane);
}

static hipError_t launch_sub_wide(const GemmJobs &jobs, hipStream_t s)
{
    constexpr size_t lds = SubWideShape::kLds;
    static const hipError_t attr =
        hipFuncSetAttribute((const void *)leaf_gemm_sub_wide,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess)
        return attr;
    hipLaunchKernelGGL(leaf_gemm_sub_wide, dim3(jobs.nblocks), dim3(64 * kWideWaves), lds, s,
                       jobs);
    return hipGetLastError();
}

static hipError_t launch_wide32(const GemmJobs &jobs, hipStream_t s)
{
    constexpr size_t lds = WideShape::kLds;
    static const hipError_t attr =
        hipFuncSetAttribute((const void *)leaf_gemm_wide32,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess)
        return attr;
    hipLaunchKernelGGL(leaf_gemm_wide32, dim3(jobs.nblocks), dim3(64 * kWideWaves), lds, s, jobs);
    return hipGetLastError();
}

// jobs.block0 / nblocks count 4 x 4 blocks here
template <bool X3>
static hipError_t launch_split_wide(const GemmJobs &jobs, hipStream_t s)
{
    constexpr size_t lds = WideShape::kLds;
    static const hipError_t attr =
        hipFuncSetAttribute((const void *)leaf_gemm_split_wide<X3>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess)
        return attr;
    hipLaunchKernelGGL(leaf_gemm_split_wide<X3>, dim3(jobs.nblocks), dim3(64 * kWideWaves), lds,
                       s, jobs);
    return hipGetLastError();
}

template <int B>
static hipError_t launch_fp32(const GemmJobs &jobs, hipStream_t s)
{
    using S = GemmShape<B>;
    // once per process (thread-safe static initialization)
    static const hipError_t attr =
        hipFuncSetAttribute((const void *)leaf_gemm<B>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)S::kLds);
    if (attr != hipSuccess)
        return attr;
    hipLaunchKernelGGL((leaf_gemm<B>), dim3(jobs.nblocks), dim3(256), S::kLds, s, jobs);
    return hipGetLastError();
}

static hipError_t launch_sub(const GemmJobs &jobs, hipStream_t s)
{
    constexpr size_t lds = SubShape<64>::kLds;
    static const hipError_t attr =
        hipFuncSetAttribute((const void *)leaf_gemm_sub<64>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess)
        return attr;
    hipLaunchKernelGGL((leaf_gemm_sub<64>), dim3(jobs.nblocks), dim3(256), lds, s, jobs);
    return hipGetLastError();
}

template <int B, bool F16, bool X3 = false>
static hipError_t launch_split(const GemmJobs &jobs, hipStream_t s)
{
    constexpr size_t lds = SplitShape<B, F16>::kLds;
    static const hipError_t attr =
        hipFuncSetAttribute((const void *)leaf_gemm_split<B, F16, X3>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess)
        return attr;
    hipLaunchKernelGGL((leaf_gemm_split<B, F16, X3>), dim3(jobs.nblocks), dim3(256), lds, s,
                       jobs);
    return hipGetLastError();
}

// One batched launch over the jobs' blocks; all jobs share the leaf size and
// the kind.
hipError_t launch_gemm_jobs(int leaf, GemmKind kind, const GemmJobs &jobs, hipStream_t s)
{
    if (jobs.njobs <= 0 || jobs.nblocks == 0)
        return hipSuccess;
    switch (kind) {
    case GemmKind::Sub:
        return leaf == 64 ? launch_sub(jobs, s) : hipErrorInvalidValue;
    case GemmKind::SplitWide:
        return leaf == 64 ? launch_split_wide<false>(jobs, s) : hipErrorInvalidValue;
    case GemmKind::SplitWideX3:
        return leaf == 64 ? launch_split_wide<true>(jobs, s) : hipErrorInvalidValue;
    case GemmKind::SplitX3:
        switch (leaf) {
        case 32: return launch_split<32, false, true>(jobs, s);
        case 64: return launch_split<64, false, true>(jobs, s);
        default: return hipErrorInvalidValue;
        }
    case GemmKind::Wide32:
        return leaf == 64 ? launch_wide32(jobs, s) : hipErrorInvalidValue;
    case GemmKind::SubWide:
        return leaf == 64 ? launch_sub_wide(jobs, s) : hipErrorInvalidValue;
    case GemmKind::Split:
        switch (leaf) {
        case 32: return launch_split<32, false>(jobs, s);
        case 64: return launch_split<64, false>(jobs, s);
        default: return hipErrorInvalidValue;
        }
    case GemmKind::SplitF16:
        switch (leaf) {
        case 32: return launch_split<32, true>(jobs, s);
        case 64: return launch_split<64, true>(jobs, s);
        default: return hipErrorInvalidValue;
        }
    case GemmKind::Fp32:
        switch (leaf) {
        case 16: return launch_fp32<16>(jobs, s);
        case 32: return launch_fp32<32>(jobs, s);
        case 64: return launch_fp32<64>(jobs, s);
        default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

GemmKind plan_kind(const spamm_plan *p)
{
    // sub-leaf culling at 64 x 64 leaves: 4 x 4 blocks from depth 2 (258.5
    // against 279.0 ms for 2 x 2 at n = 32768, tau = 1e-8, the same C)
    if (p->sub)
        return p->depth >= 2 ? GemmKind::SubWide : GemmKind::Sub;
    if (p->precision == SPAMM_PREC_SPLIT_BF16 && p->leaf == 64 && p->depth >= 2)
        return GemmKind::SplitWide;
    if (p->precision == SPAMM_PREC_SPLIT_BF16X3)
        return p->leaf == 64 && p->depth >= 2 ? GemmKind::SplitWideX3 : GemmKind::SplitX3;
    // FP32 at 64 x 64 leaves: 4 x 4 blocks (313.6 against 330.6 ms for 2 x 2
    // at n = 32768, tau = 1e-8, bit-identical C, with the unrotated XCD
    // mapping)
    if (p->precision == SPAMM_PREC_FP32 && p->leaf == 64 && p->depth >= 2)
        return GemmKind::Wide32;
    return p->precision == SPAMM_PREC_SPLIT_FP16   ? GemmKind::SplitF16
           : p->precision == SPAMM_PREC_SPLIT_BF16 ? GemmKind::Split
                                                   : GemmKind::Fp32;
}

// The plan's job: FP32 copies and HIGH (or only) schedule; with split
// precision also the 16-bit copies and the LOW schedule.
void plan_jobs(const spamm_plan *p, float *C, GemmJob &j)
{
    const bool split = p->precision != SPAMM_PREC_FP32;
    j.tA = p->A->tiles;
    j.tBT = p->B->tilesT;
    j.browptr = p->browptr;
    j.bent = p->bent;
    j.C = C;
    j.n = p->n;
    j.nleaf = 1u << p->depth;
    // the wide kernels' workgroups own 4 x 4 output leaves
    const GemmKind kind = plan_kind(p);
    j.nblocks = (uint32_t)p->nblocks / (kind == GemmKind::SplitWide || kind == GemmKind::Wide32 ||
                                                kind == GemmKind::SubWide ||
                                                kind == GemmKind::SplitWideX3
                                            ? 4u
                                            : 1u);
    j.block0 = 0;
    j.single = p->depth == 0 ? 1 : 0;
    j.skip_empty = 0;
    j.tA16 = split ? (const void *)p->A->tiles16 : nullptr;
    j.tBT16 = split ? (const void *)p->B->tilesT16 : nullptr;
    j.browptr_lo = split ? p->browptr_lo : nullptr;
    j.bent_lo = split ? p->bent_lo : nullptr;
    j.subA = j.subB = nullptr;
    j.submask = nullptr;
    j.subK = nullptr;
    j.T2 = p->T2;
    j.slotA = p->A->slot;
    j.slotB = p->B->slot;
    j.escA = p->precision == SPAMM_PREC_SPLIT_FP16 ? p->A->scale16 : nullptr;
    j.escB = p->precision == SPAMM_PREC_SPLIT_FP16 ? p->B->scale16 : nullptr;
    if (p->sub) {
        j.subA = p->A->norms + tier_offset(p->depth + 1);
        j.subB = p->B->norms + tier_offset(p->depth + 1);
        j.submask = p->submask;
        j.subK = (unsigned long long *)(p->leafK + 2);
    }
}

// Clears one counter (a kernel rather than a memset node, so the launch
// sequence stays valid under stream capture).
__global__ void zero_counter(unsigned long long *c) { *c = 0ull; }

hipError_t launch_gemm(const spamm_plan *p, float *C, hipStream_t s)
{
    GemmJobs jobs{};
    jobs.njobs = 1;
    if (p->sub) {
        hipLaunchKernelGGL(zero_counter, dim3(1), dim3(1), 0, s,
                           (unsigned long long *)(p->leafK + 2));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    plan_jobs(p, C, jobs.job[0]);
    jobs.nblocks = jobs.job[0].nblocks;
    return launch_gemm_jobs(p->leaf, plan_kind(p), jobs, s);
}

}  // namespace spamm
