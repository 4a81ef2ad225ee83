// Numeric multiply: C_ij = sum over kept k (ascending) of A_ik B_kj
// (Eq. product, Alg. 1 steps 7-9) on FP32 MFMA with FP32 accumulation.
//
// A workgroup of 4 waves owns one block of 2 x 2 output leaves (the children
// of one tier-(d-1) tile); wave q = 2a + b owns leaf (2I+a, 2J+b) and is the
// only writer of it, so no atomics touch C.  The block walks the union of its
// leaves' kept k (entries k | mask << 16 from the cull): it stages the needed
// A_(2I+a, k) and B_(k, 2J+b) leaves in LDS once and every wave whose mask
// bit is set runs its leaf product from there.  Every output leaf is written
// once, with zeros where nothing was kept, cropped to n.
//
// MFMA layouts (v_mfma_f32_32x32x2_f32): A operand lane l = A[l%32][l/32],
// B operand lane l = B[l/32][l%32]; result register v of lane l is
// D[8(v/4) + 4(l/32) + v%4][l%32].  16x16x4: A[l%16][l/16], B[l/16][l%16],
// D[4(l/16) + v][l%16].  The A leaves sit in LDS with a row pitch of n_b + 1
// floats so that the 32 rows read by one MFMA operand fall in distinct banks.
#include "common.hpp"

namespace spamm {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

template <int B>
struct GemmShape {
    static constexpr int kPitchA = B + 1;
    static constexpr int kTileA = B * kPitchA;
    static constexpr int kTileB = B * B;
    static constexpr size_t kLds = sizeof(float) * 2 * (kTileA + kTileB);
};

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of blocks (linear-index order) so its L2 sees neighbours.
__device__ inline uint32_t xcd_block(uint32_t bid, uint32_t nblocks)
{
    if (nblocks % 8u != 0u)
        return bid;
    return (bid % 8u) * (nblocks / 8u) + bid / 8u;
}

// One entry's operand leaves in registers: A_(2I, k), A_(2I+1, k),
// B_(k, 2J), B_(k, 2J+1); thread t holds float4 number t + 256 i of each leaf.
template <int B>
struct Stage {
    static constexpr int kVec = B * B / 4;                   // float4 per leaf
    static constexpr int kPer = kVec >= 256 ? kVec / 256 : 1;
    float4 v[4][kPer];
};

template <int B>
__device__ inline void stage_load(Stage<B> &st, uint32_t ent, const float *__restrict__ tA,
                                  const float *__restrict__ tB, uint32_t I0, uint32_t J0)
{
    using S = Stage<B>;
    const uint32_t k = ent & 0xFFFFu, mask = ent >> 16;
    const bool need[4] = {(mask & 0x3u) != 0, (mask & 0xCu) != 0, (mask & 0x5u) != 0,
                          (mask & 0xAu) != 0};
    const float4 *src[4] = {
        reinterpret_cast<const float4 *>(tA + (int64_t)lin_index(I0, k) * (B * B)),
        reinterpret_cast<const float4 *>(tA + (int64_t)lin_index(I0 + 1, k) * (B * B)),
        reinterpret_cast<const float4 *>(tB + (int64_t)lin_index(k, J0) * (B * B)),
        reinterpret_cast<const float4 *>(tB + (int64_t)lin_index(k, J0 + 1) * (B * B))};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (!need[t])
            continue;
#pragma unroll
        for (int i = 0; i < S::kPer; ++i) {
            const int f = threadIdx.x + 256 * i;
            if (S::kVec >= 256 || f < S::kVec)
                st.v[t][i] = src[t][f];
        }
    }
}

template <int B>
__device__ inline void stage_store(const Stage<B> &st, uint32_t ent, float *__restrict__ As,
                                   float *__restrict__ Bs)
{
    using S = Stage<B>;
    using G = GemmShape<B>;
    const uint32_t mask = ent >> 16;
    const bool need[4] = {(mask & 0x3u) != 0, (mask & 0xCu) != 0, (mask & 0x5u) != 0,
                          (mask & 0xAu) != 0};
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        if (!need[t])
            continue;
        float *dst = As + t * G::kTileA;
#pragma unroll
        for (int i = 0; i < S::kPer; ++i) {
            const int f = threadIdx.x + 256 * i;
            if (S::kVec >= 256 || f < S::kVec) {
                const int r = (4 * f) / B, c = (4 * f) % B;
                float *o = dst + r * G::kPitchA + c;
                o[0] = st.v[t][i].x;
                o[1] = st.v[t][i].y;
                o[2] = st.v[t][i].z;
                o[3] = st.v[t][i].w;
            }
        }
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        if (!need[2 + t])
            continue;
        float4 *dst = reinterpret_cast<float4 *>(Bs + t * G::kTileB);
#pragma unroll
        for (int i = 0; i < S::kPer; ++i) {
            const int f = threadIdx.x + 256 * i;
            if (S::kVec >= 256 || f < S::kVec)
                dst[f] = st.v[2 + t][i];
        }
    }
}

template <int B>
__global__ __launch_bounds__(256) void leaf_gemm(const float *__restrict__ tA,
                                                 const float *__restrict__ tB,
                                                 const uint32_t *__restrict__ browptr,
                                                 const uint32_t *__restrict__ bent,
                                                 uint32_t nblocks, int single, int64_t n,
                                                 float *__restrict__ C)
{
    using S = GemmShape<B>;
    extern __shared__ float smem[];
    float *As = smem;                    // 2 leaves, pitch B+1
    float *Bs = smem + 2 * S::kTileA;    // 2 leaves, pitch B
    const uint32_t blk = xcd_block(blockIdx.x, nblocks);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int qa = w >> 1, qb = w & 1;
    uint32_t I0 = 0, J0 = 0;
    if (!single) {
        I0 = 2 * lin_row(blk);
        J0 = 2 * lin_col(blk);
    }
    const float *Am = As + qa * S::kTileA;
    const float *Bm = Bs + qb * S::kTileB;

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

    // Register double buffering: the leaves of entry e+1 are in flight from
    // memory while entry e is multiplied out of LDS.
    const uint32_t e0 = browptr[blk], e1 = browptr[blk + 1];
    Stage<B> st;
    uint32_t ent = 0;
    if (e0 < e1) {
        ent = bent[e0];
        stage_load<B>(st, ent, tA, tB, I0, J0);
    }
    for (uint32_t e = e0; e < e1; ++e) {
        __syncthreads();                 // every wave is done with the previous entry
        stage_store<B>(st, ent, As, Bs);
        __syncthreads();
        const uint32_t mask = ent >> 16;
        if (e + 1 < e1) {
            ent = bent[e + 1];
            stage_load<B>(st, ent, tA, tB, I0, J0);
        }
        if ((mask >> w) & 1u) {
            if constexpr (B >= 32) {
                const int r = lane & 31, h = lane >> 5;
#pragma unroll 4
                for (int kk = 0; kk < B; kk += 2) {
                    float av[MB], bv[MB];
#pragma unroll
                    for (int i = 0; i < MB; ++i)
                        av[i] = Am[(i * 32 + r) * S::kPitchA + kk + h];
#pragma unroll
                    for (int j = 0; j < MB; ++j)
                        bv[j] = Bm[(kk + h) * B + j * 32 + r];
#pragma unroll
                    for (int i = 0; i < MB; ++i)
#pragma unroll
                        for (int j = 0; j < MB; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv[j], acc[i][j],
                                                                             0, 0, 0);
                }
            } else {
                const int r = lane & 15, h = lane >> 4;
#pragma unroll
                for (int kk = 0; kk < B; kk += 4) {
                    const float av = Am[r * S::kPitchA + kk + h];
                    const float bv = Bm[(kk + h) * B + r];
                    acc16 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc16, 0, 0, 0);
                }
            }
        }
    }

    if (single && w != 0)
        return;
    const int64_t row0 = (int64_t)(I0 + qa) * B, col0 = (int64_t)(J0 + qb) * B;
    if constexpr (B >= 32) {
#pragma unroll
        for (int i = 0; i < MB; ++i)
#pragma unroll
            for (int j = 0; j < MB; ++j)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int64_t row = row0 + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                    const int64_t col = col0 + j * 32 + (lane & 31);
                    if (row < n && col < n)
                        C[row * n + col] = acc[i][j][v];
                }
    } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t row = row0 + 4 * (lane >> 4) + v;
            const int64_t col = col0 + (lane & 15);
            if (row < n && col < n)
                C[row * n + col] = acc16[v];
        }
    }
}

template <int B>
static hipError_t launch_gemm_b(const spamm_plan *p, float *C, hipStream_t s)
{
    using S = GemmShape<B>;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)leaf_gemm<B>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)S::kLds);
        if (e != hipSuccess)
            return e;
        attr_set = true;
    }
    hipLaunchKernelGGL(leaf_gemm<B>, dim3((uint32_t)p->nblocks), dim3(256), S::kLds, s,
                       p->A->tiles, p->B->tiles, p->browptr, p->bent, (uint32_t)p->nblocks,
                       p->depth == 0 ? 1 : 0, p->n, C);
    return hipGetLastError();
}

hipError_t launch_gemm(const spamm_plan *p, float *C, hipStream_t s)
{
    switch (p->leaf) {
    case 16: return launch_gemm_b<16>(p, C, s);
    case 32: return launch_gemm_b<32>(p, C, s);
    case 64: return launch_gemm_b<64>(p, C, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace spamm
