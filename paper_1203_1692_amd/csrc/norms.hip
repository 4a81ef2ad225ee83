// Quadtree construction (Sec. II.A, II.B): pack the zero-padded leaves and
// build the FP64 squared-Frobenius-norm pyramid bottom-up (Eq. norm).
//
// Canonical order (the cull decisions depend on every bit of these values):
//   leaf   s = pairwise (recursive-halving) sum of x_e^2 over the leaf's
//          row-major flattened index e in [0, b^2);
//   parent s = (s_11 + s_12) + (s_21 + s_22).
// A wave owns one leaf.  Load m of lane L covers e = 256 m + 4 L + x
// (x = 0..3, one float4): the tree over e is then the in-lane pair sums
// (bits 0-1 of e), a six-step xor butterfly over lanes (bits 2-7) and an
// in-register tree over m (bits 8 and up).  Squares of FP32 values are exact
// in FP64, so only the additions round and their order is fixed.
#include <algorithm>
#include <vector>

#include "runtime.hpp"

namespace spamm {

template <int VEC>
__device__ inline float4 load_row4(const float *__restrict__ A, int64_t n, int64_t row,
                                   int64_t col)
{
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (row >= n || col >= n)
        return v;
    const float *p = A + row * n + col;
    if (col + 3 < n) {
        if constexpr (VEC == 4) {
            v = *reinterpret_cast<const float4 *>(p);
        } else if constexpr (VEC == 2) {
            const float2 a = reinterpret_cast<const float2 *>(p)[0];
            const float2 b = reinterpret_cast<const float2 *>(p)[1];
            v = make_float4(a.x, a.y, b.x, b.y);
        } else {
            v = make_float4(p[0], p[1], p[2], p[3]);
        }
    } else {
        v.x = p[0];
        if (col + 1 < n) v.y = p[1];
        if (col + 2 < n) v.z = p[2];
    }
    return v;
}

// Four consecutive elements of a row, rounded to BF16 (8 bytes, aligned).
__device__ inline uint2 pack_bf16x4(float4 v)
{
    return make_uint2((uint32_t)to_bf16(v.x) | ((uint32_t)to_bf16(v.y) << 16),
                      (uint32_t)to_bf16(v.z) | ((uint32_t)to_bf16(v.w) << 16));
}

__device__ inline void store_bf16x4(uint16_t *dst, float4 v)
{
    *reinterpret_cast<uint2 *>(dst) = pack_bf16x4(v);
}

// ---- FP16 leaf copies (split precision with FP16 LOW operands) ---------------
// Leaf l is multiplied by 2^e before rounding, e fixed by its squared norm S
// alone: with S = f 2^E (1 <= f < 2), 4^(13-e) <= S < 4^(14-e) for
// e = 14 - floor((E + 2) / 2), so every entry (|x| <= sqrt(S)) is below 2^14
// once scaled.  A zero leaf (never multiplied) gets e = 0.
__device__ inline int fp16_scale_exponent(double S)
{
    if (!(S > 0.0))
        return 0;
    const int E = (int)((__double_as_longlong(S) >> 52) & 0x7FF) - 1023;   // S >= 2^-298: normal
    return 14 - ((E + 2) >> 1);
}

// x 2^e (|x 2^e| < 2^14) rounded to binary16, nearest with ties to even; a
// result below the normal range (2^-14) is flushed to zero, because the
// matrix units' products of binary16 subnormals are not exact.  Bit pattern,
// from integer rounding on the FP32 bits.
__device__ inline uint16_t to_fp16_scaled(float x, int e)
{
    const uint32_t u = __float_as_uint(ldexpf(x, e));    // exact: a power-of-two scaling up
    const uint32_t sign = (u >> 16) & 0x8000u, mag = u & 0x7FFFFFFFu;
    const int ef = (int)(mag >> 23);                      // biased FP32 exponent
    if (ef >= 113) {                                      // >= 2^-14: normal binary16
        const uint32_t frac = mag & 0x7FFFFFu, keep = frac >> 13, rest = frac & 0x1FFFu;
        uint32_t h = ((uint32_t)(ef - 112) << 10) | keep;
        if (rest > 0x1000u || (rest == 0x1000u && (keep & 1u)))
            h += 1u;                                      // a carry moves to the next binade
        return (uint16_t)(sign | h);
    }
    if (ef < 112)                                         // below 2^-15: never reaches 2^-14
        return 0;
    // [2^-15, 2^-14): in units of 2^-24, sig 2^(ef - 126) with sig the 24-bit
    // significand; it stays only if it rounds up to 1024 (= 2^-14, normal)
    const uint32_t sig = (mag & 0x7FFFFFu) | 0x800000u;
    uint32_t q = sig >> 14;
    const uint32_t rest = sig & 0x3FFFu;
    if (rest > 0x2000u || (rest == 0x2000u && (q & 1u)))
        q += 1u;
    return q == 1024u ? (uint16_t)(sign | 0x400u) : (uint16_t)0;
}

// Four consecutive elements x 2^e, rounded to binary16 (8 bytes, aligned).
__device__ inline uint2 pack_fp16x4(float4 v, int e)
{
    return make_uint2((uint32_t)to_fp16_scaled(v.x, e) | ((uint32_t)to_fp16_scaled(v.y, e) << 16),
                      (uint32_t)to_fp16_scaled(v.z, e) | ((uint32_t)to_fp16_scaled(v.w, e) << 16));
}

__device__ inline void store_fp16x4(uint16_t *dst, float4 v, int e)
{
    *reinterpret_cast<uint2 *>(dst) = pack_fp16x4(v, e);
}

// Block of 4 waves = the 4 children of one tier-(d-1) node (linear indices
// 4p .. 4p+3); the block also writes that parent's norm when `parent` != null.
// Each leaf is stored twice in LeafLayout: as is (left-operand copy) and
// transposed through LDS (right-operand copy), so that the GEMM reads both of
// its operands along k with contiguous 16-byte loads.  With tiles16 the two
// 16-bit copies follow in Leaf16Layout: BF16 from the loads, or, with
// scale16, FP16 at the leaf's scale, which needs the leaf's norm and so is
// written from the LDS copy after the norm is known (with its exponent).
//
// SUB (n_b = 64, sub-leaf culling): the norms are those of a tree with 32 x 32
// leaves one tier deeper.  Sub-block (a, b) (rows 32a.., columns 32b..) is
// summed pairwise over its own row-major flattened index f = 32 r' + c'; in
// the load pattern above its bits are f0-1 = in-lane, f2-4 = lane bits 0-2,
// f5-6 = lane bits 4-5, f7-9 = m bits 0-2, while lane bit 3 is b and m bit 3
// is a.  So the butterfly skips lane bit 3, the register tree stops below m
// bit 3, and the leaf norm is the parent of its four sub-blocks:
// (s_00 + s_01) + (s_10 + s_11), written to sub_norm[4 l + 2a + b].
// The body of one workgroup (block `bid` of the leaves' grid).  SKIP: leaves
// may be known zero (keep flags) or dropped (drop_s); without it neither test
// is compiled in (the dense build keeps its register budget).
template <int B, int VEC, bool SUB, bool TWO, bool SKIP>
__device__ inline void norm_pack_block(const float *__restrict__ A, int64_t n,
                                       float *__restrict__ tiles, float *__restrict__ tilesT,
                                       uint16_t *__restrict__ tiles16,
                                       uint16_t *__restrict__ tilesT16,
                                       double *__restrict__ leaf_norm,
                                       double *__restrict__ parent,
                                       double *__restrict__ sub_norm,
                                       const uint32_t *__restrict__ keep,
                                       const uint32_t *__restrict__ slot,
                                       int32_t *__restrict__ scale16, uint32_t ntiles,
                                       int known_zero, uint32_t bid,
                                       const double *__restrict__ drop_s = nullptr,
                                       const double *__restrict__ rootA = nullptr,
                                       const double *__restrict__ rootB = nullptr,
                                       double T2 = 0.0)
{
    static_assert(!SUB || B == 64, "sub-block norms are built for 64 x 64 leaves");
    using L = LeafLayout<B>;
    constexpr int M = (B * B) / 256;   // float4 loads per lane
    constexpr int P = B + 1;           // LDS pitch of the transpose buffer
    static_assert(M >= 1 && (M & (M - 1)) == 0, "leaf must be 16, 32 or 64");
    // TWO (64 x 64 leaves): the transpose runs in two halves of 32 source
    // rows (one k-panel of the transposed copy each, FP32 and 16-bit alike),
    // which halves the LDS and lets more workgroups share a CU.
    static_assert(!TWO || B == 64, "two-pass transpose for 64 x 64 leaves");
    constexpr int NPASS = TWO ? 2 : 1;
    constexpr int RH = B / NPASS, MH = M / NPASS;
    extern __shared__ float tr_smem[];
    __shared__ double part[4];
    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const uint32_t l = bid * 4u + (uint32_t)w;
    const bool valid = l < ntiles;
    float *tr = tr_smem + w * (RH * P);
    double s = 0.0;
    // pack this leaf?  (tiles null: norms only; keep/slot: a sparsified tree
    // stores only its kept leaves, leaf l at slot[l].  known_zero: a leaf
    // that is not kept is known to be all zeros, so it is not read and its
    // norm is +0, the value the pairwise sum of its squares gives.)
    // drop_s (a pack after the norms are built): a leaf whose squared norm s
    // passes no product test against a leaf of norm at most the larger root
    // (s = 0, or fl64(s m) < T2 with m = max(rootA, rootB)) can never be read,
    // so it is not packed (Sec. II.C)
    bool zero = false;
    if constexpr (SKIP) {
        const bool dropped =
            valid && drop_s != nullptr &&
            !(drop_s[l] > 0.0 && !(drop_s[l] * fmax(rootA[0], rootB[0]) < T2));
        zero = valid && ((known_zero && keep[l] == 0u) || dropped);
    }
    const bool pack = valid && tiles != nullptr && (keep == nullptr || keep[l] != 0u);
    const int64_t dl = pack && slot != nullptr ? (int64_t)slot[l] : (int64_t)l;
    float4 v[M];
    if constexpr (SKIP) {
        // defined on every path (a skipped leaf is never stored)
#pragma unroll
        for (int m = 0; m < M; ++m)
            v[m] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    if (zero && lane == 0 && scale16 != nullptr)
        scale16[l] = 0;                   // the exponent of a zero leaf
    if (zero && lane == 0 && leaf_norm != nullptr) {
        leaf_norm[l] = 0.0;
        if constexpr (SUB) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                sub_norm[4 * (int64_t)l + i] = 0.0;
        }
    }
    if (valid && !zero) {
        const int64_t I = lin_row(l), J = lin_col(l);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int e = 256 * m + 4 * lane;
            v[m] = load_row4<VEC>(A, n, I * B + e / B, J * B + e % B);
        }
        double sm[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int e = 256 * m + 4 * lane;
            const int r = e / B, c = e % B;
            if (pack) {
                *reinterpret_cast<float4 *>(tiles + dl * (B * B) + L::index(r, c)) = v[m];
                if constexpr (B >= 32) {
                    if (tiles16 != nullptr && scale16 == nullptr)
                        store_bf16x4(tiles16 + dl * (B * B) + Leaf16Layout<B>::index(r, c), v[m]);
                }
            }
            const double x0 = v[m].x, x1 = v[m].y, x2 = v[m].z, x3 = v[m].w;
            double t = (x0 * x0 + x1 * x1) + (x2 * x2 + x3 * x3);
#pragma unroll
            for (int o2 = 1; o2 < 64; o2 <<= 1)
                if (!SUB || o2 != 8)
                    t += __shfl_xor(t, o2);
            sm[m] = t;
        }
        if constexpr (SUB) {
#pragma unroll
            for (int st = 1; st < M / 2; st <<= 1)
#pragma unroll
                for (int i = 0; i < M; i += 2 * st)
                    sm[i] += sm[i + st];
            // sm[0]: sub-row a = 0, sm[M/2]: a = 1, for this lane's sub-column
            const double o0 = __shfl_xor(sm[0], 8), o1 = __shfl_xor(sm[M / 2], 8);
            const bool right = (lane >> 3) & 1;
            const double s00 = right ? o0 : sm[0], s01 = right ? sm[0] : o0;
            const double s10 = right ? o1 : sm[M / 2], s11 = right ? sm[M / 2] : o1;
            s = (s00 + s01) + (s10 + s11);
            if (lane == 0 && leaf_norm != nullptr) {
                double *sn = sub_norm + 4 * (int64_t)l;
                sn[0] = s00;
                sn[1] = s01;
                sn[2] = s10;
                sn[3] = s11;
                leaf_norm[l] = s;
            }
        } else {
#pragma unroll
            for (int st = 1; st < M; st <<= 1)
#pragma unroll
                for (int i = 0; i < M; i += 2 * st)
                    sm[i] += sm[i + st];
            s = sm[0];
            if (lane == 0 && leaf_norm != nullptr)
                leaf_norm[l] = s;
        }
    }
    // FP16: the leaf's scale exponent from its norm (s is the same in every
    // lane of the wave); the as-is copy straight from the loaded values
    const int e16 = pack && scale16 != nullptr ? fp16_scale_exponent(s) : 0;
    if (pack && scale16 != nullptr && lane == 0)
        scale16[l] = e16;                 // by linear index, also in a sparse tree
    if constexpr (B >= 32) {
        if (pack && scale16 != nullptr && tiles16 != nullptr) {
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const int e = 256 * m + 4 * lane;
                store_fp16x4(tiles16 + dl * (B * B) + Leaf16Layout<B>::index(e / B, e % B), v[m],
                             e16);
            }
        }
    }
    // transposed copies through LDS, RH source rows at a time
#pragma unroll
    for (int h = 0; h < NPASS; ++h) {
        if (pack) {
#pragma unroll
            for (int mm = 0; mm < MH; ++mm) {
                const int m = h * MH + mm;
                const int e = 256 * m + 4 * lane;
                float *o = tr + (e / B - h * RH) * P + e % B;
                o[0] = v[m].x;
                o[1] = v[m].y;
                o[2] = v[m].z;
                o[3] = v[m].w;
            }
        }
        __syncthreads();
        if (pack) {
            float *dstT = tilesT + dl * (B * B);
#pragma unroll
            for (int i = 0; i < MH; ++i) {
                // element (rt, ct..ct+3) of the transpose, ct in this half;
                // source row cr of the half.  With two halves, lane groups of
                // 8 take rows rt = 4i + g and 4i + g + 32 so that the 64 lanes
                // hit 64 distinct banks (pitch B + 1).
                int rt, cr;
                if constexpr (NPASS == 2) {
                    cr = 4 * (lane & 7);
                    rt = 4 * i + ((lane >> 3) & 3) + 32 * (lane >> 5);
                } else {
                    const int e = 256 * i + 4 * lane;
                    rt = e / B;
                    cr = e % B;
                }
                const int ct = h * RH + cr;
                const float4 t = make_float4(tr[(cr + 0) * P + rt], tr[(cr + 1) * P + rt],
                                             tr[(cr + 2) * P + rt], tr[(cr + 3) * P + rt]);
                *reinterpret_cast<float4 *>(dstT + L::index(rt, ct)) = t;
                if constexpr (B >= 32) {
                    if (tilesT16 != nullptr) {
                        uint16_t *d16 = tilesT16 + dl * (B * B) + Leaf16Layout<B>::index(rt, ct);
                        if (scale16 != nullptr) {
                            store_fp16x4(d16, t, e16);
                        } else {
                            store_bf16x4(d16, t);
                        }
                    }
                }
            }
        }
        if (h + 1 < NPASS)
            __syncthreads();        // the next half overwrites the buffer
    }
    if (parent != nullptr) {
        if (lane == 0)
            part[w] = s;
        __syncthreads();
        if (threadIdx.x == 0)
            parent[bid] = (part[0] + part[1]) + (part[2] + part[3]);
    }
}

// (at least 3 waves per SIMD: the loads of a 64 x 64 leaf are 64 registers
// a lane, and the build is an HBM stream that needs the waves in flight)
template <int B, int VEC, bool SUB, bool TWO, bool SKIP>
__global__ __launch_bounds__(256, 3) void leaf_norm_pack(const float *__restrict__ A, int64_t n,
                                                      float *__restrict__ tiles,
                                                      float *__restrict__ tilesT,
                                                      uint16_t *__restrict__ tiles16,
                                                      uint16_t *__restrict__ tilesT16,
                                                      double *__restrict__ leaf_norm,
                                                      double *__restrict__ parent,
                                                      double *__restrict__ sub_norm,
                                                      const uint32_t *__restrict__ keep,
                                                      const uint32_t *__restrict__ slot,
                                                      int32_t *__restrict__ scale16,
                                                      uint32_t ntiles, int known_zero)
{
    norm_pack_block<B, VEC, SUB, TWO, SKIP>(A, n, tiles, tilesT, tiles16, tilesT16, leaf_norm,
                                            parent,
                                      sub_norm, keep, slot, scale16, ntiles, known_zero,
                                      blockIdx.x);
}

// Tiers top-1 .. 0 from tier `top` (already built), one workgroup.
__device__ inline void pyramid_tiers(double *__restrict__ norms, int top)
{
    for (int t = top - 1; t >= 0; --t) {
        const double *ch = norms + tier_offset(t + 1);
        double *pa = norms + tier_offset(t);
        const int64_t cnt = int64_t(1) << (2 * t);
        for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x)
            pa[i] = (ch[4 * i] + ch[4 * i + 1]) + (ch[4 * i + 2] + ch[4 * i + 3]);
        __syncthreads();
    }
}

__global__ __launch_bounds__(1024) void norm_pyramid(double *__restrict__ norms, int top)
{
    pyramid_tiers(norms, top);
}

template <int B, int VEC, bool SUB, bool TWO>
static hipError_t launch_leaf_t(const float *A, int64_t n, float *tiles, float *tilesT,
                                uint16_t *t16, uint16_t *tT16, double *leaf, double *parent,
                                double *sub, const uint32_t *keep, const uint32_t *slot,
                                int32_t *scale16, uint32_t ntiles, int known_zero, hipStream_t s)
{
    constexpr size_t lds = sizeof(float) * 4 * (TWO ? B / 2 : B) * (B + 1);
    // once per process (thread-safe static initialization)
    static const hipError_t attr0 =
        hipFuncSetAttribute((const void *)leaf_norm_pack<B, VEC, SUB, TWO, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    static const hipError_t attr1 =
        hipFuncSetAttribute((const void *)leaf_norm_pack<B, VEC, SUB, TWO, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr0 != hipSuccess || attr1 != hipSuccess)
        return attr0 != hipSuccess ? attr0 : attr1;
    if (known_zero)
        hipLaunchKernelGGL((leaf_norm_pack<B, VEC, SUB, TWO, true>), dim3((ntiles + 3) / 4),
                           dim3(256), lds, s, A, n, tiles, tilesT, t16, tT16, leaf, parent, sub,
                           keep, slot, scale16, ntiles, known_zero);
    else
        hipLaunchKernelGGL((leaf_norm_pack<B, VEC, SUB, TWO, false>), dim3((ntiles + 3) / 4),
                           dim3(256), lds, s, A, n, tiles, tilesT, t16, tT16, leaf, parent, sub,
                           keep, slot, scale16, ntiles, known_zero);
    return hipGetLastError();
}

template <int B, int VEC, bool SUB>
static hipError_t launch_leaf_v(const float *A, int64_t n, float *tiles, float *tilesT,
                                uint16_t *t16, uint16_t *tT16, double *leaf, double *parent,
                                double *sub, const uint32_t *keep, const uint32_t *slot,
                                int32_t *scale16, uint32_t ntiles, int known_zero, hipStream_t s)
{
    if constexpr (B == 64)
        return launch_leaf_t<B, VEC, SUB, true>(A, n, tiles, tilesT, t16, tT16, leaf, parent, sub,
                                                keep, slot, scale16, ntiles, known_zero, s);
    else
        return launch_leaf_t<B, VEC, SUB, false>(A, n, tiles, tilesT, t16, tT16, leaf, parent,
                                                 sub, keep, slot, scale16, ntiles, known_zero, s);
}

template <int B, bool SUB>
static hipError_t launch_leaf(const float *A, int64_t n, int vec, float *tiles, float *tilesT,
                              uint16_t *t16, uint16_t *tT16, double *leaf, double *parent,
                              double *sub, const uint32_t *keep, const uint32_t *slot,
                              int32_t *scale16, uint32_t ntiles, int known_zero, hipStream_t s)
{
    if (vec == 4)
        return launch_leaf_v<B, 4, SUB>(A, n, tiles, tilesT, t16, tT16, leaf, parent, sub, keep,
                                        slot, scale16, ntiles, known_zero, s);
    if (vec == 2)
        return launch_leaf_v<B, 2, SUB>(A, n, tiles, tilesT, t16, tT16, leaf, parent, sub, keep,
                                        slot, scale16, ntiles, known_zero, s);
    return launch_leaf_v<B, 1, SUB>(A, n, tiles, tilesT, t16, tT16, leaf, parent, sub, keep, slot,
                                    scale16, ntiles, known_zero, s);
}

static hipError_t launch_leaf_any(const float *A, int64_t n, int leaf, float *tiles,
                                  float *tilesT, uint16_t *t16, uint16_t *tT16, double *leafn,
                                  double *parent, double *subn, const uint32_t *keep,
                                  const uint32_t *slot, int32_t *scale16, uint32_t ntiles,
                                  int known_zero, hipStream_t s)
{
    const uintptr_t addr = reinterpret_cast<uintptr_t>(A);
    const int vec = (n % 4 == 0 && addr % 16 == 0) ? 4 : (n % 2 == 0 && addr % 8 == 0) ? 2 : 1;
    if (scale16 != nullptr && (t16 == nullptr || tT16 == nullptr || leaf == 16))
        return hipErrorInvalidValue;
    switch (leaf) {
    case 16:
        return launch_leaf<16, false>(A, n, vec, tiles, tilesT, nullptr, nullptr, leafn, parent,
                                      nullptr, keep, slot, nullptr, ntiles, known_zero, s);
    case 32:
        return launch_leaf<32, false>(A, n, vec, tiles, tilesT, t16, tT16, leafn, parent, nullptr,
                                      keep, slot, scale16, ntiles, known_zero, s);
    case 64:
        return subn != nullptr
                   ? launch_leaf<64, true>(A, n, vec, tiles, tilesT, t16, tT16, leafn, parent,
                                           subn, keep, slot, scale16, ntiles, known_zero, s)
                   : launch_leaf<64, false>(A, n, vec, tiles, tilesT, t16, tT16, leafn, parent,
                                            nullptr, keep, slot, scale16, ntiles, known_zero, s);
    default: return hipErrorInvalidValue;
    }
}

// sub (n_b = 64 only): norms hold tiers 0..depth+1, tier depth+1 being the
// 32 x 32 sub-blocks; otherwise tiers 0..depth.  tiles == null: norms only.
hipError_t launch_build(const float *A, int64_t n, int leaf, int depth, float *tiles,
                        float *tilesT, uint16_t *t16, uint16_t *tT16, int32_t *scale16,
                        double *norms, bool sub, hipStream_t s)
{
    const uint32_t ntiles = 1u << (2 * depth);
    double *leafn = norms + tier_offset(depth);
    double *parent = depth >= 1 ? norms + tier_offset(depth - 1) : nullptr;
    double *subn = sub ? norms + tier_offset(depth + 1) : nullptr;
    if (sub && leaf != 64)
        return hipErrorInvalidValue;
    hipError_t e = launch_leaf_any(A, n, leaf, tiles, tilesT, t16, tT16, leafn, parent, subn,
                                   nullptr, nullptr, scale16, ntiles, 0, s);
    if (e != hipSuccess || depth < 2)
        return e;
    hipLaunchKernelGGL(norm_pyramid, dim3(1), dim3(1024), 0, s, norms, depth - 1);
    return hipGetLastError();
}

// ---- epsilon-sparsified trees (Sec. II.C) ------------------------------------
// Leaf l is kept iff s_l > 0 and fl64(s_l * m) >= fl64(tau^2), with
// m = max(||A||_F^2, other2) read from the dense root; a dropped leaf's norm
// becomes 0.  The dense root is copied to root_dense first.
__global__ __launch_bounds__(256) void drop_leaves(double *__restrict__ leafn, uint32_t count,
                                                   const double *__restrict__ root, double other2,
                                                   double T2, uint32_t *__restrict__ keep,
                                                   double *__restrict__ root_dense)
{
    const double r = root[0];
    const double m = r > other2 ? r : other2;
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l == 0)
        root_dense[0] = r;
    if (l >= count)
        return;
    const double v = leafn[l];
    const bool k = (v > 0.0) & !(v * m < T2);
    keep[l] = k ? 1u : 0u;
    if (!k)
        leafn[l] = 0.0;
}

// Pass 1 of a sparsified build: dense norms (no pack), drop, the exclusive
// scan of the keep flags into slots (slot[N^2] = leaves kept), and the norm
// pyramid rebuilt over the kept leaves.
hipError_t launch_sparse_norms(const float *A, int64_t n, int leaf, int depth, double *norms,
                               double tau, double other2, uint32_t *keep, uint32_t *slot,
                               uint32_t *partials, double *root_dense, hipStream_t s)
{
    const uint32_t ntiles = 1u << (2 * depth);
    hipError_t e = launch_build(A, n, leaf, depth, nullptr, nullptr, nullptr, nullptr, nullptr,
                                norms, false, s);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(drop_leaves, dim3((ntiles + 255) / 256), dim3(256), 0, s,
                       norms + tier_offset(depth), ntiles, (const double *)norms, other2,
                       tau * tau, keep, root_dense);
    if ((e = hipGetLastError()) != hipSuccess)
        return e;
    if ((e = launch_scan_u32(keep, ntiles, slot, partials, s)) != hipSuccess)
        return e;
    if (depth >= 1) {
        hipLaunchKernelGGL(norm_pyramid, dim3(1), dim3(1024), 0, s, norms, depth);
        e = hipGetLastError();
    }
    return e;
}

// Pass 2: pack the kept leaves (A is read again only where a leaf is kept).
hipError_t launch_sparse_pack(const float *A, int64_t n, int leaf, int depth, float *tiles,
                              float *tilesT, uint16_t *t16, uint16_t *tT16, const uint32_t *keep,
                              const uint32_t *slot, hipStream_t s)
{
    return launch_leaf_any(A, n, leaf, tiles, tilesT, t16, tT16, nullptr, nullptr, nullptr, keep,
                           slot, nullptr, 1u << (2 * depth), 0, s);
}

// ---- the tree of a product's output (Sec. II.C) ------------------------------
// Truncating the product space leaves every leaf of C = A B that no kept
// product reaches at zero.  The plan's leaf-tier schedule says which are
// reached: leaf 4b + q of GEMM block b (the children of a tier-(d-1) node; b
// = 0, q = 0 for the single leaf at depth 0) iff an entry of the block's
// HIGH or LOW list has bit q in its quadrant mask.  One thread per block.
__device__ inline void keep_of_block(const uint32_t *__restrict__ browptr,
                                     const uint32_t *__restrict__ bent,
                                     const uint32_t *__restrict__ browptr_lo,
                                     const uint32_t *__restrict__ bent_lo, uint32_t nblocks,
                                     uint32_t nleaves, uint32_t *__restrict__ keep, uint32_t b)
{
    if (b >= nblocks)
        return;
    uint32_t m = 0;
    for (uint32_t e = browptr[b], e1 = browptr[b + 1]; e < e1 && m != 0xFu; ++e)
        m |= bent[e] >> 16;
    if (browptr_lo != nullptr)
        for (uint32_t e = browptr_lo[b], e1 = browptr_lo[b + 1]; e < e1 && m != 0xFu; ++e)
            m |= bent_lo[e] >> 16;
#pragma unroll
    for (uint32_t q = 0; q < 4; ++q)
        if (4 * b + q < nleaves)
            keep[4 * b + q] = (m >> q) & 1u;
}

__global__ __launch_bounds__(256) void output_keep(const uint32_t *__restrict__ browptr,
                                                   const uint32_t *__restrict__ bent,
                                                   const uint32_t *__restrict__ browptr_lo,
                                                   const uint32_t *__restrict__ bent_lo,
                                                   uint32_t nblocks, uint32_t nleaves,
                                                   uint32_t *__restrict__ keep)
{
    keep_of_block(browptr, bent, browptr_lo, bent_lo, nblocks, nleaves, keep,
                  blockIdx.x * blockDim.x + threadIdx.x);
}

// Tree of C from the plan that produced it, in two parts: the keep flags
// and their exclusive scan into slots (slot[N^2] = leaves stored); then the
// pack and norms of the reached leaves only (the others are not read: norm
// +0) and the pyramid.  The norms are those of the dense tree of C bit for
// bit, as long as C holds the product on every reached leaf.
hipError_t launch_output_map(const uint32_t *browptr, const uint32_t *bent,
                             const uint32_t *browptr_lo, const uint32_t *bent_lo,
                             uint32_t nblocks, int depth, uint32_t *keep, uint32_t *slot,
                             uint32_t *partials, hipStream_t s)
{
    const uint32_t ntiles = 1u << (2 * depth);
    hipLaunchKernelGGL(output_keep, dim3((nblocks + 255) / 256), dim3(256), 0, s, browptr, bent,
                       browptr_lo, bent_lo, nblocks, ntiles, keep);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    return launch_scan_u32(keep, ntiles, slot, partials, s);
}

hipError_t launch_output_pack(const float *C, int64_t n, int leaf, int depth, float *tiles,
                              float *tilesT, uint16_t *t16, uint16_t *tT16, int32_t *scale16,
                              double *norms, const uint32_t *keep, const uint32_t *slot,
                              hipStream_t s)
{
    const uint32_t ntiles = 1u << (2 * depth);
    double *leafn = norms + tier_offset(depth);
    double *parent = depth >= 1 ? norms + tier_offset(depth - 1) : nullptr;
    hipError_t e = launch_leaf_any(C, n, leaf, tiles, tilesT, t16, tT16, leafn, parent, nullptr,
                                   keep, slot, scale16, ntiles, 1, s);
    if (e != hipSuccess || depth < 2)
        return e;
    hipLaunchKernelGGL(norm_pyramid, dim3(1), dim3(1024), 0, s, norms, depth - 1);
    return hipGetLastError();
}

// ---- rounds: the builds of several trees in shared launches ---------------
// A workgroup takes cb <= CB consecutive blocks (4 leaves each) of one tree
// (cb grows with the tree, so a small tree's blocks run side by side and a
// large one needs fewer workgroups).  The first wave finds which of them
// hold a leaf to read (neither known zero nor dropped); the workgroup then
// runs the blocks that do, and a block that does not only gets its zero
// norms (norm pass), so the workgroups of a mostly-zero or mostly-dropped
// tree finish at once.
template <int B, int VEC, bool TWO, int CB>
__global__ __launch_bounds__(256, 3) void leaf_norm_pack_jobs(const Jobs<PackJob> jobs)
{
    static_assert(4 * CB <= kWave, "one wave tests the chunk's leaves");
    const PackJob &p = job_at(jobs, blockIdx.x);
    const uint32_t cb = p.cb;
    const uint32_t b0 = (blockIdx.x - p.block0) * cb;
    __shared__ uint64_t live;
    if (threadIdx.x < kWave) {
        const uint32_t l = 4 * b0 + threadIdx.x;
        bool act = threadIdx.x < 4 * cb && l < p.ntiles;
        if (act && p.known_zero && p.keep[l] == 0u)
            act = false;
        if (act && p.drop_s != nullptr)
            act = p.drop_s[l] > 0.0 && !(p.drop_s[l] * fmax(p.rootA[0], p.rootB[0]) < p.T2);
        const uint64_t m = __ballot(act);
        if (threadIdx.x == 0)
            live = m;
    }
    __syncthreads();
    const uint64_t m = live;
    const uint32_t nblk = (p.ntiles + 3) / 4;
    for (uint32_t i = 0; i < cb && b0 + i < nblk; ++i) {
        const uint32_t b = b0 + i;
        if ((m >> (4 * i)) & 0xFu) {
            norm_pack_block<B, VEC, false, TWO, true>(p.A, p.n, p.tiles, p.tilesT, p.t16, p.tT16,
                                                p.leafn, p.parent, nullptr, p.keep, nullptr,
                                                p.scale16, p.ntiles, p.known_zero, b, p.drop_s,
                                                p.rootA, p.rootB, p.T2);
            __syncthreads();              // the block's LDS (parent partials) is reused
        } else if (p.leafn != nullptr && threadIdx.x < 4) {
            // every leaf of the block is zero: norms +0, and so is the parent
            if (4 * b + threadIdx.x < p.ntiles)
                p.leafn[4 * b + threadIdx.x] = 0.0;
            if (threadIdx.x == 0 && p.parent != nullptr)
                p.parent[b] = 0.0;
        }
    }
}

__global__ __launch_bounds__(1024) void norm_pyramid_jobs(const Jobs<PyrJob> jobs)
{
    const PyrJob &p = jobs.job[blockIdx.x];
    pyramid_tiers(p.norms, p.top);
}

__global__ __launch_bounds__(256) void output_keep_jobs(const Jobs<KeepJob> jobs)
{
    const KeepJob &k = job_at(jobs, blockIdx.x);
    keep_of_block(k.browptr, k.bent, k.browptr_lo, k.bent_lo, k.nblocks, k.nleaves, k.keep,
                  (blockIdx.x - k.block0) * blockDim.x + threadIdx.x);
}

// most blocks per workgroup of the round pack kernel, and the grid a tree's
// blocks are spread over before a workgroup takes more than one
constexpr int kPackChunk = 8;
constexpr uint32_t kPackSpread = 2048;

template <int B, int VEC>
static hipError_t launch_pack_jobs(const Jobs<PackJob> &jobs, hipStream_t s)
{
    constexpr bool TWO = B == 64;
    constexpr size_t lds = sizeof(float) * 4 * (TWO ? B / 2 : B) * (B + 1);
    static const hipError_t attr =
        hipFuncSetAttribute((const void *)leaf_norm_pack_jobs<B, VEC, TWO, kPackChunk>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (attr != hipSuccess)
        return attr;
    hipLaunchKernelGGL((leaf_norm_pack_jobs<B, VEC, TWO, kPackChunk>), dim3(jobs.nblocks),
                       dim3(256), lds, s, jobs);
    return hipGetLastError();
}

static hipError_t launch_pack_any(int leaf, int vec, const Jobs<PackJob> &jobs, hipStream_t s)
{
#define SPAMM_PACK_VEC(B)                                                                     \
    return vec == 4 ? launch_pack_jobs<B, 4>(jobs, s)                                          \
           : vec == 2 ? launch_pack_jobs<B, 2>(jobs, s) : launch_pack_jobs<B, 1>(jobs, s)
    switch (leaf) {
    case 16: SPAMM_PACK_VEC(16);
    case 32: SPAMM_PACK_VEC(32);
    case 64: SPAMM_PACK_VEC(64);
    default: return hipErrorInvalidValue;
    }
#undef SPAMM_PACK_VEC
}

static int load_width(const float *A, int64_t n)
{
    const uintptr_t addr = reinterpret_cast<uintptr_t>(A);
    return (n % 4 == 0 && addr % 16 == 0) ? 4 : (n % 2 == 0 && addr % 8 == 0) ? 2 : 1;
}

// The keep flags of the output trees, then every tree's leaves (one launch
// per leaf size and load width, at most kMaxRound trees each), then the
// pyramids.  Each tree is built exactly as by launch_build (dense) or as an
// output tree with its leaves at their linear index.
hipError_t launch_build_round(const RoundTree *trees, int ntrees, hipStream_t s)
{
    hipError_t e = hipSuccess;
    {
        Jobs<KeepJob> kj{};
        for (int i = 0; i <= ntrees && e == hipSuccess; ++i) {
            if (i < ntrees && trees[i].from != nullptr) {
                const spamm_plan *p = trees[i].from;
                const bool split = p->precision != SPAMM_PREC_FP32;
                KeepJob &k = kj.job[kj.njobs++];
                k.browptr = p->browptr;
                k.bent = p->bent;
                k.browptr_lo = split ? p->browptr_lo : nullptr;
                k.bent_lo = split ? p->bent_lo : nullptr;
                k.keep = trees[i].tree->keep;
                k.nblocks = (uint32_t)p->nblocks;
                k.nleaves = 1u << (2 * p->depth);
                k.block0 = kj.nblocks;
                kj.nblocks += (k.nblocks + 255) / 256;
            }
            if (kj.njobs > 0 && (i == ntrees || kj.njobs == kMaxRound)) {
                hipLaunchKernelGGL(output_keep_jobs, dim3(kj.nblocks), dim3(256), 0, s, kj);
                e = hipGetLastError();
                kj = Jobs<KeepJob>{};
            }
        }
    }
    // pass 1 (tau > 0): norms only; pass 2 after the pyramids: the pack of
    // the leaves that can take part in a kept product.  tau = 0: one pass.
    auto pack_pass = [&](int pass) {
        std::vector<bool> done(ntrees, false);
        for (int i = 0; i < ntrees && e == hipSuccess; ++i) {
            if (done[i])
                continue;
            const int leaf = trees[i].tree->leaf;
            const int vec = load_width(trees[i].src, trees[i].tree->n);
            Jobs<PackJob> pj{};
            for (int k = i; k < ntrees && e == hipSuccess; ++k) {
                const spamm_tree *t = trees[k].tree;
                if (done[k] || t->leaf != leaf || load_width(trees[k].src, t->n) != vec)
                    continue;
                done[k] = true;
                const bool two = trees[k].T2 > 0.0;
                if (pass == 2 && !two)
                    continue;
                const int d = t->depth;
                PackJob &p = pj.job[pj.njobs++];
                p = PackJob{};
                p.A = trees[k].src;
                p.n = t->n;
                p.ntiles = 1u << (2 * d);
                const uint32_t nblk = (p.ntiles + 3) / 4;
                p.cb = std::min<uint32_t>(kPackChunk, (nblk + kPackSpread - 1) / kPackSpread);
                p.block0 = pj.nblocks;
                pj.nblocks += (nblk + p.cb - 1) / p.cb;
                if (pass == 1) {
                    p.leafn = t->norms + tier_offset(d);
                    p.parent = d >= 1 ? t->norms + tier_offset(d - 1) : nullptr;
                    p.keep = trees[k].from != nullptr ? t->keep : nullptr;
                    p.known_zero = trees[k].from != nullptr ? 1 : 0;
                }
                if (pass == 2 || !two) {
                    p.tiles = t->tiles;
                    p.tilesT = t->tilesT;
                    p.t16 = t->tiles16;
                    p.tT16 = t->tilesT16;
                    p.scale16 = t->scale16;
                }
                if (pass == 2) {
                    p.drop_s = t->norms + tier_offset(d);
                    p.rootA = t->norms;
                    p.rootB = trees[k].other->norms;
                    p.T2 = trees[k].T2;
                }
                if (pj.njobs == kMaxRound) {
                    e = launch_pack_any(leaf, vec, pj, s);
                    pj = Jobs<PackJob>{};
                }
            }
            if (e == hipSuccess && pj.njobs > 0)
                e = launch_pack_any(leaf, vec, pj, s);
        }
    };
    pack_pass(1);
    Jobs<PyrJob> yj{};
    for (int i = 0; i <= ntrees && e == hipSuccess; ++i) {
        if (i < ntrees && trees[i].tree->depth >= 2) {
            PyrJob &y = yj.job[yj.njobs++];
            y.norms = trees[i].tree->norms;
            y.top = trees[i].tree->depth - 1;
            y.block0 = (uint32_t)yj.njobs - 1;
        }
        if (yj.njobs > 0 && (i == ntrees || yj.njobs == kMaxRound)) {
            hipLaunchKernelGGL(norm_pyramid_jobs, dim3(yj.njobs), dim3(1024), 0, s, yj);
            e = hipGetLastError();
            yj = Jobs<PyrJob>{};
        }
    }
    pack_pass(2);
    return e;
}

}  // namespace spamm
