/*
 * SpAMM reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU implementation of what the GPU path computes, written in
 * double precision from the paper (Bock & Challacombe, "An Optimized Sparse
 * Approximate Matrix Multiply for Matrices with Decay").  Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, table or helper with the GPU library.
 *
 * What it follows:
 *   depth and padding  -- Sec. II.A, Eq. for the depth d and zero padding to
 *                         n_p = n_b 2^d (d = 0 when n <= n_b).
 *   node norms         -- Sec. II.B, Eq. for the Frobenius norm: squared norms
 *                         add over the 2x2 children, built from the bottom tier.
 *                         Precision/order are not given by the paper; this
 *                         oracle fixes them: FP64, leaf sum = pairwise
 *                         (recursive halving) over the tile's row-major
 *                         flattened index, parent = (s11 + s12) + (s21 + s22).
 *   product recursion  -- Sec. II.B, Eq. product: C^t_ij = sum_k A^{t+1}_ik
 *                         B^{t+1}_kj, children visited in quadrant order
 *                         (11,12,21,22) and k = 1,2.
 *   SpAMM condition    -- Sec. II.B, Eq. norm condition: a product is dropped
 *                         when ||A|| ||B|| < tau.  Compared here in squared
 *                         form, s_A * s_B >= tau^2 keeps (equality keeps).  A
 *                         node whose norm is zero is a NULL link (Sec. II.A)
 *                         and is never multiplied, at any tau.
 *   linear index       -- Sec. III.D.1, Eq. linear index: row bits on the odd
 *                         positions, column bits on the even positions.
 *
 * Leaf products accumulate in FP64, k ascending within each output tile, and
 * the product of two FP32 values is exact in FP64.
 *
 * Split precision (the precision extension the paper's conclusions point
 * to): a kept leaf product is LOW iff s_A * s_B < L2, with L2 = low_tol^2
 * for an absolute threshold, or L2 = (theta^2 * s_A0) * s_B0 for a relative
 * one (s_A0, s_B0 the root squared norms: norm product < theta ||A|| ||B||,
 * every step in FP64 in that order); its operands
 * are rounded elementwise to bfloat16 (8 significant bits, round to nearest,
 * ties to even) before the (exact, FP64) products; other products are
 * unchanged.  The class is part of the task key (bit 63).  With binary16
 * LOW operands each leaf is scaled by a power of two 2^e fixed by its
 * squared norm before the rounding (11 significant bits; a value that rounds
 * below binary16's normal range, 2^-14, becomes zero), and the product is
 * scaled back by 2^-(eA + eB).
 *
 * Compensated HIGH products (format 2): LOW operands rounded to bfloat16 as
 * above, and each entry x of a HIGH product split into two bfloat16 parts,
 * hi = bf16(x) and lo = bf16(x - hi) (x - hi is exact in single precision),
 * with the product a b taken as hi_a hi_b + hi_a lo_b + lo_a hi_b: the
 * three-product bfloat16 method of Henry, Tang and Heinecke ("Leveraging the
 * bfloat16 artificial intelligence datatype for higher-precision
 * computations", ARITH 2019), which drops lo_a lo_b and the parts below lo.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OR_OK = 0, OR_EINVAL = -1, OR_ERANGE = -2, OR_ENOMEM = -3 };

/* Sec. II.A depth: smallest d >= 0 with n_b * 2^d >= n, i.e. ceil(log2(n/n_b))
 * clamped at 0; n_p = n_b * 2^d. */
int oracle_depth(int64_t n, int32_t b, int32_t *d_out, int64_t *np_out)
{
    if (n < 1 || b < 1)
        return OR_EINVAL;
    int32_t d = 0;
    int64_t np = b;
    while (np < n) {
        np *= 2;
        d += 1;
    }
    *d_out = d;
    *np_out = np;
    return OR_OK;
}

/* Eq. linear index: l = sum_m [ i_m 2^(2m+1) + j_m 2^(2m) ]. */
uint64_t oracle_linear_index(uint64_t i, uint64_t j)
{
    uint64_t l = 0;
    for (int m = 0; m < 32; ++m) {
        uint64_t im = (i >> m) & 1u, jm = (j >> m) & 1u;
        l += im << (2 * m + 1);
        l += jm << (2 * m);
    }
    return l;
}

/* Pairwise (recursive halving) sum of v[0..len). */
static double pairwise_sum(const double *v, int64_t len)
{
    if (len == 1)
        return v[0];
    int64_t h = len / 2;
    return pairwise_sum(v, h) + pairwise_sum(v + h, len - h);
}

/* Element (r, c) of the zero-padded matrix. */
static double elem(const float *A, int64_t n, int64_t r, int64_t c)
{
    if (r >= n || c >= n)
        return 0.0;
    return (double)A[r * n + c];
}

/* Offsets of the per-tier squared-norm arrays: tier t holds N_t x N_t values,
 * row-major, N_t = 2^t, starting at (4^t - 1) / 3. */
static int64_t tier_offset(int t) { return (((int64_t)1 << (2 * t)) - 1) / 3; }

int64_t oracle_norms_len(int32_t d) { return tier_offset(d + 1); }

/* Squared Frobenius norms of every node of every tier, tier 0 (root) first. */
int oracle_norms(const float *A, int64_t n, int32_t b, double *out)
{
    int32_t d;
    int64_t np;
    int rc = oracle_depth(n, b, &d, &np);
    if (rc)
        return rc;
    int64_t N = (int64_t)1 << d;
    double *leaf = out + tier_offset(d);
    int failed = 0;
    /* Tiles are independent; the threads only split the work. */
#pragma omp parallel
    {
        double *sq = (double *)malloc(sizeof(double) * (size_t)b * (size_t)b);
        if (!sq) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(static)
        for (int64_t I = 0; I < N; ++I) {
            if (!sq)
                continue;
            for (int64_t J = 0; J < N; ++J) {
                for (int64_t r = 0; r < b; ++r)
                    for (int64_t c = 0; c < b; ++c) {
                        double x = elem(A, n, I * b + r, J * b + c);
                        sq[r * b + c] = x * x;
                    }
                leaf[I * N + J] = pairwise_sum(sq, (int64_t)b * b);
            }
        }
        free(sq);
    }
    if (failed)
        return OR_ENOMEM;
    for (int t = d - 1; t >= 0; --t) {
        int64_t Nt = (int64_t)1 << t;
        const double *ch = out + tier_offset(t + 1);
        double *pa = out + tier_offset(t);
        for (int64_t I = 0; I < Nt; ++I)
            for (int64_t J = 0; J < Nt; ++J) {
                int64_t N2 = 2 * Nt;
                double s11 = ch[(2 * I) * N2 + 2 * J], s12 = ch[(2 * I) * N2 + 2 * J + 1];
                double s21 = ch[(2 * I + 1) * N2 + 2 * J], s22 = ch[(2 * I + 1) * N2 + 2 * J + 1];
                pa[I * Nt + J] = (s11 + s12) + (s21 + s22);
            }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------- */
/* Recursive multiply                                                         */
/* ------------------------------------------------------------------------- */
typedef struct {
    const float *A, *B;
    int64_t n;
    int32_t b, d;
    double T2;             /* tau * tau */
    double L2;             /* low_tol * low_tol (0: nothing is LOW) */
    const double *sA, *sB; /* all tiers, oracle_norms layout */
    double *C;             /* n x n, may be NULL */
    uint64_t *keys;        /* may be NULL */
    int64_t cap, nkeys;
    int64_t *Kt;           /* kept count per tier, d+1 entries */
    int64_t Klow;          /* kept leaf products classed LOW */
    int fmt;               /* LOW operands: 0 bfloat16, 1 binary16 with a leaf scale,
                              2 bfloat16 with compensated HIGH products */
} mul_ctx;

static int kept(const mul_ctx *x, int t, int64_t I, int64_t K, int64_t J)
{
    int64_t Nt = (int64_t)1 << t;
    double sa = x->sA[tier_offset(t) + I * Nt + K];
    double sb = x->sB[tier_offset(t) + K * Nt + J];
    if (sa == 0.0 || sb == 0.0)   /* NULL link */
        return 0;
    if (sa * sb < x->T2)          /* SpAMM condition: product dropped */
        return 0;
    return 1;
}

/* x rounded to the nearest bfloat16 (ties to even), returned as a double.
 * bfloat16 keeps the sign, the 8 exponent bits and the top 7 fraction bits of
 * an IEEE single; the 16 dropped bits decide the rounding. */
static double to_bf16(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    uint32_t hi = u >> 16, rem = u & 0xFFFFu;
    if (rem > 0x8000u || (rem == 0x8000u && (hi & 1u)))
        hi += 1u;
    uint32_t r = hi << 16;
    float y;
    memcpy(&y, &r, 4);
    return (double)y;
}

double oracle_bf16(float x) { return to_bf16(x); }

/* The two bfloat16 parts of x: hi = bf16(x), lo = bf16(x - hi).  hi keeps
 * the top 8 significant bits of x (rounded), so x - hi is a multiple of x's
 * single-precision spacing below 2^-8 |x| and is exact as a float. */
static void bf16_parts(float x, double *hi, double *lo)
{
    *hi = to_bf16(x);
    float r = x - (float)*hi;
    *lo = to_bf16(r);
}

void oracle_bf16_parts(float x, double *hi, double *lo) { bf16_parts(x, hi, lo); }

/* Scale exponent of a leaf whose squared norm is S, for binary16 operands:
 * with S = m 2^p (0.5 <= m < 1) every entry has |x| <= sqrt(S) < 2^q,
 * q = ceil(p / 2), so e = 14 - q keeps every scaled entry |x| 2^e below 2^14,
 * well inside binary16's range (largest finite 65504).  A zero leaf is never
 * multiplied; it gets 0. */
int oracle_fp16_exponent(double S)
{
    if (!(S > 0.0))
        return 0;
    int p;
    frexp(S, &p);
    int q = p >= 0 ? (p + 1) / 2 : -((-p) / 2);
    return 14 - q;
}

/* x 2^e rounded to the nearest binary16 value (ties to even), scaled back by
 * 2^-e, as a double (exact).  binary16 keeps 11 significant bits for
 * magnitudes in [2^-14, 2^16) and a fixed spacing 2^-24 below 2^-14; a
 * result below 2^-14 (a subnormal) is flushed to zero, since the matrix
 * units' products of binary16 subnormals are not exact.  The caller keeps
 * |x 2^e| below 2^15. */
double oracle_fp16_scaled(float x, int e)
{
    double y = ldexp((double)x, e);
    if (y == 0.0)
        return 0.0;
    int E;
    frexp(fabs(y), &E);             /* leading bit of |y| is 2^(E-1) */
    int lead = E - 1 < -14 ? -14 : E - 1;
    double quantum = ldexp(1.0, lead - 10);
    double r = nearbyint(y / quantum) * quantum;   /* default mode: nearest, ties to even */
    if (fabs(r) < ldexp(1.0, -14))
        return 0.0;
    return ldexp(r, -e);
}
static int is_low(const mul_ctx *x, int t, int64_t I, int64_t K, int64_t J)
{
    int64_t Nt = (int64_t)1 << t;
    double sa = x->sA[tier_offset(t) + I * Nt + K];
    double sb = x->sB[tier_offset(t) + K * Nt + J];
    return sa * sb < x->L2;
}

/* Element (r, c) of the padded matrix; for a LOW product rounded to
 * bfloat16, or (fmt 1) to binary16 at the leaf's scale exponent e. */
static double elem_p(const float *A, int64_t n, int64_t r, int64_t c, int low, int fmt, int e)
{
    if (r >= n || c >= n)
        return 0.0;
    if (!low)
        return (double)A[r * n + c];
    return fmt == 1 ? oracle_fp16_scaled(A[r * n + c], e) : to_bf16(A[r * n + c]);
}

/* a b of a HIGH product in format 2: hi_a hi_b + hi_a lo_b + lo_a hi_b. */
static double comp_product(const float *A, const float *B, int64_t n, int64_t r, int64_t l,
                           int64_t c)
{
    if (r >= n || l >= n || c >= n)
        return 0.0;
    double ha, la, hb, lb;
    bf16_parts(A[r * n + l], &ha, &la);
    bf16_parts(B[l * n + c], &hb, &lb);
    return ha * hb + ha * lb + la * hb;
}

/* C_IJ += A_IK * B_KJ over the n x n (unpadded) part, l ascending; operands
 * rounded to the LOW format for a LOW product. */
static void leaf_product(mul_ctx *x, int64_t I, int64_t K, int64_t J, double *Ct,
                         int64_t ldc, int64_t r0, int64_t c0, int low)
{
    int64_t b = x->b, n = x->n;
    int64_t Nd = (int64_t)1 << x->d;
    int eA = 0, eB = 0;
    if (low && x->fmt == 1) {
        eA = oracle_fp16_exponent(x->sA[tier_offset(x->d) + I * Nd + K]);
        eB = oracle_fp16_exponent(x->sB[tier_offset(x->d) + K * Nd + J]);
    }
    for (int64_t p = 0; p < b; ++p) {
        int64_t row = I * b + p;
        if (row >= n)
            break;
        for (int64_t q = 0; q < b; ++q) {
            int64_t col = J * b + q;
            if (col >= n)
                break;
            double acc = 0.0;
            if (!low && x->fmt == 2) {
                for (int64_t l = 0; l < b; ++l)
                    acc += comp_product(x->A, x->B, n, row, K * b + l, col);
            } else {
                for (int64_t l = 0; l < b; ++l)
                    acc += elem_p(x->A, n, row, K * b + l, low, x->fmt, eA) *
                           elem_p(x->B, n, K * b + l, col, low, x->fmt, eB);
            }
            Ct[(row - r0) * ldc + (col - c0)] += acc;
        }
    }
}

static void emit(mul_ctx *x, int64_t I, int64_t K, int64_t J, int low)
{
    if (x->keys && x->nkeys < x->cap)
        x->keys[x->nkeys] = (oracle_linear_index((uint64_t)I, (uint64_t)J) << 32) | (uint64_t)K |
                            ((uint64_t)low << 63);
    x->nkeys += 1;
}

/* Eq. product applied at tier t to the node triple (I, K, J). */
static void spamm(mul_ctx *x, int t, int64_t I, int64_t K, int64_t J)
{
    if (!kept(x, t, I, K, J))
        return;
    x->Kt[t] += 1;
    if (t == x->d) {
        int low = is_low(x, t, I, K, J);
        x->Klow += low;
        emit(x, I, K, J, low);
        if (x->C)
            leaf_product(x, I, K, J, x->C, x->n, 0, 0, low);
        return;
    }
    for (int a = 0; a < 2; ++a)          /* child row    (quadrants 11,12,21,22) */
        for (int bq = 0; bq < 2; ++bq)   /* child column */
            for (int c = 0; c < 2; ++c)  /* inner index k = 1, 2 */
                spamm(x, t + 1, 2 * I + a, 2 * K + c, 2 * J + bq);
}

/* Keys compare on (leaf, k); bit 63 only carries the class. */
static int cmp_u64(const void *a, const void *b)
{
    uint64_t m = ~((uint64_t)1 << 63);
    uint64_t x = *(const uint64_t *)a & m, y = *(const uint64_t *)b & m;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static int check_inputs(int64_t n, int32_t b, double tau)
{
    if (n < 1 || b < 1 || (b & (b - 1)) != 0)
        return OR_EINVAL;
    if (!(tau >= 0.0) || isinf(tau))
        return OR_EINVAL;
    return OR_OK;
}

/*
 * Full recursive SpAMM product C~ = A B (n x n FP64, fully overwritten when C
 * is not NULL).  Kept leaf triples are returned as sorted keys
 * (linear_index(I,J) << 32) | K; *nkeys gets the total (keys beyond cap are
 * counted, not stored; OR_ERANGE then).  Kt[t] = kept triples at tier t.
 */
int oracle_spamm_split_fmt(const float *A, const float *B, int64_t n, int32_t b, double tau,
                           double low_tol, int fmt, double *C, uint64_t *keys, int64_t cap,
                           int64_t *nkeys, int64_t *Kt, int64_t *Klow);
static int run_split(const float *A, const float *B, int64_t n, int32_t b, double tau,
                     double low_tol, double theta, int fmt, double *C, uint64_t *keys,
                     int64_t cap, int64_t *nkeys, int64_t *Kt, int64_t *Klow);

int oracle_spamm(const float *A, const float *B, int64_t n, int32_t b, double tau,
                 double *C, uint64_t *keys, int64_t cap, int64_t *nkeys, int64_t *Kt)
{
    int64_t Klow;
    return oracle_spamm_split_fmt(A, B, n, b, tau, 0.0, 0, C, keys, cap, nkeys, Kt, &Klow);
}

/* As oracle_spamm with split precision: LOW iff s_A s_B < low_tol^2, LOW
 * operands in bfloat16. */
int oracle_spamm_split(const float *A, const float *B, int64_t n, int32_t b, double tau,
                       double low_tol, double *C, uint64_t *keys, int64_t cap, int64_t *nkeys,
                       int64_t *Kt, int64_t *Klow)
{
    return oracle_spamm_split_fmt(A, B, n, b, tau, low_tol, 0, C, keys, cap, nkeys, Kt, Klow);
}

/* Split precision with the LOW operand format fmt: 0 bfloat16, 1 binary16
 * with a per-leaf power-of-two scale. */
int oracle_spamm_split_fmt(const float *A, const float *B, int64_t n, int32_t b, double tau,
                           double low_tol, int fmt, double *C, uint64_t *keys, int64_t cap,
                           int64_t *nkeys, int64_t *Kt, int64_t *Klow)
{
    return run_split(A, B, n, b, tau, low_tol, 0.0, fmt, C, keys, cap, nkeys, Kt, Klow);
}

/* Split precision with a relative threshold: LOW iff s_A s_B <
 * (theta^2 s_A0) s_B0, i.e. ||A_ik|| ||B_kj|| < theta ||A||_F ||B||_F on the
 * stored squared norms, the roots s_A0, s_B0 taken from this product's own
 * norm pyramids. */
int oracle_spamm_split_rel(const float *A, const float *B, int64_t n, int32_t b, double tau,
                           double theta, int fmt, double *C, uint64_t *keys, int64_t cap,
                           int64_t *nkeys, int64_t *Kt, int64_t *Klow)
{
    return run_split(A, B, n, b, tau, 0.0, theta, fmt, C, keys, cap, nkeys, Kt, Klow);
}

/* L2 of the LOW test: low_tol^2 (absolute) or (theta^2 s_A0) s_B0 (relative). */
static double low_threshold(double low_tol, double theta, const double *sA, const double *sB)
{
    if (theta > 0.0) {
        double t2 = theta * theta;
        double u = t2 * sA[0];
        return u * sB[0];
    }
    return low_tol * low_tol;
}

static int check_split(double low_tol, double theta, int fmt)
{
    if (!(low_tol >= 0.0) || isinf(low_tol) || fmt < 0 || fmt > 2)
        return OR_EINVAL;
    if (!(theta >= 0.0) || isinf(theta) || (theta > 0.0 && low_tol > 0.0))
        return OR_EINVAL;
    return OR_OK;
}

static int run_split(const float *A, const float *B, int64_t n, int32_t b, double tau,
                     double low_tol, double theta, int fmt, double *C, uint64_t *keys,
                     int64_t cap, int64_t *nkeys, int64_t *Kt, int64_t *Klow)
{
    int rc = check_inputs(n, b, tau);
    if (rc)
        return rc;
    if ((rc = check_split(low_tol, theta, fmt)))
        return rc;
    mul_ctx x;
    memset(&x, 0, sizeof x);
    int64_t np;
    oracle_depth(n, b, &x.d, &np);
    int64_t len = oracle_norms_len(x.d);
    double *sA = (double *)malloc(sizeof(double) * (size_t)len);
    double *sB = (double *)malloc(sizeof(double) * (size_t)len);
    if (!sA || !sB) {
        free(sA);
        free(sB);
        return OR_ENOMEM;
    }
    oracle_norms(A, n, b, sA);
    oracle_norms(B, n, b, sB);
    x.A = A;
    x.B = B;
    x.n = n;
    x.b = b;
    x.T2 = tau * tau;
    x.L2 = low_threshold(low_tol, theta, sA, sB);
    x.fmt = fmt;
    x.sA = sA;
    x.sB = sB;
    x.C = C;
    x.keys = keys;
    x.cap = cap;
    x.Kt = Kt;
    for (int t = 0; t <= x.d; ++t)
        Kt[t] = 0;
    if (C)
        memset(C, 0, sizeof(double) * (size_t)n * (size_t)n);
    spamm(&x, 0, 0, 0, 0);
    *nkeys = x.nkeys;
    *Klow = x.Klow;
    if (keys)
        qsort(keys, (size_t)(x.nkeys < cap ? x.nkeys : cap), sizeof(uint64_t), cmp_u64);
    free(sA);
    free(sB);
    return x.nkeys > cap && keys ? OR_ERANGE : OR_OK;
}

/*
 * The same recursion restricted to chosen output tiles: for target leaf tile
 * (I, J) the row and column of every ancestor are fixed, so only the inner
 * index K branches (k = 1, 2 at every tier).  Produces, per target tile, the
 * b x b block of C~ (FP64, rows/columns beyond n left at zero), the number of
 * kept leaf products and, optionally, their K values in ascending order.
 * Tiles are independent and may run on several threads.
 */
typedef struct {
    mul_ctx *x;
    int64_t I, J;         /* target leaf tile */
    double *Ct;           /* b x b */
    int64_t count;
    int32_t *kl;          /* may be NULL; capacity N */
} tile_ctx;

static void spamm_tile(tile_ctx *y, int t, int64_t K)
{
    mul_ctx *x = y->x;
    int64_t I = y->I >> (x->d - t), J = y->J >> (x->d - t);
    if (!kept(x, t, I, K, J))
        return;
    if (t == x->d) {
        int low = is_low(x, t, I, K, J);
        if (y->kl)
            y->kl[y->count] = (int32_t)K | (low << 30);
        y->count += 1;
        leaf_product(x, I, K, J, y->Ct, x->b, I * x->b, J * x->b, low);
        return;
    }
    for (int c = 0; c < 2; ++c)
        spamm_tile(y, t + 1, 2 * K + c);
}

int oracle_spamm_tiles_split_fmt(const float *A, const float *B, int64_t n, int32_t b,
                                 double tau, double low_tol, int fmt, const int64_t *tiles,
                                 int64_t ntiles, double *Ctiles, int64_t *counts,
                                 int32_t *klists, int nthreads);
static int run_tiles(const float *A, const float *B, int64_t n, int32_t b, double tau,
                     double low_tol, double theta, int fmt, const int64_t *tiles,
                     int64_t ntiles, double *Ctiles, int64_t *counts, int32_t *klists,
                     int nthreads);

int oracle_spamm_tiles(const float *A, const float *B, int64_t n, int32_t b, double tau,
                       const int64_t *tiles, int64_t ntiles, double *Ctiles,
                       int64_t *counts, int32_t *klists, int nthreads)
{
    return oracle_spamm_tiles_split_fmt(A, B, n, b, tau, 0.0, 0, tiles, ntiles, Ctiles, counts,
                                        klists, nthreads);
}

int oracle_spamm_tiles_split(const float *A, const float *B, int64_t n, int32_t b, double tau,
                             double low_tol, const int64_t *tiles, int64_t ntiles, double *Ctiles,
                             int64_t *counts, int32_t *klists, int nthreads)
{
    return oracle_spamm_tiles_split_fmt(A, B, n, b, tau, low_tol, 0, tiles, ntiles, Ctiles,
                                        counts, klists, nthreads);
}

/* klists entries: K | (1 << 30) for a LOW product. */
int oracle_spamm_tiles_split_fmt(const float *A, const float *B, int64_t n, int32_t b,
                                 double tau, double low_tol, int fmt, const int64_t *tiles,
                                 int64_t ntiles, double *Ctiles, int64_t *counts,
                                 int32_t *klists, int nthreads)
{
    return run_tiles(A, B, n, b, tau, low_tol, 0.0, fmt, tiles, ntiles, Ctiles, counts, klists,
                     nthreads);
}

/* As oracle_spamm_tiles_split_fmt with the relative LOW threshold of
 * oracle_spamm_split_rel (roots of the whole operands' pyramids). */
int oracle_spamm_tiles_split_rel(const float *A, const float *B, int64_t n, int32_t b,
                                 double tau, double theta, int fmt, const int64_t *tiles,
                                 int64_t ntiles, double *Ctiles, int64_t *counts,
                                 int32_t *klists, int nthreads)
{
    return run_tiles(A, B, n, b, tau, 0.0, theta, fmt, tiles, ntiles, Ctiles, counts, klists,
                     nthreads);
}

static int run_tiles(const float *A, const float *B, int64_t n, int32_t b, double tau,
                     double low_tol, double theta, int fmt, const int64_t *tiles,
                     int64_t ntiles, double *Ctiles, int64_t *counts, int32_t *klists,
                     int nthreads)
{
    int rc = check_inputs(n, b, tau);
    if (rc)
        return rc;
    if ((rc = check_split(low_tol, theta, fmt)))
        return rc;
    mul_ctx x;
    memset(&x, 0, sizeof x);
    int64_t np;
    oracle_depth(n, b, &x.d, &np);
    int64_t N = (int64_t)1 << x.d;
    for (int64_t s = 0; s < ntiles; ++s)
        if (tiles[2 * s] < 0 || tiles[2 * s] >= N || tiles[2 * s + 1] < 0 || tiles[2 * s + 1] >= N)
            return OR_EINVAL;
    int64_t len = oracle_norms_len(x.d);
    double *sA = (double *)malloc(sizeof(double) * (size_t)len);
    double *sB = (double *)malloc(sizeof(double) * (size_t)len);
    if (!sA || !sB) {
        free(sA);
        free(sB);
        return OR_ENOMEM;
    }
    oracle_norms(A, n, b, sA);
    oracle_norms(B, n, b, sB);
    x.A = A;
    x.B = B;
    x.n = n;
    x.b = b;
    x.T2 = tau * tau;
    x.L2 = low_threshold(low_tol, theta, sA, sB);
    x.fmt = fmt;
    x.sA = sA;
    x.sB = sB;
    int64_t bb = (int64_t)b * b;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t s = 0; s < ntiles; ++s) {
        tile_ctx y;
        y.x = &x;
        y.I = tiles[2 * s];
        y.J = tiles[2 * s + 1];
        y.Ct = Ctiles + s * bb;
        memset(y.Ct, 0, sizeof(double) * (size_t)bb);
        y.count = 0;
        y.kl = klists ? klists + s * N : NULL;
        spamm_tile(&y, 0, 0);
        counts[s] = y.count;
    }
    free(sA);
    free(sB);
    return OR_OK;
}
