/*
 * Seeded synthetic matrices with decay, shared by the CPU reference and the
 * GPU path as plain FP32 bytes.  Nothing here computes any part of the
 * multiply; it only draws inputs.
 *
 * Noise: u(i,j) in [-1,1), symmetric in (i,j).  It is output number idx+1 of
 * the SplitMix64 generator (Steele, Lea & Flood, OOPSLA 2014) started from
 * state `seed`, with idx = (min(i,j) << 32) | max(i,j).  The top 53 bits give a
 * double in [0,1) which is mapped to [-1,1).
 *
 * Decay models follow the introduction of the paper (exponential
 * |a_ij| < c*lambda^|i-j| and algebraic c/(|i-j|^lambda + 1)); the molecular
 * cluster form replaces |i-j| by the distance between the centres of the two
 * molecules that own basis functions i and j.
 *
 * Every element is formed in double precision and rounded to float once
 * (round to nearest, denormals kept).  Rows [row0, row0+nrows) of an n-column
 * row-major matrix are written to out; OpenMP splits the rows.
 */
#include <math.h>
#include <stdint.h>

#define SM64_GAMMA 0x9E3779B97F4A7C15ULL

uint64_t spgen_splitmix64_at(uint64_t seed, uint64_t idx)
{
    uint64_t z = seed + (idx + 1u) * SM64_GAMMA;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

double spgen_sym_u(uint64_t seed, int64_t i, int64_t j)
{
    uint64_t lo = (uint64_t)(i < j ? i : j);
    uint64_t hi = (uint64_t)(i < j ? j : i);
    uint64_t z = spgen_splitmix64_at(seed, (lo << 32) | hi);
    return (double)(z >> 11) * 0x1.0p-53 * 2.0 - 1.0;
}

void spgen_exp_decay(float *out, int64_t n, int64_t row0, int64_t nrows,
                     double rate, uint64_t seed)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = row0 + r;
        float *row = out + r * n;
        for (int64_t j = 0; j < n; ++j) {
            double dist = (double)(i > j ? i - j : j - i);
            row[j] = (float)(spgen_sym_u(seed, i, j) * exp(-rate * dist));
        }
    }
}

void spgen_alg_decay(float *out, int64_t n, int64_t row0, int64_t nrows,
                     double power, uint64_t seed)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = row0 + r;
        float *row = out + r * n;
        for (int64_t j = 0; j < n; ++j) {
            double dist = (double)(i > j ? i - j : j - i);
            row[j] = (float)(spgen_sym_u(seed, i, j) / (pow(dist, power) + 1.0));
        }
    }
}

/* a_ij = u_ij * env[group[i] * ngroups + group[j]]; env is precomputed by the
 * caller (e.g. exp(-lambda * r) between molecule centres). */
void spgen_group_decay(float *out, int64_t n, int64_t row0, int64_t nrows,
                       const int32_t *group, const double *env,
                       int64_t ngroups, uint64_t seed)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = row0 + r;
        float *row = out + r * n;
        const double *erow = env + (int64_t)group[i] * ngroups;
        for (int64_t j = 0; j < n; ++j)
            row[j] = (float)(spgen_sym_u(seed, i, j) * erow[group[j]]);
    }
}
