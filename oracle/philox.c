/*
 * Oracle counter-based generator (test infrastructure only).
 *
 * Philox4x64-10 as published by Salmon, Moraes, Dror and Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3" (SC'11): ten rounds of two 64x64->128 bit
 * multiplications with the round key advanced by the Weyl constants between
 * rounds.  The paper under test only asks for "a suitable random number
 * generator" available to row updates (Sec. 2.1); a counter-based one lets the
 * GPU and this oracle replay the same draws from (seed, step, row, slot).
 */
#include <math.h>
#include "oracle.h"

static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void orc_philox4x64_10(uint64_t key0, uint64_t key1, const uint64_t ctr[4], uint64_t out[4])
{
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    for (int r = 0; r < 10; ++r) {
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, x0, &hi0, &lo0);
        mulhilo64(M1, x2, &hi1, &lo1);
        uint64_t n0 = hi1 ^ x1 ^ key0;
        uint64_t n2 = hi0 ^ x3 ^ key1;
        x0 = n0;
        x1 = lo1;
        x2 = n2;
        x3 = lo0;
        key0 += W0;
        key1 += W1;
    }
    out[0] = x0;
    out[1] = x1;
    out[2] = x2;
    out[3] = x3;
}

static void block(uint64_t seed, uint32_t tag, uint32_t proj, uint64_t c0, uint64_t c1,
                  uint64_t c2, uint64_t c3, uint64_t out[4])
{
    uint64_t ctr[4] = {c0, c1, c2, c3};
    orc_philox4x64_10(seed, (uint64_t)tag | ((uint64_t)proj << 8), ctr, out);
}

uint32_t orc_u32(uint64_t seed, uint32_t tag, uint32_t proj, uint64_t c0, uint64_t c1,
                 uint64_t c2, uint64_t c3)
{
    uint64_t o[4];
    block(seed, tag, proj, c0, c1, c2, c3, o);
    return (uint32_t)(o[0] >> 32);
}

/* Integer uniformly below n by multiply-shift (no rejection). */
uint32_t orc_below(uint32_t u, uint32_t n)
{
    return (uint32_t)(((uint64_t)u * (uint64_t)n) >> 32);
}

/* Bernoulli threshold: a trial with probability p succeeds when u32 < T(p). */
uint64_t orc_threshold(double p)
{
    if (!(p > 0.0)) return 0;
    if (p >= 1.0) return 1ull << 32;
    return (uint64_t)floor(p * 4294967296.0);
}

/* Standard normal by the Box-Muller transform of output words 0 and 1. */
double orc_normal(uint64_t seed, uint32_t tag, uint32_t proj, uint64_t c0, uint64_t c1,
                  uint64_t c2, uint64_t c3)
{
    uint64_t o[4];
    block(seed, tag, proj, c0, c1, c2, c3, o);
    const double two_m53 = 1.0 / 9007199254740992.0;
    double u1 = (double)((o[0] >> 11) + 1) * two_m53; /* (0, 1] */
    double u2 = (double)(o[1] >> 11) * two_m53;       /* [0, 1) */
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

/* Threads the loops with OpenMP pragmas run on: 1 in the parity build. */
#ifdef _OPENMP
#include <omp.h>
int32_t orc_threads(void) { return (int32_t)omp_get_max_threads(); }
#else
int32_t orc_threads(void) { return 1; }
#endif
