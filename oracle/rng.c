/*
 * rng.c -- oracle random numbers. Test infrastructure only (see omc_oracle.h).
 *
 * The paper (Sec. 2.2.3) gives every work-item its own RANECU seed drawn from
 * the host clock. That makes results depend on scheduling, so the build keys
 * a counter-based generator instead: Philox4x32 with 10 rounds (Salmon, Moraes,
 * Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11), with
 *   key     = (seed, h)            h = global history index
 *   counter = (n, q_lo, q_hi, 0)   q = 64-bit particle id, n = block index
 * The four output words of a block are used in order. A uniform in (0,1) is
 * u = (2*(x >> 9) + 1) * 2^-24, exact in both float and double.
 */
#include <stddef.h>
#include "omc_oracle.h"

/* One Philox round: two 32x32->64 products; the high halves are mixed with the
 * other two words and the key, the low halves become the new odd words. */
static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0];
    const uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        philox_round(c, k);
        /* the key is bumped by the Weyl constants between rounds */
        k[0] += 0x9E3779B9u;
        k[1] += 0xBB67AE85u;
    }
    out[0] = c[0];
    out[1] = c[1];
    out[2] = c[2];
    out[3] = c[3];
}

double orc_u01(uint32_t x)
{
    const uint32_t odd = ((x >> 9) << 1) | 1u; /* 24-bit odd integer */
    return (double)odd * (1.0 / 16777216.0);
}

void orc_stream_words(uint32_t seed, uint32_t h, uint64_t q, uint32_t n0, uint32_t nblocks,
                      uint32_t* out)
{
    const uint32_t key[2] = {seed, h};
    for (uint32_t b = 0; b < nblocks; ++b) {
        const uint32_t ctr[4] = {n0 + b, (uint32_t)q, (uint32_t)(q >> 32), 0u};
        orc_philox4x32_10(ctr, key, out + 4 * (size_t)b);
    }
}

void orc_u01_array(const uint32_t* x, size_t n, double* out)
{
    for (size_t i = 0; i < n; ++i) out[i] = orc_u01(x[i]);
}
