/*
 * philox.c -- oracle copy of the counter-based generator Philox4x32-10
 * (J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11, Sec. 3 and Table 2).
 *
 * Test infrastructure: see oracle.h.  The paper's own generator
 * (Parisi-Rapuano + congruential, appendix A.4) keeps per-thread state; a
 * counter-based generator replaces it so that any update can be replayed
 * from (seed, counter) alone.
 *
 * Definition used: a round maps (x0, x1, x2, x3) with key (k0, k1) to
 *   (hi(M1*x2) ^ x1 ^ k0,  lo(M1*x2),  hi(M0*x0) ^ x3 ^ k1,  lo(M0*x0))
 * with M0 = 0xD2511F53, M1 = 0xCD9E8D57; the key is advanced by the Weyl
 * increments (0x9E3779B9, 0xBB67AE85) before every round but the first.
 */
#include "oracle.h"

void or_philox4x32_10(const uint32_t key[2], const uint32_t ctr[4], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t k0 = key[0], k1 = key[1];
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* 23 random bits, centred in their bin: ((w >> 9) + 1/2) 2^-23.
 * The numerator is an odd integer below 2^24, so the value is exact in FP32
 * as well as in FP64, and so is 1 - u. */
double or_u23(uint32_t w)
{
    return ((double)(w >> 9) + 0.5) * 0x1p-23;
}

/* 52 random bits (26 from each word), centred: exact in FP64. */
double or_u52(uint32_t w0, uint32_t w1)
{
    uint64_t m = ((uint64_t)(w0 >> 6) << 26) | (uint64_t)(w1 >> 6);
    return ((double)m + 0.5) * 0x1p-52;
}

uint32_t or_ctr3(uint32_t tag, uint32_t tslot, uint32_t rep)
{
    return (tag << 28) | (tslot << 16) | (rep << 8);
}
