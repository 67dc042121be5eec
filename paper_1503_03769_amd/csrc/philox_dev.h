// Device-side counter-based random numbers for libpphd.
//
// Philox-4x32-10 from Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
// as easy as 1, 2, 3" (SC'11): ten applications of a bijective round on four
// 32-bit words.  A round forms the two 64-bit products of words 0 and 2 with the
// multipliers 0xD2511F53 and 0xCD9E8D57, returns
//   (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)),
// and the key is advanced by the Weyl increments 0x9E3779B9, 0xBB67AE85 between
// rounds.  Each (slot, step, purpose, run) tuple owns one block, so any thread
// can draw its numbers without state.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pphd {

enum : uint32_t { RNG_INIT = 1, RNG_PREDICT = 2, RNG_BIRTH = 3, RNG_RESAMPLE = 4, RNG_EXCHANGE = 5 };

struct Block4 {
    uint32_t a, b, c, d;
};

__device__ __forceinline__ Block4 philox4x32_10(Block4 x, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
        uint32_t hi0 = __umulhi(m0, x.a), lo0 = m0 * x.a;
        uint32_t hi1 = __umulhi(m1, x.c), lo1 = m1 * x.c;
        x = Block4{ hi1 ^ x.b ^ k0, lo1, hi0 ^ x.d ^ k1, lo0 };
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return x;
}

// Counter layout shared with every consumer of the streams:
// (c0 = slot or group index, step, purpose * 16 + sub-draw, run id), key = seed.
__device__ __forceinline__ Block4 rng_block(uint32_t key0, uint32_t key1, uint32_t c0, uint32_t step,
                                            uint32_t purpose, uint32_t sub, uint32_t run)
{
    return philox4x32_10(Block4{ c0, step, purpose * 16u + sub, run }, key0, key1);
}

// 53-bit uniform on (0, 1]: (hi:32 bits of a, 21 bits of b) + 1, times 2^-53.
__device__ __forceinline__ double uniform53(uint32_t a, uint32_t b)
{
    uint64_t k = ((uint64_t)a << 21) | (uint64_t)(b >> 11);
    return (double)(k + 1u) * 0x1p-53;
}

// Box-Muller: two independent N(0, 1) values from two uniforms.
__device__ __forceinline__ void normal_pair(double u1, double u2, double& n1, double& n2)
{
    // sin/cos of 2 pi u2 through sincospi (one argument reduction, exact
    // scaling by pi inside the routine)
    const double rad = sqrt(-2.0 * log(u1));
    double sn, cs;
    sincospi(2.0 * u2, &sn, &cs);
    n1 = rad * cs;
    n2 = rad * sn;
}

}  // namespace pphd
