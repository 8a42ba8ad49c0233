// Philox4x32-10 counter-based generator (J. K. Salmon, M. A. Moraes,
// R. O. Dror, D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3",
// SC'11, sect. 3.2): per round two 32x32->64-bit products of counter words
// with fixed multipliers, the high halves xored with the other counter words
// and the key; the key is bumped by the two Weyl constants between rounds.
//
// Event-parallel sampling (the paper's event axis, sect. 1) draws the uniforms
// of event `ev` from key = (seed_lo, seed_hi), counter = (ev_lo, ev_hi, j, 0),
// j = dimension / 2; the four output words (r0, r1, r2, r3) give
// u0 = r1:r0 and u1 = r3:r2 (64-bit) for dimensions 2j and 2j+1, mapped to
// (u >> 11) * 2^-53 in [0, 1).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(M0, c[0]), lo0 = M0 * c[0];
        const uint32_t hi1 = __umulhi(M1, c[2]), lo1 = M1 * c[2];
        const uint32_t n0 = hi1 ^ c[1] ^ k0;
        const uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
        k0 += W0; k1 += W1;
    }
}

__device__ __forceinline__ double u64_to_unit(uint64_t u)
{
    return (double)(u >> 11) * 1.1102230246251565404e-16;   // 2^-53
}

// Uniforms of global event `ev` for dimensions 0..d-1.
template <int D>
__device__ __forceinline__ void event_uniforms(uint64_t seed, uint64_t ev, double x[D])
{
#pragma unroll
    for (int j = 0; j < (D + 1) / 2; ++j) {
        uint32_t c[4] = {(uint32_t)ev, (uint32_t)(ev >> 32), (uint32_t)j, 0u};
        philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
        const uint64_t u0 = ((uint64_t)c[1] << 32) | c[0];
        const uint64_t u1 = ((uint64_t)c[3] << 32) | c[2];
        x[2 * j] = u64_to_unit(u0);
        if (2 * j + 1 < D) x[2 * j + 1] = u64_to_unit(u1);
    }
}
