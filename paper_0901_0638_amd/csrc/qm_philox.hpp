/*
 * qm_philox.hpp -- the counter-based generator Philox4x32-10 on the device
 * (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as 1, 2,
 * 3", SC'11), and the open uniforms drawn from it.
 *
 * One block: counter (c0, c1, c2, c3), key (k0, k1); ten rounds of
 *   (hi0, lo0) = M0 * c0,  (hi1, lo1) = M1 * c2   (32 x 32 -> 64 bits)
 *   c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0),  k <- k + (W0, W1)
 * with the published multipliers M0, M1 and Weyl constants W0, W1.
 *
 * Stream layout: key = (seed, stream) (32 bits each); the block of index b
 * has counter (b mod 2^32, b div 2^32, 0, 0).  FP64 element e takes block
 * e/2, words (0,1) for even e and (2,3) for odd e as one 64-bit value (low
 * word first) whose top 53 bits k give u = (k + 1/2) 2^-53, rounded to
 * nearest: exact for k < 2^52, a tie (to even) above, so u lies in
 * [2^-54, 1] and equals 1 only for k = 2^53 - 1 (probability 2^-53).  FP32
 * element e takes word e mod 4 of block e/4, whose top 23 bits k give
 * u = (k + 1/2) 2^-23, exact in FP32 (at most 24 significant bits): u lies
 * in [2^-24, 1 - 2^-24], open at both ends.
 */
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qm {

struct PhiloxWords {
    uint32_t w[4];
};

__device__ __forceinline__ PhiloxWords philox4x32_10(uint64_t block, uint32_t k0, uint32_t k1)
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = (uint32_t)block, c1 = (uint32_t)(block >> 32), c2 = 0u, c3 = 0u;
    /* The key (uniform across the wave) is passed through an empty asm
       statement, so that the round keys below are formed per block by
       scalar adds instead of being hoisted out of the caller's loop: held
       for the whole loop, the twenty of them crowd the scalar registers of
       the fused kernels, which then spill them to vector lanes and reload
       them with vector instructions in every block. */
    asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += W0;
        k1 += W1;
    }
    PhiloxWords o;
    o.w[0] = c0;
    o.w[1] = c1;
    o.w[2] = c2;
    o.w[3] = c3;
    return o;
}

/* u = (k + 1/2) 2^-53, k the top 53 bits of (hi:lo): k is exact in FP64,
   the addition rounds to nearest even (a tie for k >= 2^52; 1.0 for
   k = 2^53 - 1), the scaling is exact */
__device__ __forceinline__ double open_u53(uint32_t lo, uint32_t hi)
{
    uint64_t k = ((((uint64_t)hi) << 32) | lo) >> 11;
    return ((double)k + 0.5) * 0x1p-53;
}

/* u = (k + 1/2) 2^-23, k the top 23 bits of the word: k + 1/2 has at most
   24 significant bits, so every step is exact and 0 < u < 1 */
__device__ __forceinline__ float open_u23(uint32_t word)
{
    return ((float)(word >> 9) + 0.5f) * 0x1p-23f;
}

/* element e of the stream, one at a time (heads, tails, unaligned outputs) */
template <typename T> __device__ T stream_uniform(uint64_t e, uint32_t k0, uint32_t k1);
template <> __device__ __forceinline__ double stream_uniform<double>(uint64_t e, uint32_t k0, uint32_t k1)
{
    PhiloxWords b = philox4x32_10(e >> 1, k0, k1);
    return (e & 1) ? open_u53(b.w[2], b.w[3]) : open_u53(b.w[0], b.w[1]);
}
template <> __device__ __forceinline__ float stream_uniform<float>(uint64_t e, uint32_t k0, uint32_t k1)
{
    PhiloxWords b = philox4x32_10(e >> 2, k0, k1);
    uint32_t lo = (e & 1) ? b.w[1] : b.w[0], hi = (e & 1) ? b.w[3] : b.w[2];
    return open_u23((e & 2) ? hi : lo);
}

}  // namespace qm
