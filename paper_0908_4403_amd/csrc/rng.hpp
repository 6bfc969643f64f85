// Counter-based random numbers on the device: Philox4x32-10 (Salmon, Moraes,
// Dror, Shaw, SC'11).  One call maps (counter, key) to four 32-bit words with
// ten rounds of two 32x32->64 multiplies; the key is bumped by the Weyl
// constants between rounds.  Stateless, so any point can be regenerated from
// its index alone.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace heget {

struct Words4 {
    uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                uint32_t c3, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 multiply gives both halves of each product
        const uint64_t pA = static_cast<uint64_t>(kMulA) * c0;
        const uint64_t pB = static_cast<uint64_t>(kMulB) * c2;
        // three-input XOR in one instruction (bit table 0x96: odd number of ones)
        const uint32_t t0 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(pB >> 32), c1, k0, 0x96);
        const uint32_t t2 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(pA >> 32), c3, k1, 0x96);
        c0 = t0;
        c1 = static_cast<uint32_t>(pB);
        c2 = t2;
        c3 = static_cast<uint32_t>(pA);
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return {c0, c1, c2, c3};
}

// Uniform in (0,1) from 53 bits of the 64-bit word (hi:lo): (w >> 11 + 1/2) 2^-53.
__device__ __forceinline__ double open_unit(uint32_t lo, uint32_t hi)
{
    const uint64_t w = (static_cast<uint64_t>(hi) << 32) | lo;
    return (static_cast<double>(w >> 11) + 0.5) * 0x1.0p-53;
}

// Uniform in (0,1) from one 32-bit word: (w + 1/2) 2^-32.
__device__ __forceinline__ double open_unit32(uint32_t w)
{
    return (static_cast<double>(w) + 0.5) * 0x1.0p-32;
}

// Four uniforms for (seed, point, block, stream), one per word of one call.
// Counter = {lo(point), hi(point), block, stream}, key = {lo(seed), hi(seed)}.
// Stream 0 block i feeds photon i (cos theta, azimuth, two for the energy).
__device__ __forceinline__ void uniform_quad(uint64_t seed, uint64_t point, uint32_t block,
                                             uint32_t stream, double (&u)[4])
{
    const Words4 r = philox4x32_10(static_cast<uint32_t>(point),
                                   static_cast<uint32_t>(point >> 32), block, stream,
                                   static_cast<uint32_t>(seed),
                                   static_cast<uint32_t>(seed >> 32));
    u[0] = open_unit32(r.w0);
    u[1] = open_unit32(r.w1);
    u[2] = open_unit32(r.w2);
    u[3] = open_unit32(r.w3);
}

// Two uniforms of 53 bits for (seed, point, block, stream), same counter and
// key.  Stream 1 feeds the partonic kinematics (block 0: parton momentum
// fractions, block 1: sqrt(shat)).
__device__ __forceinline__ void uniform_pair(uint64_t seed, uint64_t point, uint32_t block,
                                             uint32_t stream, double &u0, double &u1)
{
    const Words4 r = philox4x32_10(static_cast<uint32_t>(point),
                                   static_cast<uint32_t>(point >> 32), block, stream,
                                   static_cast<uint32_t>(seed),
                                   static_cast<uint32_t>(seed >> 32));
    u0 = open_unit(r.w0, r.w1);
    u1 = open_unit(r.w2, r.w3);
}

}  // namespace heget
