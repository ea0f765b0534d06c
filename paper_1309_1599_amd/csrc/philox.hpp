// philox.hpp -- device Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
//
// Counter-based: every draw is a pure function of (key, counter), so any
// heat-bath update or tempering decision can be recomputed anywhere without
// per-thread generator state.  This replaces the per-thread lagged
// Parisi-Rapuano + congruential generators of appendix A.4.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ptsg {

// Ten rounds of the Philox4x32 bijection.  Round: multiply words 0 and 2
// by the two Philox multipliers, then
//   out = (hi(B*c2) ^ c1 ^ k0, lo(B*c2), hi(A*c0) ^ c3 ^ k1, lo(A*c0));
// the key moves by the Weyl constants between rounds.
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t A = 0xD2511F53u, B = 0xCD9E8D57u;
    constexpr uint32_t WA = 0x9E3779B9u, WB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hA = __umulhi(A, c.x), lA = A * c.x;
        const uint32_t hB = __umulhi(B, c.z), lB = B * c.z;
        c = make_uint4(hB ^ c.y ^ k0, lB, hA ^ c.w ^ k1, lA);
        k0 += WA;
        k1 += WB;
    }
    return c;
}

// Fourth counter word: tag (4 bits) | temperature slot (12) | replica (8).
__device__ __forceinline__ uint32_t ctr_word3(uint32_t tag, uint32_t slot, uint32_t rep)
{
    return (tag << 28) | (slot << 16) | (rep << 8);
}

// 23 bits centred in their bin, exact in FP32 (odd numerator < 2^24).
__device__ __forceinline__ float unit23(uint32_t w)
{
    return (static_cast<float>(w >> 9) + 0.5f) * 0x1p-23f;
}

// 52 bits centred in their bin, exact in FP64.
__device__ __forceinline__ double unit52(uint32_t w0, uint32_t w1)
{
    const uint64_t m = (static_cast<uint64_t>(w0 >> 6) << 26) | static_cast<uint64_t>(w1 >> 6);
    return (static_cast<double>(m) + 0.5) * 0x1p-52;
}

}  // namespace ptsg
