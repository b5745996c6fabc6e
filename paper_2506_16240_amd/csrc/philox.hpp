// Philox4x32-10 counter-based generator for the device (Salmon, Moraes,
// Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).
// Ten rounds of two 32x32->64 multiplications; the key is advanced by the
// Weyl increments between rounds.  Counter-based: one call per (stream,
// sample, replica, site group, time), no state to carry or checkpoint.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace micsa {

struct u32x4 {
    uint32_t v0, v1, v2, v3;
};

__device__ __forceinline__ u32x4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                          uint32_t k1)
{
    constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
    constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)kMulA * c0;
        const uint64_t pb = (uint64_t)kMulB * c2;
        // three-input XORs in one v_bitop3 each (truth table 0x96)
        const uint32_t t0 = __builtin_amdgcn_bitop3_b32((uint32_t)(pb >> 32), c1, k0, 0x96);
        const uint32_t t2 = __builtin_amdgcn_bitop3_b32((uint32_t)(pa >> 32), c3, k1, 0x96);
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = t0;
        c2 = t2;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return {c0, c1, c2, c3};
}

// Stream tags in the top byte of the last counter word; sample in the low 24 bits.
enum : uint32_t { kStreamCoupling = 1u, kStreamSpin = 2u, kStreamDaemon = 3u, kStreamHeatBath = 4u, kStreamMetropolis = 5u };

__device__ __forceinline__ uint32_t stream_word(uint32_t stream, uint32_t sample)
{
    return (stream << 24) | sample;
}

}  // namespace micsa
