// Device-side geometry of the byte layout and SWAR (SIMD-within-a-register)
// helpers shared by the byte-layout kernels.
//
// Byte layout (per lattice l = sample*R + replica):
//   Sites are split by checkerboard parity p = (x+y+z) & 1 (Sec. 2.1).  In a
//   row (y, z) the sites of parity p sit at x = 2k + ((p + y + z) & 1),
//   k = x >> 1 in 0..Lx/2-1, and are stored contiguously:
//       h = k + (Lx/2) * (y + Ly*z)            (0 <= h < N/2)
//   spin[l][p][h], daemon[l][p][h]: one byte each (spin bit, daemon level).
//   With this split, the four y/z neighbours of a site sit at the same k in
//   the adjacent rows of the other parity, and the two x neighbours at k and
//   k +- 1 of the same row -- so 4 sites packed in a 32-bit word see their
//   neighbours as whole words (or one byte-shifted word).
//   daemon[l][a][p][h] for the gamma daemon (walker) families a of a site.
//   Couplings: every bond joins an even and an odd site, so each bond is
//   stored once, with its even end, in the even site's spin byte: bit 0 is
//   the spin, bit 1 + d the coupling bit of its bond in direction d = +x, -x,
//   +y, -y, +z, -z.  Odd spin bytes hold the spin only.  A sweep reads and
//   writes the spin bytes anyway, so the couplings cost no extra traffic;
//   every replica of a sample carries the same bits.  Four even bytes form a
//   32-bit word, so bond d of 4 sites is (word >> (1 + d)) & 0x01010101.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace micsa {

enum : int { kPx = 0, kMx = 1, kPy = 2, kMy = 3, kPz = 4, kMz = 5 };

struct Geom {
    int32_t Lx, Ly, Lz;
    int32_t Kx;    // Lx / 2: sites of one parity per row
    int32_t Wr;    // 4-site words per row = Kx / 4
    int32_t rows;  // Ly * Lz
    int64_t Nh;    // N / 2: sites of one parity
    int32_t S, R;  // samples, replicas per sample
    uint32_t key0, key1;
    int32_t gamma;  // daemons (walkers) per site: daemon arrays are [S*R][gamma][2][Nh]
};

// Daemon levels are drawn as m = #{k : u >= t_k} from a 32-bit uniform u,
// t_k = floor(2^32 P(m <= k)) (eq. prob-daemons-walkers); the heat bath sets
// s = +1 iff u < tau[v].  Thresholds are 64-bit so 2^32 ("always") fits.
struct DaemonThresholds {
    uint64_t t0, t1, t2;
};

// m = #{k : u >= t_k} in 32-bit compares.  Every t_k lies in [2^30, 2^32]:
// P(m <= 0) = 1 / (1 + x + x^2 + x^3) >= 1/4 with x = e^{-4 beta} in (0, 1),
// so t_k - 1 fits 32 bits and u >= t_k  <=>  u > t_k - 1.
__device__ __forceinline__ uint32_t daemon_level(uint32_t u, const DaemonThresholds& th)
{
    return (uint32_t)(u > (uint32_t)(th.t0 - 1u)) + (uint32_t)(u > (uint32_t)(th.t1 - 1u)) +
           (uint32_t)(u > (uint32_t)(th.t2 - 1u));
}

struct HeatBathThresholds {
    uint64_t tau[7];
};

// Metropolis: a proposed flip with energy change dH = 4q - 12 (q in 0..6) is
// accepted iff u < theta[q], theta = floor(2^32 e^{-beta dH}) uphill, 2^32
// for dH <= 0.  Same 7-entry shape as the heat-bath table.
using MetropolisThresholds = HeatBathThresholds;

// Byte-wise sum of a 32-bit word whose bytes add up to less than 256.
__device__ __forceinline__ uint32_t bytesum(uint32_t v) { return (v * 0x01010101u) >> 24; }

// Coupling bits of bond d for the 4 sites of a word of bond bytes (the even
// spin bytes shifted right by one).
__device__ __forceinline__ uint32_t jbits(uint32_t jw, int d) { return (jw >> d) & 0x01010101u; }

// Same shift for a word of 4 byte-sites.
__device__ __forceinline__ uint32_t shift_word(uint32_t w0, uint32_t w1, int dir)
{
    return dir > 0 ? ((w0 >> 8) | (w1 << 24)) : ((w0 << 8) | (w1 >> 24));
}

// a ^ b ^ c in one v_bitop3 (truth table 0x96, symmetric in its operands).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Every per-lattice integer accumulator (energy tally, reduction outputs) is
// spread over kSlots 64-bit slots; a block adds its sum to slot
// blockIdx.x % kSlots, so no single address takes more than 1/kSlots of the
// atomics.  Readers sum the slots (integer addition: order-independent).
constexpr int kSlots = 64;

__device__ __forceinline__ long long wave_sum64(long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Work-group barrier that orders LDS accesses only.  __syncthreads() also
// fences global memory, which makes every wave wait for all of its global
// loads before the barrier; kernels that prefetch the next step's operands
// from global memory into registers, and share nothing through global memory
// within a work-group, use this one so that the loads stay in flight.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Block-wide sum of v, added by one thread to slots[blockIdx.x % kSlots].
// Must be reached by every thread of the block.
__device__ __forceinline__ void block_add(unsigned long long* slots, long long v)
{
    __shared__ long long part[16];
    v = wave_sum64(v);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long t = 0;
        for (unsigned i = 0; i < (blockDim.x + 63u) >> 6; ++i) t += part[i];
        if (t != 0) atomicAdd(&slots[blockIdx.x % kSlots], (unsigned long long)t);
    }
}

}  // namespace micsa
