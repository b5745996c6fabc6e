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
//   Couplings: every bond joins an even and an odd site, so each bond is
//   stored once, with its even end, as a bit in one of six planes
//   d = +x, -x, +y, -y, +z, -z over the even sites: J[s][d][h / 32] bit h % 32.
//   That is 6 bits per even site = 3 bits per site.
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
    int32_t P32;   // 32-bit words per coupling plane
    int32_t S, R;  // samples, replicas per sample
    uint32_t key0, key1;
};

// Byte-wise sum of a 32-bit word whose bytes add up to less than 256.
__device__ __forceinline__ uint32_t bytesum(uint32_t v) { return (v * 0x01010101u) >> 24; }

// Spread a nibble b3b2b1b0 into bytes: bit i -> bit 0 of byte i.  The
// partial products b << 7i never overlap, so no carries cross bytes.
__device__ __forceinline__ uint32_t spread4(uint32_t nib) { return (nib * 0x00204081u) & 0x01010101u; }

// 4 bits of coupling plane d for the even sites h .. h+3 (h % 4 == 0).
__device__ __forceinline__ uint32_t jnib(const uint32_t* __restrict__ Js, int32_t P32, int d, int64_t h)
{
    return (__ldg(&Js[(int64_t)d * P32 + (h >> 5)]) >> (h & 31)) & 0xFu;
}

// Nibble of the group shifted by one site along the row: dir > 0 takes
// sites k+1 .. k+4 (n1 = group after), dir < 0 takes k-1 .. k+2 (n1 = group before).
__device__ __forceinline__ uint32_t shift_nib(uint32_t n0, uint32_t n1, int dir)
{
    return dir > 0 ? ((n0 >> 1) | ((n1 & 1u) << 3)) : (((n0 << 1) & 0xFu) | (n1 >> 3));
}

// Same shift for a word of 4 byte-sites.
__device__ __forceinline__ uint32_t shift_word(uint32_t w0, uint32_t w1, int dir)
{
    return dir > 0 ? ((w0 >> 8) | (w1 << 24)) : ((w0 << 8) | (w1 >> 24));
}

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) { return a ^ b ^ c; }

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
