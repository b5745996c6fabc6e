// LDS-resident sweeps for small lattices (byte layout): one work-group owns
// one lattice, copies its spins, daemons and coupling bytes into LDS, runs
// many sweeps there -- refreshes (Sec. 2.7), even half, odd half (Sec. 2.8),
// optional from-scratch energy logging -- separated only by work-group
// barriers, and writes the state back at the end.  A launch replaces
// thousands of per-half launches, which dominate lattices of a few thousand
// sites.  The SWAR move is the fused sweep's (creutz4); spins and daemon
// levels share one LDS byte per site.
#pragma once
#include "byte_kernels.hpp"

namespace micsa {

// Schedule slice for one resident launch: thresholds of refreshes
// rho0 .. rho0 + nrho - 1 (a device table), refresh period (0 = logarithmic).
struct ResidentSched {
    int64_t k0;      // first sweep index
    int64_t n;       // sweeps in this launch
    int64_t rho0;    // refresh index of the first table entry
    int32_t period;  // refresh period, 0 = before sweeps k with k+1 a power of two
    int32_t log_stride;  // 0 = no logging
    int64_t log_row0;    // first log row written by this launch
};

__device__ __forceinline__ bool dev_is_refresh(int64_t k, int32_t P)
{
    return P >= 1 ? (k % P == 0) : (((k + 1) & k) == 0);
}

__device__ __forceinline__ int64_t dev_refresh_index(int64_t k, int32_t P)
{
    if (P >= 1) return k / P;
    return 63 - __clzll((unsigned long long)(k + 1));  // floor(log2(k + 1))
}

// Work-group sum (every thread must call); returns the sum in every thread.
__device__ __forceinline__ long long block_sum(long long v, long long* red)
{
    v = wave_sum64(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    long long t = 0;
    for (unsigned i = 0; i < (blockDim.x + 63u) >> 6; ++i) t += red[i];
    return t;
}

// Neighbourhood of word (y, z, c) from a row-major array of words (Wr per
// row); the same arithmetic as gather<P>, with the row coordinates given.
// The state words hold spin bits in bit 0 of each byte and possibly other
// bits above (the daemon level); only bit 0 of the neighbours is used.
template <int P>
__device__ __forceinline__ uint32_t unsat_resident(const Geom& g, const uint32_t* st, const uint32_t* Js, int y, int z,
                                                   int c, uint32_t S)
{
    const int q = (y + z) & 1;
    const int dir = (q ^ P) ? 1 : -1;
    const int cs = dir > 0 ? (c + 1 == g.Wr ? 0 : c + 1) : (c == 0 ? g.Wr - 1 : c - 1);
    const int yp = y + 1 == g.Ly ? 0 : y + 1, ym = y == 0 ? g.Ly - 1 : y - 1;
    const int zp = z + 1 == g.Lz ? 0 : z + 1, zm = z == 0 ? g.Lz - 1 : z - 1;
    const int wr = g.Wr;
    const int row = y + g.Ly * z;
    const int r_yp = yp + g.Ly * z, r_ym = ym + g.Ly * z, r_zp = y + g.Ly * zp, r_zm = y + g.Ly * zm;
    const uint32_t m1 = 0x01010101u;
    const uint32_t A = st[row * wr + c];
    const uint32_t B = shift_word(A, st[row * wr + cs], dir);
    const int dA = q ? kMx : kPx, dB = q ? kPx : kMx;
    uint32_t jA, jB, jyp, jym, jzp, jzm;
    if (P == 0) {
        const uint32_t jw = Js[row * wr + c];
        jA = jbits(jw, dA);
        jB = jbits(jw, dB);
        jyp = jbits(jw, kPy);
        jym = jbits(jw, kMy);
        jzp = jbits(jw, kPz);
        jzm = jbits(jw, kMz);
    } else {
        const uint32_t jw = Js[row * wr + c];
        jA = jbits(jw, dA);
        jB = jbits(shift_word(jw, Js[row * wr + cs], dir), dB);
        jyp = jbits(Js[r_yp * wr + c], kMy);
        jym = jbits(Js[r_ym * wr + c], kPy);
        jzp = jbits(Js[r_zp * wr + c], kMz);
        jzm = jbits(Js[r_zm * wr + c], kPz);
    }
    // (S ^ j) is clean (bit 0 only), the neighbour's bit 0 is masked in
    return xor_and(S ^ jA, A, m1) + xor_and(S ^ jB, B, m1) + xor_and(S ^ jyp, st[r_yp * wr + c], m1) +
           xor_and(S ^ jym, st[r_ym * wr + c], m1) + xor_and(S ^ jzp, st[r_zp * wr + c], m1) +
           xor_and(S ^ jzm, st[r_zm * wr + c], m1);
}

// Sweeps of lattice l of one context (all threads of the work-group call it).
// hth: per-refresh table of the baseline (heat bath or Metropolis), unused
// by MicSA.
// LDS: per site one state byte (spin in bit 0, daemon level in bits 1-2),
// plus one coupling byte per even site: 1.5 B per site.
template <int ALGO>  // 0 MicSA, 1 heat bath, 2 Metropolis
__device__ __forceinline__ void resident_body(const Geom& g, uint8_t* __restrict__ spin, uint8_t* __restrict__ dem,
                                              unsigned long long* __restrict__ tally,
                                              const ResidentSched& rs, const DaemonThresholds* __restrict__ dth,
                                              const HeatBathThresholds* __restrict__ hth, long long* __restrict__ log,
                                              int l, int n_lattices, uint32_t* lds32, long long* red, uint64_t* tau)
{
    const int s = l / g.R, r = l % g.R;
    const int W = (int)(g.Nh / 4);  // words per parity
    uint32_t* st = lds32;          // [2][W] packed state
    uint32_t* jb = lds32 + 2 * W;  // [W] coupling bytes of the even sites
    const uint32_t m1 = 0x01010101u;

    const uint32_t* spg = reinterpret_cast<const uint32_t*>(spin + (int64_t)l * 2 * g.Nh);
    const uint32_t* dmg = reinterpret_cast<const uint32_t*>(dem + (int64_t)l * 2 * g.Nh);
    // even spin bytes carry their bond bits in bits 1..6 (geometry.hpp)
    for (int w = threadIdx.x; w < 2 * W; w += blockDim.x) st[w] = (spg[w] & m1) | (ALGO == 0 ? dmg[w] << 1 : 0u);
    for (int w = threadIdx.x; w < W; w += blockDim.x) jb[w] = (spg[w] >> 1) & 0x3F3F3F3Fu;

    // The words of this thread: w = threadIdx.x + j * blockDim.x.  Their
    // (y, z, c) are advanced incrementally instead of divided out per word.
    const int c0 = threadIdx.x % g.Wr;
    const int row0 = threadIdx.x / g.Wr;
    const int y0 = row0 % g.Ly, z0 = row0 / g.Ly;
    const int drow = blockDim.x / g.Wr, dc = blockDim.x % g.Wr;
    __syncthreads();

    int dE = 0;
    int64_t row_out = rs.log_row0;
    for (int64_t it = 0; it < rs.n; ++it) {
        const int64_t k = rs.k0 + it;
        const int64_t rho = dev_refresh_index(k, rs.period);
        if (ALGO == 0 && dev_is_refresh(k, rs.period)) {
            const DaemonThresholds th = dth[rho - rs.rho0];
            const uint32_t sw = stream_word(kStreamDaemon, (uint32_t)s);
            for (int t = threadIdx.x; t < W; t += blockDim.x) {
                const int64_t i0 = 8 * (int64_t)t;
                const u32x4 a = philox10((uint32_t)(i0 >> 2), (uint32_t)rho, (uint32_t)r, sw, g.key0, g.key1);
                const u32x4 b = philox10((uint32_t)(i0 >> 2) + 1u, (uint32_t)rho, (uint32_t)r, sw, g.key0, g.key1);
                uint32_t we, wo;
                split8(g, i0, a, b,
                       [&](uint32_t u) { return daemon_level(u, th); },
                       we, wo);
                st[t] = (st[t] & m1) | (we << 1);
                st[W + t] = (st[W + t] & m1) | (wo << 1);
            }
            __syncthreads();
        }
        if (ALGO != 0) {  // the baseline's table (heat bath tau or Metropolis theta) of refresh rho
            if (threadIdx.x < 7) tau[threadIdx.x] = hth[rho - rs.rho0].tau[threadIdx.x];
            __syncthreads();
        }
#pragma unroll
        for (int P = 0; P < 2; ++P) {
            uint32_t* own = st + P * W;
            const uint32_t* oth = st + (1 - P) * W;
            int y = y0, z = z0, c = c0;
            for (int w = threadIdx.x; w < W; w += blockDim.x) {
                const uint32_t B0 = own[w];
                uint32_t S = B0 & m1;
                const uint32_t u = P == 0 ? unsat_resident<0>(g, oth, jb, y, z, c, S)
                                          : unsat_resident<1>(g, oth, jb, y, z, c, S);
                if (ALGO == 0) {
                    uint32_t M = (B0 >> 1) & 0x03030303u;
                    const uint32_t t = M + u + 0x05050505u;
                    const uint32_t acc = and_andn(t >> 3, t >> 2, m1);
                    const uint32_t low2 = (acc << 1) + acc;
                    const uint32_t Mn = bitsel(low2, t, M);
                    // dH = 4 (m - m') per accepted move (eq. Creutz), 0 otherwise
                    dE += 4 * ((int)__builtin_amdgcn_sad_u8(M, 0u, 0u) - (int)__builtin_amdgcn_sad_u8(Mn, 0u, 0u));
                    own[w] = (S ^ acc) | (Mn << 1);
                } else {
                    // v = #neighbours with J s_nb = -1; the site's unsatisfied count is u = S ? 6 - v : v,
                    // so v = S ? 6 - u : u (bytewise, 6 - u never borrows)
                    const uint32_t mS = (S << 8) - S;
                    const uint32_t vbytes = bitsel(mS, 0x06060606u - u, u);
                    const u32x4 rnd = philox10((uint32_t)w, (uint32_t)(2 * k + P), (uint32_t)r,
                                               canonical_stream<ALGO == 2>((uint32_t)s), g.key0, g.key1);
                    own[w] = canonical4<ALGO == 2>(S, vbytes, rnd, tau, dE);
                }
                // next word of this thread: advance (c, y, z) by blockDim words
                c += dc;
                int adv = drow;
                if (c >= g.Wr) {
                    c -= g.Wr;
                    ++adv;
                }
                y += adv;
                while (y >= g.Ly) {
                    y -= g.Ly;
                    ++z;
                }
            }
            __syncthreads();
        }
        if (rs.log_stride > 0 && (it + 1) % rs.log_stride == 0) {
            // from-scratch energy (unsatisfied bonds, each counted at its even end) and daemon sum
            long long U = 0, D = 0;
            int y = y0, z = z0, c = c0;
            for (int w = threadIdx.x; w < W; w += blockDim.x) {
                const uint32_t S = st[w] & m1;
                U += bytesum(unsat_resident<0>(g, st + W, jb, y, z, c, S));
                D += bytesum((st[w] >> 1) & 0x03030303u) + bytesum((st[W + w] >> 1) & 0x03030303u);
                c += dc;
                int adv = drow;
                if (c >= g.Wr) {
                    c -= g.Wr;
                    ++adv;
                }
                y += adv;
                while (y >= g.Ly) {
                    y -= g.Ly;
                    ++z;
                }
            }
            U = block_sum(U, red);
            D = block_sum(D, red);
            if (threadIdx.x == 0) {
                log[(row_out * n_lattices + l) * 2 + 0] = U;
                log[(row_out * n_lattices + l) * 2 + 1] = D;
            }
            ++row_out;
        }
    }

    uint32_t* spo = reinterpret_cast<uint32_t*>(spin + (int64_t)l * 2 * g.Nh);
    uint32_t* dmo = reinterpret_cast<uint32_t*>(dem + (int64_t)l * 2 * g.Nh);
    for (int w = threadIdx.x; w < 2 * W; w += blockDim.x) {
        spo[w] = (st[w] & m1) | (w < W ? jb[w] << 1 : 0u);
        if (ALGO == 0) dmo[w] = (st[w] >> 1) & 0x03030303u;
    }
    block_add(tally + (int64_t)l * kSlots, dE);
}

template <int ALGO>
__global__ void __launch_bounds__(512) k_resident(Geom g, uint8_t* __restrict__ spin, uint8_t* __restrict__ dem,
                                                  unsigned long long* __restrict__ tally,
                                                  ResidentSched rs, const DaemonThresholds* __restrict__ dth,
                                                  const HeatBathThresholds* __restrict__ hth,
                                                  long long* __restrict__ log)
{
    extern __shared__ uint32_t lds32[];
    __shared__ long long red[16];
    __shared__ uint64_t tau[8];
    resident_body<ALGO>(g, spin, dem, tally, rs, dth, hth, log, blockIdx.x, gridDim.x, lds32, red, tau);
}

// One lattice of some context per work-group: the batched launch of the
// serving pool, where lattices of different sizes, schedules and sweep
// indices advance together (each keeps its own counters and thresholds).
struct ResidentItem {
    Geom g;
    uint8_t* spin;
    uint8_t* dem;
    unsigned long long* tally;
    const DaemonThresholds* dth;
    ResidentSched rs;
    int32_t lattice;
};

__global__ void __launch_bounds__(512) k_resident_batch(const ResidentItem* __restrict__ items)
{
    extern __shared__ uint32_t lds32[];
    __shared__ long long red[16];
    __shared__ uint64_t tau[8];
    const ResidentItem it = items[blockIdx.x];
    resident_body<0>(it.g, it.spin, it.dem, it.tally, it.rs, it.dth, nullptr, nullptr, it.lattice,
                     it.g.S * it.g.R, lds32, red, tau);
}

}  // namespace micsa
