// One launch per MicSA sweep for mid-size byte-layout lattices (too large
// for one work-group's LDS, too few sites to fill the GPU with the z-marching
// fused sweep, e.g. L = 64): a work-group owns one z plane of one lattice,
// with one thread per 4-site word of a plane (Ly * Lx / 8 <= 1024 words).
//
// Both halves of the sweep (Sec. 2.8) run in the work-group:
//   1. every load is issued up front: the old odd words of planes z - 2 ..
//      z + 2, the even words (spins with their six coupling bits) of planes
//      z - 1 .. z + 1 with their daemon words, the odd daemon word of plane z;
//      at a refresh point (Sec. 2.7) the daemons of those even planes and of
//      the odd plane are drawn here instead, with the counters of k_refresh;
//   2. the old odd planes go to LDS; the even half runs on planes z - 1, z,
//      z + 1 (the outer two recomputed from the same old state as their
//      owners, so no work-group waits for another) and leaves the new even
//      words in LDS;
//      a word's x and y neighbours come from LDS, its own column at z and
//      z +- 1 from the thread's registers;
//   3. the odd half runs on plane z with its neighbours' new even words; an
//      odd site's couplings are read from those words (the bond bits ride in
//      the even spin bytes, geometry.hpp).
// State is read from the current arrays and written to the alternate ones.
// The Creutz move is micsa_word (4 sites per 32-bit word, byte-wise).
#pragma once
#include "byte_kernels.hpp"

namespace micsa {

constexpr int kSlabLanes = 1024;

// Neighbourhood of a 4-site word from the other parity's words: w0, up and
// dn the thread's own column at z, z + 1 and z - 1 (registers), src the
// LDS plane at z for the x and y neighbours.
template <int P>
__device__ __forceinline__ Nbhd slab_gather(const Geom& g, uint32_t own, uint32_t w0, uint32_t up, uint32_t dn,
                                            const uint32_t* src, int y, int c, int yp, int ym, int cp, int cm, int q)
{
    const uint32_t m1 = 0x01010101u;
    const int dir = (q ^ P) ? 1 : -1;
    const uint32_t w[6] = {w0, shift_word(w0, src[y * g.Wr + (dir > 0 ? cp : cm)], dir), src[yp * g.Wr + c],
                           src[ym * g.Wr + c], up, dn};
    Nbhd n;
#pragma unroll
    for (int d = 0; d < 6; ++d) n.nb[d] = w[d] & m1;
    const int dA = q ? kMx : kPx, dB = q ? kPx : kMx;
    if (P == 0) {
        const uint32_t jw = own >> 1;
        n.jb[0] = jbits(jw, dA);
        n.jb[1] = jbits(jw, dB);
        n.jb[2] = jbits(jw, kPy);
        n.jb[3] = jbits(jw, kMy);
        n.jb[4] = jbits(jw, kPz);
        n.jb[5] = jbits(jw, kMz);
    } else {  // an odd site reads each bond from its even neighbour's opposite slot
        n.jb[0] = jbits(w[0] >> 1, dA);
        n.jb[1] = jbits(w[1] >> 1, dB);
        n.jb[2] = jbits(w[2] >> 1, kMy);
        n.jb[3] = jbits(w[3] >> 1, kPy);
        n.jb[4] = jbits(w[4] >> 1, kMz);
        n.jb[5] = jbits(w[5] >> 1, kPz);
    }
    return n;
}

template <bool REFRESH>
__global__ __launch_bounds__(kSlabLanes) void k_micsa_slab(Geom g, const uint8_t* __restrict__ spin_in,
                                                          const uint8_t* __restrict__ dem_in,
                                                          uint8_t* __restrict__ spin_out,
                                                          uint8_t* __restrict__ dem_out,
                                                          unsigned long long* __restrict__ tally, uint32_t rho,
                                                          DaemonThresholds th)
{
    extern __shared__ uint32_t lds_slab[];
    const int P = g.Ly * g.Wr;  // 4-site words of one parity in a plane
    uint32_t* LO = lds_slab;          // old odd words, planes z - 2 .. z + 2
    uint32_t* LE = lds_slab + 5 * P;  // new even words, planes z - 1 .. z + 1
    // One-dimensional grid over (lattice, plane); XCD x (block b on XCD b % 8)
    // takes the contiguous planes [x T/8, (x + 1) T/8) when T divides by 8.
    const int nt = gridDim.x;
    int t = blockIdx.x;
    if ((nt & 7) == 0) t = (t & 7) * (nt >> 3) + (t >> 3);
    const int l = t / g.Lz, z0 = t - l * g.Lz;
    const int s = l / g.R, r = l - s * g.R;
    const int pos = threadIdx.x;
    const bool live = pos < P;
    const int pq = live ? pos : 0;  // idle lanes read word 0 (in bounds) and store nothing
    const int y = pq / g.Wr, c = pq - y * g.Wr;
    const int yp = y + 1 == g.Ly ? 0 : y + 1, ym = y == 0 ? g.Ly - 1 : y - 1;
    const int cp = c + 1 == g.Wr ? 0 : c + 1, cm = c == 0 ? g.Wr - 1 : c - 1;
    auto wrapz = [&](int z) { return z < 0 ? z + g.Lz : (z >= g.Lz ? z - g.Lz : z); };
    const int64_t Nh = g.Nh;
    const uint32_t* ev_in = reinterpret_cast<const uint32_t*>(spin_in + (int64_t)l * 2 * Nh);
    const uint32_t* od_in = reinterpret_cast<const uint32_t*>(spin_in + ((int64_t)l * 2 + 1) * Nh);
    const uint32_t* de_in = reinterpret_cast<const uint32_t*>(dem_in + (int64_t)l * 2 * Nh);
    const uint32_t* do_in = reinterpret_cast<const uint32_t*>(dem_in + ((int64_t)l * 2 + 1) * Nh);
    uint32_t* ev_out = reinterpret_cast<uint32_t*>(spin_out + (int64_t)l * 2 * Nh);
    uint32_t* od_out = reinterpret_cast<uint32_t*>(spin_out + ((int64_t)l * 2 + 1) * Nh);
    uint32_t* de_out = reinterpret_cast<uint32_t*>(dem_out + (int64_t)l * 2 * Nh);
    uint32_t* do_out = reinterpret_cast<uint32_t*>(dem_out + ((int64_t)l * 2 + 1) * Nh);
    const uint32_t m1 = 0x01010101u;

    // ---- loads (and draws)
    uint32_t Od[5], Ev[3], Me[3], Mo = 0;
#pragma unroll
    for (int e = 0; e < 5; ++e) Od[e] = od_in[(int64_t)wrapz(z0 - 2 + e) * P + pq];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int64_t w = (int64_t)wrapz(z0 - 1 + e) * P + pq;
        Ev[e] = ev_in[w];
        if (!REFRESH) Me[e] = de_in[w];
    }
    if (!REFRESH) Mo = do_in[(int64_t)z0 * P + pq];
    if (REFRESH) {
        // word w of either parity holds natural sites 8w .. 8w + 7 (the two
        // Philox calls of k_refresh)
        const uint32_t sw = stream_word(kStreamDaemon, (uint32_t)s);
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const int64_t i0 = 8 * ((int64_t)wrapz(z0 - 1 + e) * P + pq);
            const u32x4 a = philox10((uint32_t)(i0 >> 2), rho, (uint32_t)r, sw, g.key0, g.key1);
            const u32x4 b = philox10((uint32_t)(i0 >> 2) + 1u, rho, (uint32_t)r, sw, g.key0, g.key1);
            uint32_t we, wo;
            // sites 8w .. 8w + 7 start at x = 8 (w mod Lx / 8), an even x
            split8q((y + wrapz(z0 - 1 + e)) & 1, a, b, [&](uint32_t u) { return daemon_level(u, th); }, we, wo);
            Me[e] = we;
            if (e == 1) Mo = wo;
        }
    }

    // ---- old odd planes into LDS
    if (live) {
#pragma unroll
        for (int e = 0; e < 5; ++e) LO[e * P + pos] = Od[e];
    }
    __syncthreads();

    int dE = 0;
    uint32_t En[3];  // new even words of planes z - 1, z, z + 1
    // ---- even half on planes z - 1, z, z + 1
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int z = wrapz(z0 - 1 + e);
        const int q = (y + z) & 1;
        const uint32_t W0 = Ev[e];
        const Nbhd n = slab_gather<0>(g, W0, Od[e + 1], Od[e + 2], Od[e], LO + (e + 1) * P, y, c, yp, ym, cp, cm, q);
        const uint32_t S0 = W0 & m1;
        uint32_t S = S0, M = Me[e];
        int d_e = 0;
        micsa_word(S, M, n, d_e);
        const uint32_t Wn = W0 ^ S ^ S0;  // the bond bits stay
        En[e] = Wn;
        if (live) {
            LE[e * P + pos] = Wn;
            if (e == 1) {
                ev_out[(int64_t)z * P + pos] = Wn;
                de_out[(int64_t)z * P + pos] = M;
                dE += d_e;
            }
        }
    }
    __syncthreads();

    // ---- odd half on plane z, with the new even words
    {
        const int z = z0;
        const int q = (y + z) & 1;
        const Nbhd n = slab_gather<1>(g, Od[2], En[1], En[2], En[0], LE + P, y, c, yp, ym, cp, cm, q);
        const uint32_t W0 = Od[2];
        const uint32_t S0 = W0 & m1;
        uint32_t S = S0, M = Mo;
        int d_o = 0;
        micsa_word(S, M, n, d_o);
        if (live) {
            od_out[(int64_t)z * P + pos] = W0 ^ S ^ S0;
            do_out[(int64_t)z * P + pos] = M;
            dE += d_o;
        }
    }
    block_add(tally + (int64_t)l * kSlots, dE);
}

}  // namespace micsa

namespace micsa {

// Two sweeps (A, then B) per launch on the slab layout: the four half sweeps
// A-even, A-odd, B-even, B-odd run on 7, 5, 3 and 1 planes around the owned
// plane z (each ring plane recomputed from the same old state as its owner),
// with the old odd planes z - 4 .. z + 4 and each half's results exchanged
// through LDS, so the state is read and written once per pair of sweeps.
// REFA / REFB: sweep A / B is a refresh point; its levels are drawn in the
// kernel (the counters of k_refresh, refresh index and thresholds per sweep).
struct SlabRefresh {
    uint32_t rho;
    DaemonThresholds th;
};


// DRAW: also draw the levels of a later refresh rn for the owned plane (both
// parities) into dnext (daemon layout), for the launch that will start at
// that refresh; levels depend on the refresh index and temperature only.
template <bool REFA, bool REFB, bool DRAW>
__global__ __launch_bounds__(kSlabLanes) void k_micsa_slab2(Geom g, const uint8_t* __restrict__ spin_in,
                                                           const uint8_t* __restrict__ dem_in,
                                                           uint8_t* __restrict__ spin_out,
                                                           uint8_t* __restrict__ dem_out,
                                                           unsigned long long* __restrict__ tally, SlabRefresh ra,
                                                           SlabRefresh rb, SlabRefresh rn,
                                                           uint8_t* __restrict__ dnext)
{
    static_assert(!(DRAW && (REFA || REFB)), "a launch that draws at a refresh draws nothing ahead");
    extern __shared__ uint32_t lds_slab2[];
    const int P = g.Ly * g.Wr;
    uint32_t* LO = lds_slab2;        // old odd words, planes z - 4 .. z + 4
    uint32_t* LEA = LO + 9 * P;      // A-even results, planes z - 3 .. z + 3
    uint32_t* LOA = LEA + 7 * P;     // A-odd results, planes z - 2 .. z + 2
    uint32_t* LEB = LOA + 5 * P;     // B-even results, planes z - 1 .. z + 1
    const int nt = gridDim.x;
    int t = blockIdx.x;
    if ((nt & 7) == 0) t = (t & 7) * (nt >> 3) + (t >> 3);
    const int l = t / g.Lz, z0 = t - l * g.Lz;
    const int s = l / g.R, r = l - s * g.R;
    const int pos = threadIdx.x;
    const bool live = pos < P;
    const int pq = live ? pos : 0;
    const int y = pq / g.Wr, c = pq - y * g.Wr;
    const int yp = y + 1 == g.Ly ? 0 : y + 1, ym = y == 0 ? g.Ly - 1 : y - 1;
    const int cp = c + 1 == g.Wr ? 0 : c + 1, cm = c == 0 ? g.Wr - 1 : c - 1;
    auto wrapz = [&](int z) {
        z %= g.Lz;
        return z < 0 ? z + g.Lz : z;
    };
    const int64_t Nh = g.Nh;
    const uint32_t* ev_in = reinterpret_cast<const uint32_t*>(spin_in + (int64_t)l * 2 * Nh);
    const uint32_t* od_in = reinterpret_cast<const uint32_t*>(spin_in + ((int64_t)l * 2 + 1) * Nh);
    const uint32_t* de_in = reinterpret_cast<const uint32_t*>(dem_in + (int64_t)l * 2 * Nh);
    const uint32_t* do_in = reinterpret_cast<const uint32_t*>(dem_in + ((int64_t)l * 2 + 1) * Nh);
    uint32_t* ev_out = reinterpret_cast<uint32_t*>(spin_out + (int64_t)l * 2 * Nh);
    uint32_t* od_out = reinterpret_cast<uint32_t*>(spin_out + ((int64_t)l * 2 + 1) * Nh);
    uint32_t* de_out = reinterpret_cast<uint32_t*>(dem_out + (int64_t)l * 2 * Nh);
    uint32_t* do_out = reinterpret_cast<uint32_t*>(dem_out + ((int64_t)l * 2 + 1) * Nh);
    const uint32_t m1 = 0x01010101u;
    const uint32_t sw = stream_word(kStreamDaemon, (uint32_t)s);
    // levels of the even and odd words of plane zz drawn for refresh f
    auto draw = [&](const SlabRefresh& f, int zz, uint32_t& we, uint32_t& wo) {
        const int64_t i0 = 8 * ((int64_t)wrapz(zz) * P + pq);
        const u32x4 a = philox10((uint32_t)(i0 >> 2), f.rho, (uint32_t)r, sw, g.key0, g.key1);
        const u32x4 b = philox10((uint32_t)(i0 >> 2) + 1u, f.rho, (uint32_t)r, sw, g.key0, g.key1);
        // sites 8w .. 8w + 7 start at x = 8 (w mod Lx / 8), an even x
        split8q((y + wrapz(zz)) & 1, a, b, [&](uint32_t u) { return daemon_level(u, f.th); }, we, wo);
    };

    // ---- loads (and the draws of sweep A)
    uint32_t Od[9], Ev[7], Me[7], Mo[5];
#pragma unroll
    for (int e = 0; e < 9; ++e) Od[e] = od_in[(int64_t)wrapz(z0 - 4 + e) * P + pq];
#pragma unroll
    for (int e = 0; e < 7; ++e) {
        const int64_t w = (int64_t)wrapz(z0 - 3 + e) * P + pq;
        Ev[e] = ev_in[w];
        if (!REFA) Me[e] = de_in[w];
    }
    if (!REFA) {
#pragma unroll
        for (int e = 0; e < 5; ++e) Mo[e] = do_in[(int64_t)wrapz(z0 - 2 + e) * P + pq];
    } else {
#pragma unroll
        for (int e = 0; e < 7; ++e) {
            uint32_t we, wo;
            draw(ra, z0 - 3 + e, we, wo);
            Me[e] = we;
            if (e >= 1 && e <= 5) Mo[e - 1] = wo;
        }
    }
    if (live) {
#pragma unroll
        for (int e = 0; e < 9; ++e) LO[e * P + pos] = Od[e];
    }
    __syncthreads();

    int dE = 0;
    // ---- A even: planes z - 3 .. z + 3 (old odd neighbours)
#pragma unroll
    for (int e = 0; e < 7; ++e) {
        const int z = wrapz(z0 - 3 + e);
        const uint32_t* src = LO + (e + 1) * P;
        const Nbhd n = slab_gather<0>(g, Ev[e], Od[e + 1], Od[e + 2], Od[e], src, y, c, yp, ym, cp, cm, (y + z) & 1);
        const uint32_t S0 = Ev[e] & m1;
        uint32_t S = S0;
        int d = 0;
        micsa_word(S, Me[e], n, d);
        Ev[e] ^= S ^ S0;  // the bond bits stay
        if (live) LEA[e * P + pos] = Ev[e];
        if (e == 3) dE += d;
    }
    __syncthreads();
    // ---- A odd: planes z - 2 .. z + 2 (A-even neighbours)
    uint32_t Oa[5];
#pragma unroll
    for (int e = 0; e < 5; ++e) {
        const int z = wrapz(z0 - 2 + e);
        const uint32_t* src = LEA + (e + 1) * P;
        const uint32_t W0 = Od[e + 2];
        const Nbhd n = slab_gather<1>(g, W0, Ev[e + 1], Ev[e + 2], Ev[e], src, y, c, yp, ym, cp, cm, (y + z) & 1);
        const uint32_t S0 = W0 & m1;
        uint32_t S = S0;
        int d = 0;
        micsa_word(S, Mo[e], n, d);
        Oa[e] = W0 ^ S ^ S0;
        if (live) LOA[e * P + pos] = Oa[e];
        if (e == 2) dE += d;
    }
    __syncthreads();
    // ---- B even: planes z - 1 .. z + 1 (A-odd neighbours); levels of B drawn at its refresh
    uint32_t Eb[3], Mb1 = 0;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int z = wrapz(z0 - 1 + e);
        const uint32_t* src = LOA + (e + 1) * P;
        const uint32_t W0 = Ev[e + 2];
        uint32_t M = Me[e + 2];
        if (REFB) {
            uint32_t we, wo;
            draw(rb, z0 - 1 + e, we, wo);
            M = we;
            if (e == 1) Mo[2] = wo;
        }
        const Nbhd n = slab_gather<0>(g, W0, Oa[e + 1], Oa[e + 2], Oa[e], src, y, c, yp, ym, cp, cm, (y + z) & 1);
        const uint32_t S0 = W0 & m1;
        uint32_t S = S0;
        int d = 0;
        micsa_word(S, M, n, d);
        Eb[e] = W0 ^ S ^ S0;
        if (live) LEB[e * P + pos] = Eb[e];
        if (e == 1) {
            Mb1 = M;
            dE += d;
        }
    }
    __syncthreads();
    // ---- B odd: plane z (B-even neighbours)
    {
        const int z = z0;
        const uint32_t* src = LEB + P;
        const uint32_t W0 = Oa[2];
        const Nbhd n = slab_gather<1>(g, W0, Eb[1], Eb[2], Eb[0], src, y, c, yp, ym, cp, cm, (y + z) & 1);
        const uint32_t S0 = W0 & m1;
        uint32_t S = S0, M = Mo[2];
        int d = 0;
        micsa_word(S, M, n, d);
        dE += d;
        if (live) {
            const int64_t w = (int64_t)z * P + pos;
            ev_out[w] = Eb[1];
            de_out[w] = Mb1;
            od_out[w] = W0 ^ S ^ S0;
            do_out[w] = M;
        }
    }
    if (DRAW) {  // last, when the registers of the four halves are free
        uint32_t we, wo;
        draw(rn, z0, we, wo);
        if (live) {
            const int64_t w = (int64_t)z0 * P + pos;
            reinterpret_cast<uint32_t*>(dnext + (int64_t)l * 2 * Nh)[w] = we;
            reinterpret_cast<uint32_t*>(dnext + ((int64_t)l * 2 + 1) * Nh)[w] = wo;
        }
    }
    block_add(tally + (int64_t)l * kSlots, live ? dE : 0);  // idle lanes repeat word 0's moves
}

}  // namespace micsa
