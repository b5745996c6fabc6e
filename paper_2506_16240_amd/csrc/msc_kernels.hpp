// Multispin coding of one lattice (Sec. 2.5: the bits of a word are different
// spins; two bit planes hold the 2-bit daemons): 64 sites of one row and one
// checkerboard parity per 64-bit word, with every step of the Creutz move
// done on whole words by boolean algebra.
//
// Planes of lattice l (all [row][w], row = y + Ly z, w = 0 .. W-1, W = Lx/128;
// bit b of word w is site k = 64 w + b of the row's parity-p sites, at
// x = 2k + ((p + y + z) & 1)):
//   spin[l][p]      spin bits sigma
//   dem0/dem1[l][p] bits 0 and 1 of the daemon level m
//   bond[l][d]      coupling bit j of the bond from each even site in
//                   direction d (+x, -x, +y, -y, +z, -z): every bond has one
//                   even end, so these six planes hold every coupling once
// The planes are a working form of the byte layout: the library packs them
// from the byte arrays at the start of a sweep call and unpacks them at its
// end, so every other entry point reads the byte layout as before.
//
// Neighbours of parity-p site k of a row, in the other parity's planes: y
// and z neighbours at the same k of the adjacent rows; x + 1 at k + q and
// x - 1 at k + q - 1 of the same row (q = (p + y + z) & 1), i.e. the word
// itself or the word shifted by one site with the carry from the adjacent
// word (wrapping around the row).  An odd site's coupling in direction d is
// its even neighbour's coupling in the opposite direction.
//
// Creutz move (Sec. 2.3, 2.5) bit-sliced: the six unsatisfied-bond bits
// s ^ neighbour ^ j are counted into u = (u2 u1 u0) by two carry-save
// adders; w = m + u (four bits); the flip is accepted iff 3 <= w <= 6, i.e.
// iff !w3 and (w2 ^ (w1 & w0)), and then m' = w - 3 = (w2 & (w1 | w0), !w0).
// The energy tally adds dH = 4 (m - m') over the word (conservation).
#pragma once
#include "byte_kernels.hpp"

namespace micsa {

struct MscGeom {
    int32_t W;      // words per row and parity = Lx / 128
    int32_t R;      // rows = Ly * Lz
    int64_t plane;  // words per plane = R * W
};

__device__ __forceinline__ uint64_t shift_next(uint64_t v, uint64_t nxt)  // site k <- site k + 1
{
    return (v >> 1) | (nxt << 63);
}
__device__ __forceinline__ uint64_t shift_prev(uint64_t v, uint64_t prv)  // site k <- site k - 1
{
    return (v << 1) | (prv >> 63);
}
__device__ __forceinline__ uint64_t maj3(uint64_t a, uint64_t b, uint64_t c) { return (a & b) | (c & (a | b)); }

// Daemon levels of the 64 parity-p sites of word w of a row, drawn as in
// the byte layout: site i = x + Lx row takes word i & 3 of Philox (i >> 2,
// rho, replica, 3 << 24 | sample); sites k and k + 1 (k even) share a call.
__device__ __forceinline__ void msc_draw(const Geom& g, int row, int w, int q, uint32_t rho, uint32_t r,
                                         uint32_t sw, const DaemonThresholds& th, uint64_t& m0, uint64_t& m1)
{
    m0 = 0;
    m1 = 0;
    const uint32_t base = (uint32_t)(((int64_t)g.Lx * row) >> 2);
#pragma unroll 4
    for (int b = 0; b < 64; b += 2) {
        const int k = 64 * w + b;  // even: x = 2k + q and 2k + 2 + q fall in one group of four
        const u32x4 o = philox10(base + (uint32_t)(k >> 1), rho, r, sw, g.key0, g.key1);
        const uint32_t ua = q ? o.v1 : o.v0, ub = q ? o.v3 : o.v2;
        const uint32_t la = daemon_level(ua, th), lb = daemon_level(ub, th);
        m0 |= (uint64_t)((la & 1u) | ((lb & 1u) << 1)) << b;
        m1 |= (uint64_t)((la >> 1) | ((lb >> 1) << 1)) << b;
    }
}

// One half sweep (parity P) of every lattice, in place: the half writes
// only its own parity's planes and reads the other parity's.
// Grid (ceil(plane / 256), L), block 256.
template <int P, bool REFRESH>
__global__ __launch_bounds__(256) void k_msc_half(Geom g, MscGeom m, uint64_t* __restrict__ spin,
                                                  uint64_t* __restrict__ dem0, uint64_t* __restrict__ dem1,
                                                  const uint64_t* __restrict__ bond,
                                                  unsigned long long* __restrict__ tally, uint32_t rho,
                                                  DaemonThresholds th)
{
    const int l = blockIdx.y;
    const int64_t gw = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    long long dE = 0;
    if (gw < m.plane) {
        const int row = (int)(gw / m.W), w = (int)(gw - (int64_t)row * m.W);
        const int y = row % g.Ly, z = row / g.Ly;
        const int ryp = (y + 1 == g.Ly ? 0 : y + 1) + g.Ly * z, rym = (y == 0 ? g.Ly - 1 : y - 1) + g.Ly * z;
        const int rzp = y + g.Ly * (z + 1 == g.Lz ? 0 : z + 1), rzm = y + g.Ly * (z == 0 ? g.Lz - 1 : z - 1);
        const int wn = w + 1 == m.W ? 0 : w + 1, wp = w == 0 ? m.W - 1 : w - 1;
        const int q = (P + y + z) & 1;
        const uint64_t* own = spin + ((int64_t)l * 2 + P) * m.plane;
        const uint64_t* oth = spin + ((int64_t)l * 2 + (1 - P)) * m.plane;
        const uint64_t* bl = bond + (int64_t)l * 6 * m.plane;
        auto at = [&](int r, int ww) { return (int64_t)r * m.W + ww; };
        auto bp = [&](int d, int r, int ww) { return bl[(int64_t)d * m.plane + at(r, ww)]; };

        const int64_t me = at(row, w);
        const uint64_t s = own[me];
        const uint64_t O = oth[me];
        const uint64_t nxp = q ? shift_next(O, oth[at(row, wn)]) : O;
        const uint64_t nxm = q ? O : shift_prev(O, oth[at(row, wp)]);
        const uint64_t nyp = oth[at(ryp, w)], nym = oth[at(rym, w)];
        const uint64_t nzp = oth[at(rzp, w)], nzm = oth[at(rzm, w)];
        uint64_t jxp, jxm, jyp, jym, jzp, jzm;
        if (P == 0) {
            jxp = bp(kPx, row, w);
            jxm = bp(kMx, row, w);
            jyp = bp(kPy, row, w);
            jym = bp(kMy, row, w);
            jzp = bp(kPz, row, w);
            jzm = bp(kMz, row, w);
        } else {  // the even neighbour's coupling in the opposite direction
            const uint64_t Mx = bp(kMx, row, w), Px = bp(kPx, row, w);
            jxp = q ? shift_next(Mx, bp(kMx, row, wn)) : Mx;
            jxm = q ? Px : shift_prev(Px, bp(kPx, row, wp));
            jyp = bp(kMy, ryp, w);
            jym = bp(kPy, rym, w);
            jzp = bp(kMz, rzp, w);
            jzm = bp(kPz, rzm, w);
        }
        // unsatisfied-bond bits and their count u (carry-save adders)
        const uint64_t a = s ^ nxp ^ jxp, b = s ^ nxm ^ jxm, c = s ^ nyp ^ jyp;
        const uint64_t d = s ^ nym ^ jym, e = s ^ nzp ^ jzp, f = s ^ nzm ^ jzm;
        const uint64_t s1 = a ^ b ^ c, c1 = maj3(a, b, c);
        const uint64_t s2 = d ^ e ^ f, c2 = maj3(d, e, f);
        const uint64_t u0 = s1 ^ s2, k0 = s1 & s2;
        const uint64_t u1 = c1 ^ c2 ^ k0, u2 = maj3(c1, c2, k0);
        uint64_t m0, m1;
        uint64_t* d0 = dem0 + ((int64_t)l * 2 + P) * m.plane;
        uint64_t* d1 = dem1 + ((int64_t)l * 2 + P) * m.plane;
        if (REFRESH) {
            msc_draw(g, row, w, q, rho, (uint32_t)(l % g.R), stream_word(kStreamDaemon, (uint32_t)(l / g.R)), th,
                     m0, m1);
        } else {
            m0 = d0[me];
            m1 = d1[me];
        }
        // w = m + u, accept iff 3 <= w <= 6, m' = w - 3
        const uint64_t w0 = m0 ^ u0, cw0 = m0 & u0;
        const uint64_t w1 = m1 ^ u1 ^ cw0, cw1 = maj3(m1, u1, cw0);
        const uint64_t w2 = u2 ^ cw1, w3 = u2 & cw1;
        const uint64_t acc = ~w3 & (w2 ^ (w1 & w0));
        const uint64_t n0 = (acc & ~w0) | (~acc & m0);
        const uint64_t n1 = (acc & (w2 & (w1 | w0))) | (~acc & m1);
        spin[((int64_t)l * 2 + P) * m.plane + me] = s ^ acc;
        d0[me] = n0;
        d1[me] = n1;
        dE = 4ll * ((long long)__popcll(m0) + 2ll * __popcll(m1) - __popcll(n0) - 2ll * __popcll(n1));
    }
    block_add(tally + (int64_t)l * kSlots, dE);
}

// Byte layout -> planes (and back): one thread per (lattice, parity, row,
// word), 64 consecutive bytes of the parity array.  An even spin byte holds
// the spin in bit 0 and the coupling of direction d in bit 1 + d.
__global__ __launch_bounds__(256) void k_msc_pack(Geom g, MscGeom m, const uint8_t* __restrict__ spin_b,
                                                  const uint8_t* __restrict__ dem_b, uint64_t* __restrict__ spin,
                                                  uint64_t* __restrict__ dem0, uint64_t* __restrict__ dem1,
                                                  uint64_t* __restrict__ bond)
{
    const int64_t gw = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int l = blockIdx.y;
    if (gw >= 2 * m.plane) return;
    const int p = (int)(gw / m.plane);
    const int64_t pw = gw - p * m.plane;  // row * W + w: its 64 bytes start at byte 64 pw of the parity array
    const uint8_t* sb = spin_b + ((int64_t)l * 2 + p) * g.Nh + 64 * pw;
    const uint8_t* db = dem_b + ((int64_t)l * 2 + p) * g.Nh + 64 * pw;
    uint64_t s = 0, m0 = 0, m1 = 0, j[6] = {0, 0, 0, 0, 0, 0};
    for (int v = 0; v < 4; ++v) {
        const uint4 S4 = reinterpret_cast<const uint4*>(sb)[v];
        const uint4 D4 = reinterpret_cast<const uint4*>(db)[v];
        const uint32_t sw[4] = {S4.x, S4.y, S4.z, S4.w}, dw[4] = {D4.x, D4.y, D4.z, D4.w};
        for (int t = 0; t < 16; ++t) {
            const int b = 16 * v + t;
            const uint32_t sbyte = (sw[t >> 2] >> (8 * (t & 3))) & 0xFFu;
            const uint32_t dbyte = (dw[t >> 2] >> (8 * (t & 3))) & 0xFFu;
            s |= (uint64_t)(sbyte & 1u) << b;
            m0 |= (uint64_t)(dbyte & 1u) << b;
            m1 |= (uint64_t)((dbyte >> 1) & 1u) << b;
            if (p == 0)
                for (int d = 0; d < 6; ++d) j[d] |= (uint64_t)((sbyte >> (1 + d)) & 1u) << b;
        }
    }
    spin[((int64_t)l * 2 + p) * m.plane + pw] = s;
    dem0[((int64_t)l * 2 + p) * m.plane + pw] = m0;
    dem1[((int64_t)l * 2 + p) * m.plane + pw] = m1;
    if (p == 0)
        for (int d = 0; d < 6; ++d) bond[((int64_t)l * 6 + d) * m.plane + pw] = j[d];
}

__global__ __launch_bounds__(256) void k_msc_unpack(Geom g, MscGeom m, const uint64_t* __restrict__ spin,
                                                    const uint64_t* __restrict__ dem0,
                                                    const uint64_t* __restrict__ dem1,
                                                    const uint64_t* __restrict__ bond, uint8_t* __restrict__ spin_b,
                                                    uint8_t* __restrict__ dem_b)
{
    const int64_t gw = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int l = blockIdx.y;
    if (gw >= 2 * m.plane) return;
    const int p = (int)(gw / m.plane);
    const int64_t pw = gw - p * m.plane;
    const uint64_t s = spin[((int64_t)l * 2 + p) * m.plane + pw];
    const uint64_t m0 = dem0[((int64_t)l * 2 + p) * m.plane + pw];
    const uint64_t m1 = dem1[((int64_t)l * 2 + p) * m.plane + pw];
    uint64_t j[6] = {0, 0, 0, 0, 0, 0};
    if (p == 0)
        for (int d = 0; d < 6; ++d) j[d] = bond[((int64_t)l * 6 + d) * m.plane + pw];
    uint8_t* sb = spin_b + ((int64_t)l * 2 + p) * g.Nh + 64 * pw;
    uint8_t* db = dem_b + ((int64_t)l * 2 + p) * g.Nh + 64 * pw;
    for (int v = 0; v < 4; ++v) {
        uint32_t sw[4] = {0, 0, 0, 0}, dw[4] = {0, 0, 0, 0};
        for (int t = 0; t < 16; ++t) {
            const int b = 16 * v + t;
            uint32_t sbyte = (uint32_t)((s >> b) & 1u);
            for (int d = 0; d < 6; ++d) sbyte |= (uint32_t)((j[d] >> b) & 1u) << (1 + d);
            const uint32_t dbyte = (uint32_t)((m0 >> b) & 1u) | ((uint32_t)((m1 >> b) & 1u) << 1);
            sw[t >> 2] |= sbyte << (8 * (t & 3));
            dw[t >> 2] |= dbyte << (8 * (t & 3));
        }
        reinterpret_cast<uint4*>(sb)[v] = make_uint4(sw[0], sw[1], sw[2], sw[3]);
        reinterpret_cast<uint4*>(db)[v] = make_uint4(dw[0], dw[1], dw[2], dw[3]);
    }
}

}  // namespace micsa
