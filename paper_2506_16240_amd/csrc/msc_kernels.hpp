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

// Daemon levels of both parities' words w of a row at a refresh: the Philox
// call of sites x = 4a .. 4a + 3 serves even sites k = 2a, 2a + 1 (words i & 3
// = q, 2 + q, q = x offset of the row's even sites) and odd sites k = 2a,
// 2a + 1 (words 1 - q, 3 - q) of the same word index.
__device__ __forceinline__ void msc_draw2(const Geom& g, int row, int w, int q, uint32_t rho, uint32_t r,
                                          uint32_t sw, const DaemonThresholds& th, uint64_t& e0, uint64_t& e1,
                                          uint64_t& o0, uint64_t& o1)
{
    e0 = e1 = o0 = o1 = 0;
    const uint32_t base = (uint32_t)(((int64_t)g.Lx * row) >> 2);
#pragma unroll 2
    for (int b = 0; b < 64; b += 2) {
        const u32x4 v = philox10(base + (uint32_t)((64 * w + b) >> 1), rho, r, sw, g.key0, g.key1);
        const uint32_t ea = daemon_level(q ? v.v1 : v.v0, th), eb = daemon_level(q ? v.v3 : v.v2, th);
        const uint32_t oa = daemon_level(q ? v.v0 : v.v1, th), ob = daemon_level(q ? v.v2 : v.v3, th);
        e0 |= (uint64_t)((ea & 1u) | ((eb & 1u) << 1)) << b;
        e1 |= (uint64_t)((ea >> 1) | ((eb >> 1) << 1)) << b;
        o0 |= (uint64_t)((oa & 1u) | ((ob & 1u) << 1)) << b;
        o1 |= (uint64_t)((oa >> 1) | ((ob >> 1) << 1)) << b;
    }
}

// Three-input XOR and majority of 64-bit words, one v_bitop3 per 32-bit half
// (truth tables 0x96 and 0xE8, the same for any order of the operands).
__device__ __forceinline__ uint64_t xor3(uint64_t a, uint64_t b, uint64_t c)
{
    const uint32_t lo = __builtin_amdgcn_bitop3_b32((uint32_t)a, (uint32_t)b, (uint32_t)c, 0x96);
    const uint32_t hi =
        __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), (uint32_t)(b >> 32), (uint32_t)(c >> 32), 0x96);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}
__device__ __forceinline__ uint64_t maj3w(uint64_t a, uint64_t b, uint64_t c)
{
    const uint32_t lo = __builtin_amdgcn_bitop3_b32((uint32_t)a, (uint32_t)b, (uint32_t)c, 0xE8);
    const uint32_t hi =
        __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), (uint32_t)(b >> 32), (uint32_t)(c >> 32), 0xE8);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// The Creutz move on a word: s the spins, n[] the six neighbour words and j[]
// the six coupling words (+x, -x, +y, -y, +z, -z), m0/m1 the levels (updated);
// returns the new spins and adds the level sums before/after to so/sn.
__device__ __forceinline__ uint64_t msc_move(uint64_t s, const uint64_t (&n)[6], const uint64_t (&j)[6], uint64_t& m0,
                                             uint64_t& m1, long long& so, long long& sn)
{
    const uint64_t a = xor3(s, n[0], j[0]), b = xor3(s, n[1], j[1]), c = xor3(s, n[2], j[2]);
    const uint64_t d = xor3(s, n[3], j[3]), e = xor3(s, n[4], j[4]), f = xor3(s, n[5], j[5]);
    const uint64_t s1 = xor3(a, b, c), c1 = maj3w(a, b, c);
    const uint64_t s2 = xor3(d, e, f), c2 = maj3w(d, e, f);
    const uint64_t u0 = s1 ^ s2, k0 = s1 & s2;
    const uint64_t u1 = xor3(c1, c2, k0), u2 = maj3w(c1, c2, k0);
    const uint64_t w0 = m0 ^ u0, cw0 = m0 & u0;
    const uint64_t w1 = xor3(m1, u1, cw0), cw1 = maj3w(m1, u1, cw0);
    const uint64_t w2 = u2 ^ cw1, w3 = u2 & cw1;
    const uint64_t acc = ~w3 & (w2 ^ (w1 & w0));
    const uint64_t n0 = (acc & ~w0) | (~acc & m0);
    const uint64_t n1 = (acc & (w2 & (w1 | w0))) | (~acc & m1);
    so += (long long)__popcll(m0) + 2ll * __popcll(m1);
    sn += (long long)__popcll(n0) + 2ll * __popcll(n1);
    m0 = n0;
    m1 = n1;
    return s ^ acc;
}

struct MscTile {
    int32_t TY, TZ;  // rows and planes (divides Lz) a work-group owns
    int32_t nty, ntz;
    int32_t xcd;  // 1: tiles numbered XCD by XCD (tiles per lattice divisible by 8);
                  // 2: XCD x takes the z band [x ntz/8, (x + 1) ntz/8) of every y tile (ntz divisible by 8)
};

// One whole sweep per launch (both halves), marching along z like the byte
// layout's fused sweep: at step st, with z = zstart + dz st, the even half
// on plane z and the odd half on plane z - dz, whose even neighbours (planes
// z - 2dz .. z) are then all final.  A work-group owns TY rows (the last tile
// along y what is left of Ly) x TZ planes of one lattice, all words of a
// row; the even half also runs on one ring of rows and planes and odd spins
// are read on two rings, so no tile needs another tile's new values (state
// read from the "in" planes, written to the "out" planes).  Lanes: (TY + 4)
// rows x W words; in-plane neighbours (rows y +- 1, the x carry from words
// w +- 1) come through LDS, one buffer per step parity (old odd spins, new
// even spins and the even sites' x and y couplings of plane z); z neighbours
// through registers.  Each coupling word is read once per sweep.
// REFRESH: the even half draws both parities' levels of its word and keeps
// the odd ones for the next step (used when the levels are not drawn ahead).
// Loads and barriers: every lane issues every load of a step (a lane outside
// a word's rows reads a row of its own tile instead, a line the work-group
// fetches anyway), so that no load sits under a lane-dependent branch; two
// register stages alternate (the loop is unrolled by two), so that a value in
// flight is never copied; each step starts with one explicit wait for the
// stage it uses; and the barrier orders LDS only.  The loads of step st + 1
// are thus in flight through the whole of step st.
// Walkers (WALK > 0): the owed wandering's shift is applied when the levels
// are used, with the carry word of the row's neighbouring word taken from the
// lane that loaded it (WALK = 1; needs Lx / 128 to divide 64, so that a row's
// lanes share a wave) or loaded beside the word (WALK = 2).
// Grid (nty * ntz, L); block 64 ceil((TY + 4) W / 64) <= kMscSweepLanes;
// LDS 96 (TY + 4) W bytes.
struct MscStage {
    uint64_t O, Es, J[6], me0, me1, mo0, mo1;
    uint64_t mc0, mc1, oc0, oc1;  // WALK = 2: carry words of the even and odd levels
};

constexpr int kMscSweepLanes = 256;  // largest work-group of the one-launch sweep (its register budget)

template <bool REFRESH, int WALK>
__global__ __launch_bounds__(kMscSweepLanes, 3) void k_msc_sweep(
    Geom g, MscGeom m, MscTile f, const uint64_t* __restrict__ spin_in, const uint64_t* __restrict__ d0_in,
    const uint64_t* __restrict__ d1_in, const uint64_t* __restrict__ bond, uint64_t* __restrict__ spin_out,
    uint64_t* __restrict__ d0_out, uint64_t* __restrict__ d1_out, unsigned long long* __restrict__ tally,
    uint32_t rho, DaemonThresholds th, int wander)
{
    static_assert(!(REFRESH && WALK), "a refresh sweep owes no wandering");
    static_assert(WALK >= 0 && WALK <= 2, "WALK: 0 none, 1 carry by shuffle, 2 carry loaded");
    // issue ahead of the refresh draw that runs beside the sweeps (its waves
    // keep the default priority 0 and fill the slots the sweep leaves while it
    // waits on memory)
    __builtin_amdgcn_s_setprio(1);
    extern __shared__ uint64_t lds64[];
    const int W = m.W;
    const int rows_slots = f.TY + 4;
    const int ps = rows_slots * W;
    // LDS planes per step buffer: 0 odd, 1 even, 2 Mx, 3 Px, 4 My, 5 Py
    auto LP = [&](int buf, int k) { return lds64 + ((size_t)buf * 6 + k) * ps; };

    const int l = blockIdx.y;
    // Work-groups go round-robin over the 8 XCDs (block b on XCD b % 8), each
    // with its own L2; with xcd set XCD x takes the contiguous tiles [x T/8,
    // (x + 1) T/8) (z fastest), so that neighbouring tiles, which read each
    // other's ring rows and planes at the same time (the z direction of the
    // march alternates from tile to tile), share an L2.
    int t = blockIdx.x, ty, tz;
    if (f.xcd == 2) {  // every y-neighbour and all but one z-neighbour in 8 on the same XCD
        const int band = f.ntz >> 3, i = t >> 3;
        ty = i / band;
        tz = (t & 7) * band + (i - ty * band);
    } else {
        if (f.xcd) t = (t & 7) * (f.nty * f.ntz / 8) + (t >> 3);
        ty = t / f.ntz;
        tz = t - ty * f.ntz;
    }
    const int y0 = ty * f.TY, z0 = tz * f.TZ;
    const int dz = (tz & 1) ? -1 : 1;
    const int zstart = dz > 0 ? z0 - 1 : z0 + f.TZ;
    const int ry = threadIdx.x / W, w = threadIdx.x - (threadIdx.x / W) * W;
    const int own = min(f.TY, g.Ly - y0);  // the last tile along y may be shorter
    const bool active = ry < own + 4;
    auto wrap = [](int v, int L) { v %= L; return v < 0 ? v + L : v; };
    const int y = wrap(y0 - 2 + ry, g.Ly);
    const bool do_even = active && ry >= 1 && ry <= own + 2;
    const bool do_odd = active && ry >= 2 && ry <= own + 1;  // the rows the tile owns
    // rows each lane loads from: odd spins on the whole ring, even-site words
    // where the even half runs, odd levels where the odd half runs
    const int yO = wrap(y0 - 2 + min(ry, own + 3), g.Ly);
    const int yE = wrap(y0 - 2 + min(max(ry, 1), own + 2), g.Ly);
    const int yD = wrap(y0 - 2 + min(max(ry, 2), own + 1), g.Ly);
    const int wn = w + 1 == W ? 0 : w + 1, wp = w == 0 ? W - 1 : w - 1;
    const int me = ry * W + w;

    // Addresses: a uniform base per plane (scalar registers) and a 32-bit
    // word offset within the plane (the plane holds fewer than 2^29 words),
    // the lane's row part fixed and the z part uniform per step.
    const int64_t lp = (int64_t)l * 2 * m.plane;  // parity-0 plane of lattice l
    const uint64_t* ev_in = spin_in + lp;
    const uint64_t* od_in = spin_in + lp + m.plane;
    const uint64_t* bl = bond + (int64_t)l * 6 * m.plane;
    const uint32_t zstride = (uint32_t)(g.Ly * W);
    const uint32_t rO = (uint32_t)(yO * W + w), rE = (uint32_t)(yE * W + w), rD = (uint32_t)(yD * W + w),
                   rY = (uint32_t)(y * W + w);
    auto zoff = [&](int zz) { return (uint32_t)zz * zstride; };
    auto ld = [](const uint64_t* base, uint32_t i) {
        return *reinterpret_cast<const uint64_t*>(reinterpret_cast<const char*>(base) + (i << 3));
    };
    auto st8 = [](uint64_t* base, uint32_t i, uint64_t v) {
        *reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(base) + (i << 3)) = v;
    };
    const uint32_t rr = (uint32_t)(l % g.R), sw = stream_word(kStreamDaemon, (uint32_t)(l / g.R));
    const int steps = f.TZ + 2;

    uint64_t O_prev = ld(od_in, zoff(wrap(zstart - dz, g.Lz)) + rO);  // old odd spins at z - dz, z, z + dz
    uint64_t O_cur = ld(od_in, zoff(wrap(zstart, g.Lz)) + rO);
    uint64_t O_next = 0;
    uint64_t E0 = 0, E1 = 0, E2 = 0;     // new even spins at z, z - dz, z - 2dz
    uint64_t MZ0 = 0, MZ1 = 0, MZ2 = 0;  // even couplings -z at z, z - dz, z - 2dz
    uint64_t PZ0 = 0, PZ1 = 0, PZ2 = 0;  // even couplings +z at the same planes
    uint64_t Go0 = 0, Go1 = 0;           // REFRESH: drawn odd levels of plane z - dz
    // Walkers (Sec. 2.6): with WALK the input levels still owe the forward-X
    // wandering of the sites of parity wander (the previous timestep's).  In
    // a row whose even sites sit at x = 2k + q, even site k pairs with odd
    // site k + q (wander = 0), odd site k with even site k + 1 - q (wander =
    // 1): the levels move by 0 or +-1 site across the two parities' planes,
    // with the carry from the neighbouring word of the row.
    auto carry = [&](int sh) { return (uint32_t)(sh > 0 ? wn - w : wp - w); };  // modulo 2^32
    auto shifted = [](uint64_t v, uint64_t c, int sh) {
        return sh > 0 ? shift_next(v, c) : sh < 0 ? shift_prev(v, c) : v;
    };
    // the loads of step st2 into a register stage
    auto load = [&](int st2, MscStage& S) {
        const int zz2 = zstart + dz * st2;
        const int z2 = wrap(zz2, g.Lz);
        S.O = ld(od_in, zoff(wrap(zz2 + dz, g.Lz)) + rO);
        const uint32_t h = zoff(z2) + rE;
        S.Es = ld(ev_in, h);
#pragma unroll
        for (int d = 0; d < 6; ++d) S.J[d] = ld(bl + (int64_t)d * m.plane, h);
        if (!REFRESH) {
            // even levels of plane z2 (walkers: from the odd planes); odd
            // levels of plane z2 - dz (walkers: from the even planes), which
            // before the first odd step repeat the even-level words
            const int64_t pe = lp + (WALK ? m.plane : 0);
            const bool odd_ok = st2 >= 2;
            const int zo2 = wrap(zz2 - dz, g.Lz);
            const int64_t po = odd_ok ? lp + (WALK ? 0 : m.plane) : pe;
            const uint32_t ho = odd_ok ? zoff(zo2) + rD : h;
            S.me0 = ld(d0_in + pe, h);
            S.me1 = ld(d1_in + pe, h);
            S.mo0 = ld(d0_in + po, ho);
            S.mo1 = ld(d1_in + po, ho);
            if (WALK == 2) {
                const int qe = (yE + z2) & 1, qo = (yD + zo2) & 1;
                const uint32_t hec = h + carry(wander == 0 ? qe : qe - 1);
                const uint32_t hoc = ho + carry(wander == 0 ? -qo : 1 - qo);
                S.mc0 = ld(d0_in + pe, hec);
                S.mc1 = ld(d1_in + pe, hec);
                S.oc0 = ld(d0_in + po, hoc);
                S.oc1 = ld(d1_in + po, hoc);
            }
        }
    };
    long long so = 0, sn = 0;
    // step st: consumes stage S (loaded during step st - 1), loads step st + 1 into N
    auto step = [&](int st, MscStage& S, MscStage& N) {
        // stage S is complete here: waiting for it once, unconditionally, lets
        // the compiler see that no load of S is pending inside the branches
        // below (vmcnt(0); expcnt and lgkmcnt left at their maximum)
        __builtin_amdgcn_s_waitcnt(0x0F70);
        const int buf = st & 1, pb = buf ^ 1;
        const int zz = zstart + dz * st;  // unwrapped: owned iff in [z0, z0 + TZ)
        const int z = wrap(zz, g.Lz), zo = wrap(zz - dz, g.Lz);
        const bool own_e = zz >= z0 && zz < z0 + f.TZ, own_o = zz - dz >= z0 && zz - dz < z0 + f.TZ;
        const bool odd_now = do_odd && st >= 2;
        O_next = S.O;
        uint64_t Es = S.Es, J[6], me0 = S.me0, me1 = S.me1, mo0 = S.mo0, mo1 = S.mo1, Gn0 = 0, Gn1 = 0;
#pragma unroll
        for (int d = 0; d < 6; ++d) J[d] = S.J[d];
        if (WALK) {
            const int qe = (y + z) & 1, qo = (y + zo) & 1;
            const int she = wander == 0 ? qe : qe - 1, sho = wander == 0 ? -qo : 1 - qo;
            uint64_t mc0 = S.mc0, mc1 = S.mc1, oc0 = S.oc0, oc1 = S.oc1;
            if (WALK == 1) {  // every lane of the row holds its own word of the same row
                const int re = (ry * W + (she > 0 ? wn : wp)) & 63, ro = (ry * W + (sho > 0 ? wn : wp)) & 63;
                mc0 = __shfl(me0, re, 64);
                mc1 = __shfl(me1, re, 64);
                oc0 = __shfl(mo0, ro, 64);
                oc1 = __shfl(mo1, ro, 64);
            }
            me0 = shifted(me0, mc0, she);
            me1 = shifted(me1, mc1, she);
            mo0 = shifted(mo0, oc0, sho);
            mo1 = shifted(mo1, oc1, sho);
        }
        if (st + 1 < steps) load(st + 1, N);
        if (do_even) {
            if (REFRESH) msc_draw2(g, y + g.Ly * z, w, (y + z) & 1, rho, rr, sw, th, me0, me1, Gn0, Gn1);
            MZ0 = J[kMz];
            PZ0 = J[kPz];
        }
        if (REFRESH && odd_now) {
            mo0 = Go0;
            mo1 = Go1;
        }
        // buffer buf was last read as the previous buffer by step st - 1's odd
        // half: the odd spins go in before this step's barrier (their readers
        // are this step's even half), everything step st + 1 reads after it
        if (active) LP(buf, 0)[me] = O_cur;
        lds_barrier();
        if (do_even) {  // ---- even half on plane z (old odd neighbours)
            LP(buf, 2)[me] = J[kMx];
            LP(buf, 3)[me] = J[kPx];
            LP(buf, 4)[me] = J[kMy];
            LP(buf, 5)[me] = J[kPy];
            const int q = (y + z) & 1;
            const uint64_t* Op = LP(buf, 0);
            const uint64_t nxp = q ? shift_next(O_cur, Op[ry * W + wn]) : O_cur;
            const uint64_t nxm = q ? O_cur : shift_prev(O_cur, Op[ry * W + wp]);
            const uint64_t nyp = Op[me + W], nym = Op[me - W];
            const uint64_t nzp = dz > 0 ? O_next : O_prev, nzm = dz > 0 ? O_prev : O_next;
            long long a = 0, b = 0;
            const uint64_t nb[6] = {nxp, nxm, nyp, nym, nzp, nzm};
            const uint64_t jb[6] = {J[kPx], J[kMx], J[kPy], J[kMy], J[kPz], J[kMz]};
            E0 = msc_move(Es, nb, jb, me0, me1, a, b);
            LP(buf, 1)[me] = E0;
            if (do_odd && own_e) {
                const uint32_t h = zoff(z) + rY;
                st8(spin_out + lp, h, E0);
                st8(d0_out + lp, h, me0);
                st8(d1_out + lp, h, me1);
                so += a;
                sn += b;
            }
        }
        if (odd_now) {  // ---- odd half on plane zo = z - dz (new even neighbours)
            const int q = (1 + y + zo) & 1;
            const uint64_t* Ep = LP(pb, 1);
            const uint64_t Ec = Ep[me];
            const uint64_t nxp = q ? shift_next(Ec, Ep[ry * W + wn]) : Ec;
            const uint64_t nxm = q ? Ec : shift_prev(Ec, Ep[ry * W + wp]);
            const uint64_t nyp = Ep[me + W], nym = Ep[me - W];
            const uint64_t nzp = dz > 0 ? E0 : E2, nzm = dz > 0 ? E2 : E0;
            // an odd site's coupling in direction d is its even neighbour's in direction -d
            const uint64_t* Mx = LP(pb, 2);
            const uint64_t* Px = LP(pb, 3);
            const uint64_t jxp = q ? shift_next(Mx[me], Mx[ry * W + wn]) : Mx[me];
            const uint64_t jxm = q ? Px[me] : shift_prev(Px[me], Px[ry * W + wp]);
            const uint64_t jyp = LP(pb, 4)[me + W], jym = LP(pb, 5)[me - W];
            const uint64_t jzp = dz > 0 ? MZ0 : MZ2, jzm = dz > 0 ? PZ2 : PZ0;
            long long a = 0, b = 0;
            const uint64_t nb[6] = {nxp, nxm, nyp, nym, nzp, nzm};
            const uint64_t jb[6] = {jxp, jxm, jyp, jym, jzp, jzm};
            const uint64_t On = msc_move(O_prev, nb, jb, mo0, mo1, a, b);
            if (own_o) {
                const uint32_t ho = zoff(zo) + rY;
                st8(spin_out + lp + m.plane, ho, On);
                st8(d0_out + lp + m.plane, ho, mo0);
                st8(d1_out + lp + m.plane, ho, mo1);
                so += a;
                sn += b;
            }
        }
        O_prev = O_cur;
        O_cur = O_next;
        E2 = E1;
        E1 = E0;
        MZ2 = MZ1;
        MZ1 = MZ0;
        PZ2 = PZ1;
        PZ1 = PZ0;
        Go0 = Gn0;
        Go1 = Gn1;
    };
    MscStage SA = {}, SB = {};
    load(0, SA);
    for (int st = 0; st < steps; st += 2) {
        step(st, SA, SB);
        if (st + 1 < steps) step(st + 1, SB, SA);
    }
    block_add(tally + (int64_t)l * kSlots, 4 * (so - sn));
}

// Daemon levels of a refresh sweep drawn ahead into planes of the working
// layout: both parities of every word, with the same Philox counters as the
// sweep's own draw.  The levels of a refresh depend on its index and
// temperature only, not on the state, so they can be drawn while the sweeps
// before that refresh run; the refresh sweep then reads them in place of the
// stored levels.  Grid-stride over every (lattice, row, word); block 64.
__global__ __launch_bounds__(64) void k_msc_draw(Geom g, MscGeom m, int32_t L, uint64_t* __restrict__ d0,
                                                 uint64_t* __restrict__ d1, uint32_t rho, DaemonThresholds th)
{
    const int64_t total = (int64_t)L * m.plane;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int l = (int)(i / m.plane);
        const int64_t pw = i - (int64_t)l * m.plane;
        const int row = (int)(pw / m.W), w = (int)(pw - (int64_t)row * m.W);
        const int y = row % g.Ly, z = row / g.Ly;
        uint64_t e0, e1, o0, o1;
        msc_draw2(g, row, w, (y + z) & 1, rho, (uint32_t)(l % g.R), stream_word(kStreamDaemon, (uint32_t)(l / g.R)),
                  th, e0, e1, o0, o1);
        const int64_t he = (int64_t)l * 2 * m.plane + pw, ho = he + m.plane;
        d0[he] = e0;
        d1[he] = e1;
        d0[ho] = o0;
        d1[ho] = o1;
    }
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
