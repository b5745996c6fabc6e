// Several MicSA sweeps per pass over the multispin planes (msc_kernels.hpp):
// T consecutive sweeps -- 2T half sweeps, even and odd alternating (Sec.
// 2.8) -- in one launch that reads and writes the state once, so the HBM
// traffic of a sweep drops by T.
//
// Dependency cone.  Half h of the pass (h = 0 .. 2T-1: sweep h / 2, parity
// h & 1) needs the results of half h - 1 at the six neighbours of each site,
// and its own site's value from half h - 2.  A work-group that owns TY rows
// and TZ planes therefore computes half h on a ring of 2T - 1 - h extra rows
// and planes on each side (recomputed from the same old state as the
// neighbouring tile, so no work-group waits for another), and loads the old
// odd spins on a ring of 2T rows and planes.  Lanes: (TY + 4T) rows x W
// words.
//
// March along z (as the one-sweep kernel): at step st, with z = zstart + dz
// st, half h works on plane z - dz h.  Half h's inputs are then at hand:
// half h - 1's results of planes z - dz h +- 1 are this step's and the step
// before last's (registers), its results in plane z - dz h (the in-plane
// neighbours: rows y +- 1, the x carry words) were written to LDS by the
// step before, and half h - 2's result at the site itself two steps ago
// (registers).  The even sites' couplings of the last 2T + 1 planes sit in
// an LDS ring (the odd halves take an odd site's bond from its even
// neighbour, in-plane and along z).  Each step writes the old odd plane and
// every half's result plane to the LDS buffer of its step parity, one
// barrier per step.  Half h is needed from step 2h on; the step count is
// TZ + 4T - 2.
//
// Refresh: the levels of a refresh sweep are drawn ahead (k_msc_draw) and
// read in place of the stored ones -- by the host passing the drawn planes
// as the input levels when the first sweep of the pass refreshes, and by
// the kernel loading them for halves 2 RJ and 2 RJ + 1 when sweep RJ >= 1 of
// the pass refreshes (RJ < 0: none does).
//
// Walkers (WALK; Sec. 2.6, forward-X wandering; a row's lanes share a wave,
// Lx / 128 dividing 64): the levels move by 0 or +-1 site across the two
// parities' planes at the end of each timestep.  The wandering owed from
// before the pass (parity `wander`, -1 none) is applied as halves 0 and 1
// load their levels, from the other parity's planes, as the one-sweep kernel
// does; that of the pass's first sweep (parity `wanderA`, -1 when the second
// sweep refreshes) moves half 1's levels of the step before into half 2 and
// half 0's levels of three steps before into half 3.  The carry word of a
// shift comes from the neighbouring lane of the row by a shuffle.  The pass
// leaves its second sweep's wandering owed.
//
// Energy tally: 4 (sum m - sum m') of every half on the owned sites.  Half
// h >= 2 starts from the levels half h - 2 left at the same site, so the sum
// telescopes: the levels going into halves 0 and 1, minus those leaving the
// last two halves, plus, at a refresh half, the drawn levels minus those
// they replace.  Walkers move levels only within a row, cyclically, and a
// tile owns whole rows of a plane, so the sum over a row's two parities
// that the next half starts from is the sum the half before left, and the
// same telescoped count holds.
//
// Cost per step.  Every lane runs every half that has started (lanes outside
// a half's rows compute values nobody reads: the rows a half reads are the
// rows its predecessor got right); only the stores and the tally look at
// ownership.  Plane indices along z move by one per step and are wrapped by
// a compare, so no step divides; the march is unrolled by six steps, so the
// three-step histories of the half results and the two register stages
// rotate by renaming, and the coupling ring's slot is the step's phase.
// The z couplings are loaded in march orientation (word 4 towards z + dz,
// word 5 towards z - dz), so no half selects by direction, and the shifted
// x neighbours are funnel shifts by the row's parity offset.
//
// LDS, lane-major: lane t owns the kMsc2Words words from t kMsc2Words on,
// its word of each plane -- the 4T result planes (two step buffers) and six
// coupling planes for each of six ring slots, slot st mod 6 written at step
// st (six slots, one more than the ring needs, so that the slot is the
// step's phase in the unrolled march) -- an odd number of 64-bit words, so
// that a wave's 64-bit reads at consecutive lanes fall in distinct banks.
// Every LDS address is then one of five per-lane registers (the lane's word
// and its x and y neighbours') plus a constant.
//
// Grid (nty * ntz, L); block B = 64 ceil((TY + 4T) W / 64) <= kMsc2Lanes;
// LDS 8 kMsc2Words (B + W) bytes (the slack W keeps the neighbour reads of
// the last lanes inside).
#pragma once
#include <type_traits>
#include "msc_kernels.hpp"

namespace micsa {

constexpr int kMsc2Lanes = 256;
constexpr int kMsc2Words = 45;  // LDS words per lane: 8 result planes + 6 x 6 coupling planes, made odd

template <bool DRAWN>
struct Msc2Stage {
    uint64_t O, Es, J[6], me0, me1, mo0, mo1;
};
template <>
struct Msc2Stage<true> {
    uint64_t O, Es, J[6], me0, me1, mo0, mo1;
    uint64_t re0, re1, ro0, ro1;  // drawn levels for the halves of the refresh sweep RJ
};

// A wrapped index moved by dz = +-1 along an axis of length L.
__device__ __forceinline__ int step_wrap(int v, int dz, int L)
{
    v += dz;
    return v == L ? 0 : (v < 0 ? L - 1 : v);
}

// The Creutz move of msc_move with the gates of a 32-bit half fused into
// three-input v_bitop3 operations (24 per half instead of about 30), every
// truth table symmetric in its first and third operands.  With x0 = ~w0
// (w0 = m0 ^ s1 ^ s2, the sum bit of m + u): cw0 = m0 & (s1 ^ s2), the
// carry into bit 1; acc = !w3 & (w2 ^ (w1 & w0)) with w2 = u2 ^ cw1 and
// w3 = u2 & cw1; m' = acc ? (w2 & (w1 | w0), ~w0) : (m1, m0).
template <int TT>
__device__ __forceinline__ uint64_t b3(uint64_t a, uint64_t b, uint64_t c)
{
    const uint32_t lo = __builtin_amdgcn_bitop3_b32((uint32_t)a, (uint32_t)b, (uint32_t)c, TT);
    const uint32_t hi = __builtin_amdgcn_bitop3_b32((uint32_t)(a >> 32), (uint32_t)(b >> 32), (uint32_t)(c >> 32), TT);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}
__device__ __forceinline__ uint64_t msc_move_fused(uint64_t s, const uint64_t (&n)[6], const uint64_t (&j)[6],
                                                   uint64_t& m0, uint64_t& m1)
{
    const uint64_t a = xor3(s, n[0], j[0]), b = xor3(s, n[1], j[1]), c = xor3(s, n[2], j[2]);
    const uint64_t d = xor3(s, n[3], j[3]), e = xor3(s, n[4], j[4]), f = xor3(s, n[5], j[5]);
    const uint64_t s1 = xor3(a, b, c), c1 = maj3w(a, b, c);
    const uint64_t s2 = xor3(d, e, f), c2 = maj3w(d, e, f);
    const uint64_t k0 = s1 & s2;
    const uint64_t u1 = xor3(c1, c2, k0), u2 = maj3w(c1, c2, k0);
    const uint64_t x0 = b3<0x69>(s1, m0, s2);   // ~(m0 ^ s1 ^ s2) = ~w0
    const uint64_t cw0 = b3<0x48>(s1, m0, s2);  // m0 & (s1 ^ s2)
    const uint64_t w1 = xor3(m1, u1, cw0), cw1 = maj3w(m1, u1, cw0);
    const uint64_t p = b3<0x30>(w1, x0, w1);    // w1 & w0 (first and third operand the same)
    const uint64_t r = b3<0xF3>(w1, x0, w1);    // w1 | w0
    const uint64_t acc = b3<0x16>(u2, p, cw1);  // ~(u2 & cw1) & (u2 ^ cw1 ^ p)
    const uint64_t v = b3<0x48>(u2, r, cw1);    // (u2 ^ cw1) & r
    const uint64_t n0 = (acc & x0) | (~acc & m0);
    const uint64_t n1 = (acc & v) | (~acc & m1);
    m0 = n0;
    m1 = n1;
    return s ^ acc;
}

// v shifted right by q in {0, 1} with bit 0 of nxt moving in at bit 63
// (shift_next for q = 1): two funnel shifts.
__device__ __forceinline__ uint64_t shr_q(uint64_t v, uint64_t nxt, uint32_t q)
{
    const uint32_t vl = (uint32_t)v, vh = (uint32_t)(v >> 32), nl = (uint32_t)nxt;
    const uint32_t lo = __builtin_amdgcn_alignbit(vh, vl, q);
    const uint32_t hi = __builtin_amdgcn_alignbit(nl, vh, q);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}
// v shifted left by t in {0, 1} with bit 63 of prv moving in at bit 0
// (shift_prev for t = 1).
__device__ __forceinline__ uint64_t shl_t(uint64_t v, uint64_t prv, uint32_t t)
{
    return (v << t) | (uint64_t)((uint32_t)(prv >> 63) & t);
}

// The levels of a row moved by amt in {0, 1} sites (the wandering) towards
// lower sites (fwd: site k takes site k + amt, the carry word from the row's
// next lane ln of the wave) or higher ones (site k takes site k - amt, the
// carry from the previous lane lp).  The direction is uniform in a step,
// the amount the row's parity offset.
__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src)
{
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)v, src, 64);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(v >> 32), src, 64);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}
__device__ __forceinline__ uint64_t wander_shift(uint64_t v, bool fwd, uint32_t amt, int ln, int lp)
{
    return fwd ? shr_q(v, shfl64(v, ln), amt) : shl_t(v, shfl64(v, lp), amt);
}

__device__ __forceinline__ int level_count(uint64_t m0, uint64_t m1)
{
    return __popcll(m0) + 2 * __popcll(m1);
}

template <int T, int RJ, bool WALK>
__global__ __launch_bounds__(kMsc2Lanes, 2) void k_msc_sweep_multi(
    Geom g, MscGeom m, MscTile f, const uint64_t* __restrict__ spin_in, const uint64_t* __restrict__ d0_in,
    const uint64_t* __restrict__ d1_in, const uint64_t* __restrict__ bond, const uint64_t* __restrict__ dr0,
    const uint64_t* __restrict__ dr1, uint64_t* __restrict__ spin_out, uint64_t* __restrict__ d0_out,
    uint64_t* __restrict__ d1_out, unsigned long long* __restrict__ tally, int wander, int wanderA)
{
    constexpr int H = 2 * T;      // halves per pass
    static_assert(!WALK || T == 2, "walkers: two sweeps per pass");
    constexpr int D = 2 * T + 1;  // planes in the coupling ring
    constexpr bool DRAWN = RJ >= 1;
    static_assert(RJ < T, "the refresh sweep is one of the pass");
    constexpr int ZH = H + 1;  // wrapped planes kept: zz, zz - dz, .., zz - H dz
    // planes of the drawn levels, as zc indices: for the next step (even, odd)
    // and for step 0 (even, odd)
    constexpr int kRe = DRAWN ? 2 * RJ - 1 : 0, kRo = DRAWN ? 2 * RJ : 0;
    constexpr int kRe0 = DRAWN ? 2 * RJ : 0, kRo0 = DRAWN ? 2 * RJ + 1 : 0;
    __builtin_amdgcn_s_setprio(1);
    static_assert(D <= 6 && 2 * H + 36 <= kMsc2Words, "six ring slots, one per step phase");
    extern __shared__ uint64_t lds_m2[];
    const int W = m.W;
    // word k of a lane: SB(buf, 0) old odd spins of plane z, SB(buf, h) half
    // h - 1's result plane; CB(slot, d) coupling d of the even sites
    constexpr auto SB = [](int buf, int k) { return buf * H + k; };
    constexpr auto CB = [](int slot, int d) { return 2 * H + slot * 6 + d; };

    const int l = blockIdx.y;
    int t = blockIdx.x, ty, tz;
    if (f.xcd == 2) {  // XCD x takes a band of z tiles of every y tile (msc_kernels.hpp)
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
    const int zstart = dz > 0 ? z0 - (H - 1) : z0 + f.TZ - 1 + (H - 1);
    const int steps = f.TZ + 2 * H - 2;
    const int ry = threadIdx.x / W, w = threadIdx.x - (threadIdx.x / W) * W;
    const int own = min(f.TY, g.Ly - y0);
    const int nrows = own + 2 * H;  // rows of this tile with their rings
    auto wrap = [](int v, int L) { v %= L; return v < 0 ? v + L : v; };
    auto clampr = [&](int lo, int hi) { return wrap(y0 - H + min(max(ry, lo), hi), g.Ly); };
    const int y = wrap(y0 - H + ry, g.Ly);
    const bool own_row = ry >= H && ry < own + H;
    const int yO = clampr(0, nrows - 1), yE = clampr(1, nrows - 2), yD = clampr(2, nrows - 3);
    const int yRe = clampr(2 * RJ + 1, nrows - 2 - 2 * RJ), yRo = clampr(2 * RJ + 2, nrows - 3 - 2 * RJ);
    const int me = threadIdx.x;  // = ry W + w
    const int rowW = ry * W;
    const int mxn = rowW + (w + 1 == W ? 0 : w + 1), mxp = rowW + (w == 0 ? W - 1 : w - 1);
    const int myn = me + W, myp = ry > 0 ? me - W : me;  // rows y +- 1 (row 0 reads itself: never used)
    uint64_t* const Lme = lds_m2 + me * kMsc2Words;
    const uint64_t* const Lxn = lds_m2 + mxn * kMsc2Words;
    const uint64_t* const Lxp = lds_m2 + mxp * kMsc2Words;
    const uint64_t* const Lyn = lds_m2 + myn * kMsc2Words;
    const uint64_t* const Lyp = lds_m2 + myp * kMsc2Words;
    const int ybit = y & 1;
    // walkers: the wave lanes holding this row's next and previous words
    const int lane_n = mxn & 63, lane_p = mxp & 63;
    const bool owedA = WALK && wander >= 0;  // A's input levels come from the other parity's planes

    const int64_t lp = (int64_t)l * 2 * m.plane;
    const uint64_t* ev_in = spin_in + lp;
    const uint64_t* od_in = spin_in + lp + m.plane;
    const uint64_t* bl = bond + (int64_t)l * 6 * m.plane;
    const uint32_t zstride = (uint32_t)(g.Ly * W);
    // z couplings in march orientation: word 4 of a stage (and of the LDS
    // coupling ring) is the bond towards z + dz, word 5 the bond towards z - dz
    const int kFw = dz > 0 ? kPz : kMz, kBw = dz > 0 ? kMz : kPz;
    const uint64_t* const bfw = bl + (int64_t)kFw * m.plane;
    const uint64_t* const bbw = bl + (int64_t)kBw * m.plane;
    const uint32_t rO = (uint32_t)(yO * W + w), rE = (uint32_t)(yE * W + w), rD = (uint32_t)(yD * W + w),
                   rY = (uint32_t)(y * W + w), rRe = (uint32_t)(yRe * W + w), rRo = (uint32_t)(yRo * W + w);
    auto zoff = [&](int z) { return (uint32_t)z * zstride; };
    auto ld = [](const uint64_t* base, uint32_t i) {
        return *reinterpret_cast<const uint64_t*>(reinterpret_cast<const char*>(base) + (i << 3));
    };
    auto st8 = [](uint64_t* base, uint32_t i, uint64_t v) {
        *reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(base) + (i << 3)) = v;
    };

    // zc[k] = the wrapped plane zz - k dz of the current step (uniform)
    int zc[ZH];
#pragma unroll
    for (int k = 0; k < ZH; ++k) zc[k] = wrap(zstart - dz * k, g.Lz);

    using Stage = Msc2Stage<DRAWN>;
    // the operands of the step whose wrapped plane zz2 is zE: odd spins at
    // zz2 + dz, even words at zz2, odd levels at zz2 - dz; drawn levels at
    // zz2 - 2 RJ dz (even) and zz2 - (2 RJ + 1) dz (odd)
    auto load = [&](Stage& S, int zOn, int zE, int zDn, int zRe, int zRo) {
        S.O = ld(od_in, zoff(zOn) + rO);
        const uint32_t h = zoff(zE) + rE;
        S.Es = ld(ev_in, h);
#pragma unroll
        for (int d = 0; d < 4; ++d) S.J[d] = ld(bl + (int64_t)d * m.plane, h);
        S.J[4] = ld(bfw, h);
        S.J[5] = ld(bbw, h);
        const int64_t pe = lp + (owedA ? m.plane : 0), po = lp + (owedA ? 0 : m.plane);
        S.me0 = ld(d0_in + pe, h);
        S.me1 = ld(d1_in + pe, h);
        const uint32_t ho = zoff(zDn) + rD;
        S.mo0 = ld(d0_in + po, ho);
        S.mo1 = ld(d1_in + po, ho);
        if constexpr (DRAWN) {
            const uint32_t he = zoff(zRe) + rRe, hr = zoff(zRo) + rRo;
            S.re0 = ld(dr0 + lp, he);
            S.re1 = ld(dr1 + lp, he);
            S.ro0 = ld(dr0 + lp + m.plane, hr);
            S.ro1 = ld(dr1 + lp + m.plane, hr);
        }
    };

    Stage STG[2] = {};
    uint64_t Oq[3];                          // old odd spins loaded at steps st, st - 1, st - 2 (by st mod 3)
    uint64_t RES[H - 1][3] = {};             // half h's result at its site, by st mod 3
    uint64_t LV0[H > 2 ? H - 2 : 1][3] = {}, LV1[H > 2 ? H - 2 : 1][3] = {};  // its levels (read by half h + 2)
    uint64_t L3a = 0, L3b = 0;               // walkers: half 0's levels three steps back
    int cin = 0, cout = 0;                   // telescoped level sums of the owned sites
    {
        // before step 0: odd spins of zstart - dz and zstart (ring positions of steps -2 and -1)
        Oq[1] = ld(od_in, zoff(zc[1]) + rO);
        Oq[2] = ld(od_in, zoff(zc[0]) + rO);
        Oq[0] = 0;
        const int zp = wrap(zstart + dz, g.Lz);
        load(STG[0], zp, zc[0], zc[1], zc[kRe0], zc[kRo0]);
    }

    // One step of the march.  FIRST: the first six steps, where half h
    // starts at step 2h (known at compile time); after them every half runs.
    auto step = [&](auto phc, auto firstc, int st) {
        constexpr int ph = decltype(phc)::value;
        constexpr bool FIRST = decltype(firstc)::value;
        constexpr auto live = [](int h) { return !FIRST || ph >= 2 * h; };
        constexpr int c0 = ph % 3, c1 = (ph + 2) % 3, c2 = (ph + 1) % 3;  // st, st - 1, st - 2 (mod 3)
        constexpr int buf = ph & 1, pb = buf ^ 1;
        Stage& C = STG[buf];
        __builtin_amdgcn_s_waitcnt(0x0F70);  // stage C complete (vmcnt(0))
        // next step's planes: zz2 = zz + dz (zz = zstart + dz st, the unwrapped plane)
        const int zp1 = step_wrap(zc[0], dz, g.Lz), zp2 = step_wrap(zp1, dz, g.Lz);
        if (st + 1 < steps)
            load(STG[pb], zp2, zp1, zc[0], zc[kRe], zc[kRo]);
        Oq[c0] = C.O;
        Lme[SB(buf, 0)] = Oq[c1];
        // the slot of this step (st mod 6) was last read at step st - 2
#pragma unroll
        for (int d = 0; d < 6; ++d) Lme[CB(ph, d)] = C.J[d];
        lds_barrier();
        constexpr auto slot = [](int k) { return ((ph - k) % 6 + 6) % 6; };  // (st - k) mod 6
        // x offset of the row's sites of the half's parity: (par + y + zh) & 1
        // = (y + zz) & 1 for every half of the step (zh = zz - dz h, even sides)
        const uint32_t q = (uint32_t)((ybit + zc[0]) & 1), qn = q ^ 1u;
#pragma unroll
        for (int h = 0; h < H; ++h) {
            if (!live(h)) continue;  // not started yet
            const int zh = zc[h];
            const int par = h & 1;
            const int src = SB(h == 0 ? buf : pb, h);
            // every read unconditional (a select, not a branch, picks the shifted word)
            const uint64_t Cc = Lme[src], Cn = Lxn[src], Cp = Lxp[src];
            const uint64_t nyp = Lyn[src], nym = Lyp[src];
            const uint64_t nxp = shr_q(Cc, Cn, q);   // q ? shift_next(Cc, Cn) : Cc
            const uint64_t nxm = shl_t(Cc, Cp, qn);  // q ? Cc : shift_prev(Cc, Cp)
            uint64_t up, dn;  // source results at planes zh + dz and zh - dz
            if (h == 0) {
                up = Oq[c0];
                dn = Oq[c2];
            } else {
                up = RES[h - 1][c0];
                dn = RES[h - 1][c2];
            }
            uint64_t jb[6];
            if (par == 0) {
                if (h == 0) {
#pragma unroll
                    for (int d = 0; d < 6; ++d) jb[d] = C.J[d];
                } else {
                    const int sl = slot(h);
#pragma unroll
                    for (int d = 0; d < 6; ++d) jb[d] = Lme[CB(sl, d)];
                }
            } else {  // an odd site's coupling in direction d is its even neighbour's in direction -d
                const int sl = slot(h);
                jb[0] = shr_q(Lme[CB(sl, kMx)], Lxn[CB(sl, kMx)], q);
                jb[1] = shl_t(Lme[CB(sl, kPx)], Lxp[CB(sl, kPx)], qn);
                jb[2] = Lyn[CB(sl, kMy)];
                jb[3] = Lyp[CB(sl, kPy)];
                // the even site at plane zh + dz (ring slot of step st - h + 1)
                // bonds to this site with its bond towards z - dz, the one at
                // zh - dz (step st - h - 1) with its bond towards z + dz
                jb[4] = Lme[CB(slot(h - 1), 5)];
                jb[5] = Lme[CB(slot(h + 1), 4)];
            }
            // the half's plane is owned iff 0 <= st - h - (H - 1) < TZ, in
            // either march direction
            const bool owned = own_row && (uint32_t)(st - h - (H - 1)) < (uint32_t)f.TZ;
            // own spin and levels
            uint64_t s0, m0, m1;
            if (h == 0) {
                s0 = C.Es;
                m0 = C.me0;
                m1 = C.me1;
                if (owedA) {  // even sites take the odd sites' levels: by +q (wander 0) or -(1 - q)
                    const bool fwd = wander == 0;
                    m0 = wander_shift(m0, fwd, fwd ? q : qn, lane_n, lane_p);
                    m1 = wander_shift(m1, fwd, fwd ? q : qn, lane_n, lane_p);
                }
            } else if (h == 1) {
                s0 = Oq[c2];
                m0 = C.mo0;
                m1 = C.mo1;
                if (owedA) {  // odd sites take the even sites' levels: by -(1 - q) (wander 0) or +q
                    const bool fwd = wander != 0;
                    m0 = wander_shift(m0, fwd, fwd ? q : qn, lane_n, lane_p);
                    m1 = wander_shift(m1, fwd, fwd ? q : qn, lane_n, lane_p);
                }
            } else {
                s0 = RES[h - 2][c2];
                m0 = LV0[h - 2][c2];
                m1 = LV1[h - 2][c2];
                bool drawn_here = false;
                if constexpr (DRAWN) {
                    if ((h >> 1) == RJ) {  // the refresh: drawn levels replace those half h - 2 left
                        const uint64_t r0 = par ? C.ro0 : C.re0, r1 = par ? C.ro1 : C.re1;
                        const int dc = level_count(r0, r1) - level_count(m0, m1);
                        cin += owned ? dc : 0;
                        m0 = r0;
                        m1 = r1;
                        drawn_here = true;
                    }
                }
                if constexpr (WALK) {
                    if (!drawn_here && wanderA >= 0) {
                        // sweep A's wandering: even sites of half 2 take half 1's
                        // levels of the step before (same plane), odd sites of
                        // half 3 half 0's of three steps before, each moved by
                        // she / sho of the parity wanderA
                        const uint64_t a0 = par ? L3a : LV0[1][c1], a1 = par ? L3b : LV1[1][c1];
                        const bool fwd = (par == 0) == (wanderA == 0);
                        m0 = wander_shift(a0, fwd, fwd ? q : qn, lane_n, lane_p);
                        m1 = wander_shift(a1, fwd, fwd ? q : qn, lane_n, lane_p);
                    }
                }
            }
            if (h < 2) cin += owned ? level_count(m0, m1) : 0;
            const uint64_t nb[6] = {nxp, nxm, nyp, nym, up, dn};
            const uint64_t Sn = msc_move_fused(s0, nb, jb, m0, m1);
            if (h < H - 1) RES[h][c0] = Sn;
            if (h < H - 2) {
                LV0[h][c0] = m0;
                LV1[h][c0] = m1;
            }
            if (h + 1 < H) Lme[SB(buf, h + 1)] = Sn;
            if (h >= H - 2) {
                cout += owned ? level_count(m0, m1) : 0;
                if (owned) {
                    const uint32_t ho = zoff(zh) + rY;
                    const int64_t pp = lp + (par ? m.plane : 0);
                    st8(spin_out + pp, ho, Sn);
                    st8(d0_out + pp, ho, m0);
                    st8(d1_out + pp, ho, m1);
                }
            }
        }
        // advance the wrapped planes by one step
#pragma unroll
        for (int k = ZH - 1; k > 0; --k) zc[k] = zc[k - 1];
        zc[0] = zp1;
        if constexpr (WALK) {  // half 0's levels of step st - 2: three steps back at the next step
            L3a = LV0[0][c2];
            L3b = LV1[0][c2];
        }
    };
    using Yes = std::true_type;
    using No = std::false_type;
    static_assert(2 * (H - 1) <= 6, "every half has started by step 6");
    // steps = TZ + 2H - 2 >= 7: the first six steps always run
    step(std::integral_constant<int, 0>{}, Yes{}, 0);
    step(std::integral_constant<int, 1>{}, Yes{}, 1);
    step(std::integral_constant<int, 2>{}, Yes{}, 2);
    step(std::integral_constant<int, 3>{}, Yes{}, 3);
    step(std::integral_constant<int, 4>{}, Yes{}, 4);
    step(std::integral_constant<int, 5>{}, Yes{}, 5);
    for (int st = 6; st < steps; st += 6) {
        step(std::integral_constant<int, 0>{}, No{}, st);
        if (st + 1 >= steps) break;
        step(std::integral_constant<int, 1>{}, No{}, st + 1);
        if (st + 2 >= steps) break;
        step(std::integral_constant<int, 2>{}, No{}, st + 2);
        if (st + 3 >= steps) break;
        step(std::integral_constant<int, 3>{}, No{}, st + 3);
        if (st + 4 >= steps) break;
        step(std::integral_constant<int, 4>{}, No{}, st + 4);
        if (st + 5 >= steps) break;
        step(std::integral_constant<int, 5>{}, No{}, st + 5);
    }
    block_add(tally + (int64_t)l * kSlots, 4ll * (long long)(cin - cout));
}

}  // namespace micsa
