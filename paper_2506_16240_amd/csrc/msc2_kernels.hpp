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
// the kernel loading them for halves 2 rj and 2 rj + 1 when sweep rj >= 1 of
// the pass refreshes.  Walkers keep the one-sweep kernel.
// The energy tally adds 4 (sum m - sum m') of every half on the owned sites.
//
// Grid (nty * ntz, L); block 64 ceil((TY + 4T) W / 64) <= kMsc2Lanes;
// LDS 8 (4T + 6 (2T + 1)) (TY + 4T) W bytes.
#pragma once
#include "msc_kernels.hpp"

namespace micsa {

constexpr int kMsc2Lanes = 256;

struct Msc2Stage {
    uint64_t O, Es, J[6], me0, me1, mo0, mo1;
    uint64_t re0, re1, ro0, ro1;  // drawn levels for the halves of a refresh sweep rj >= 1
};

template <int T>
__global__ __launch_bounds__(kMsc2Lanes, 2) void k_msc_sweep_multi(
    Geom g, MscGeom m, MscTile f, const uint64_t* __restrict__ spin_in, const uint64_t* __restrict__ d0_in,
    const uint64_t* __restrict__ d1_in, const uint64_t* __restrict__ bond, const uint64_t* __restrict__ dr0,
    const uint64_t* __restrict__ dr1, int rj, uint64_t* __restrict__ spin_out, uint64_t* __restrict__ d0_out,
    uint64_t* __restrict__ d1_out, unsigned long long* __restrict__ tally)
{
    constexpr int H = 2 * T;      // halves per pass
    constexpr int D = 2 * T + 1;  // planes in the coupling ring
    __builtin_amdgcn_s_setprio(1);
    extern __shared__ uint64_t lds_m2[];
    const int W = m.W;
    const int ps = (f.TY + 2 * H) * W;  // words per LDS plane (one per lane)
    // SB[buf][0]: old odd spins of plane z; SB[buf][h]: half h - 1's result plane
    auto SB = [&](int buf, int k) { return lds_m2 + ((size_t)buf * H + k) * ps; };
    auto CB = [&](int slot, int d) { return lds_m2 + (size_t)2 * H * ps + ((size_t)slot * 6 + d) * ps; };

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
    const bool active = ry < nrows;
    auto wrap = [](int v, int L) { v %= L; return v < 0 ? v + L : v; };
    auto clampr = [&](int lo, int hi) { return wrap(y0 - H + min(max(ry, lo), hi), g.Ly); };
    const int y = wrap(y0 - H + ry, g.Ly);
    const bool own_row = ry >= H && ry < own + H;
    const int yO = clampr(0, nrows - 1), yE = clampr(1, nrows - 2), yD = clampr(2, nrows - 3);
    const int yRe = clampr(2 * rj + 1, nrows - 2 - 2 * rj), yRo = clampr(2 * rj + 2, nrows - 3 - 2 * rj);
    const int wn = w + 1 == W ? 0 : w + 1, wp = w == 0 ? W - 1 : w - 1;
    const int me = ry * W + w;

    const int64_t lp = (int64_t)l * 2 * m.plane;
    const uint64_t* ev_in = spin_in + lp;
    const uint64_t* od_in = spin_in + lp + m.plane;
    const uint64_t* bl = bond + (int64_t)l * 6 * m.plane;
    const uint32_t zstride = (uint32_t)(g.Ly * W);
    const uint32_t rO = (uint32_t)(yO * W + w), rE = (uint32_t)(yE * W + w), rD = (uint32_t)(yD * W + w),
                   rY = (uint32_t)(y * W + w), rRe = (uint32_t)(yRe * W + w), rRo = (uint32_t)(yRo * W + w);
    auto zoff = [&](int zz) { return (uint32_t)zz * zstride; };
    auto ld = [](const uint64_t* base, uint32_t i) {
        return *reinterpret_cast<const uint64_t*>(reinterpret_cast<const char*>(base) + (i << 3));
    };
    auto st8 = [](uint64_t* base, uint32_t i, uint64_t v) {
        *reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(base) + (i << 3)) = v;
    };

    uint64_t O_prev = ld(od_in, zoff(wrap(zstart - dz, g.Lz)) + rO);  // old odd spins at z - dz, z, z + dz
    uint64_t O_cur = ld(od_in, zoff(wrap(zstart, g.Lz)) + rO);
    uint64_t O_next = 0;
    uint64_t RES[H][3];          // half h's result at its site: this step, one and two steps ago
    uint64_t LV0[H][3], LV1[H][3];  // its levels (read by half h + 2)
#pragma unroll
    for (int h = 0; h < H; ++h)
#pragma unroll
        for (int k = 0; k < 3; ++k) RES[h][k] = LV0[h][k] = LV1[h][k] = 0;

    auto load = [&](int st2, Msc2Stage& S) {
        const int zz2 = zstart + dz * st2;
        const int z2 = wrap(zz2, g.Lz);
        S.O = ld(od_in, zoff(wrap(zz2 + dz, g.Lz)) + rO);
        const uint32_t h = zoff(z2) + rE;
        S.Es = ld(ev_in, h);
#pragma unroll
        for (int d = 0; d < 6; ++d) S.J[d] = ld(bl + (int64_t)d * m.plane, h);
        S.me0 = ld(d0_in + lp, h);
        S.me1 = ld(d1_in + lp, h);
        const uint32_t ho = zoff(wrap(zz2 - dz, g.Lz)) + rD;
        S.mo0 = ld(d0_in + lp + m.plane, ho);
        S.mo1 = ld(d1_in + lp + m.plane, ho);
        if (rj > 0) {
            const uint32_t he = zoff(wrap(zz2 - dz * 2 * rj, g.Lz)) + rRe;
            const uint32_t hr = zoff(wrap(zz2 - dz * (2 * rj + 1), g.Lz)) + rRo;
            S.re0 = ld(dr0 + lp, he);
            S.re1 = ld(dr1 + lp, he);
            S.ro0 = ld(dr0 + lp + m.plane, hr);
            S.ro1 = ld(dr1 + lp + m.plane, hr);
        }
    };
    long long so = 0, sn = 0;
    auto step = [&](int st, Msc2Stage& S, Msc2Stage& N) {
        __builtin_amdgcn_s_waitcnt(0x0F70);  // stage S complete (vmcnt(0))
        const int buf = st & 1, pb = buf ^ 1;
        const int zz = zstart + dz * st;
        O_next = S.O;
        const Msc2Stage& C = S;
        if (st + 1 < steps) load(st + 1, N);
        if (active) SB(buf, 0)[me] = O_cur;
        lds_barrier();
        const int slot0 = st % D;
        if (active) {
#pragma unroll
            for (int d = 0; d < 6; ++d) CB(slot0, d)[me] = C.J[d];
        }
#pragma unroll
        for (int h = 0; h < H; ++h) {
            if (st < 2 * h) continue;  // not needed yet (uniform)
            const bool rows_h = ry >= h + 1 && ry < nrows - 1 - h;
            if (!rows_h) continue;
            const int zh_u = zz - dz * h;  // unwrapped plane of this half
            const int zh = wrap(zh_u, g.Lz);
            const int par = h & 1;
            const int q = (par + y + zh) & 1;
            const uint64_t* src = SB(h == 0 ? buf : pb, h);
            const uint64_t Cc = src[me];
            const uint64_t nxp = q ? shift_next(Cc, src[ry * W + wn]) : Cc;
            const uint64_t nxm = q ? Cc : shift_prev(Cc, src[ry * W + wp]);
            const uint64_t nyp = src[me + W], nym = src[me - W];
            uint64_t up, dn;  // source results at planes zh + dz and zh - dz
            if (h == 0) {
                up = O_next;
                dn = O_prev;
            } else {
                up = RES[h - 1][0];
                dn = RES[h - 1][2];
            }
            const uint64_t nzp = dz > 0 ? up : dn, nzm = dz > 0 ? dn : up;
            uint64_t jb[6];
            const int sl = ((st - h) % D + D) % D;
            if (par == 0) {
                if (h == 0) {
#pragma unroll
                    for (int d = 0; d < 6; ++d) jb[d] = C.J[d];
                } else {
#pragma unroll
                    for (int d = 0; d < 6; ++d) jb[d] = CB(sl, d)[me];
                }
            } else {  // an odd site's coupling in direction d is its even neighbour's in direction -d
                const uint64_t* Mx = CB(sl, kMx);
                const uint64_t* Px = CB(sl, kPx);
                jb[0] = q ? shift_next(Mx[me], Mx[ry * W + wn]) : Mx[me];
                jb[1] = q ? Px[me] : shift_prev(Px[me], Px[ry * W + wp]);
                jb[2] = CB(sl, kMy)[me + W];
                jb[3] = CB(sl, kPy)[me - W];
                const int s_up = ((st - h + 1) % D + D) % D, s_dn = ((st - h - 1) % D + D) % D;
                jb[4] = CB(dz > 0 ? s_up : s_dn, kMz)[me];  // even site at plane zh + 1
                jb[5] = CB(dz > 0 ? s_dn : s_up, kPz)[me];  // even site at plane zh - 1
            }
            // own spin and levels
            uint64_t s0, m0, m1;
            if (h == 0) {
                s0 = C.Es;
                m0 = C.me0;
                m1 = C.me1;
            } else if (h == 1) {
                s0 = O_prev;
                m0 = C.mo0;
                m1 = C.mo1;
            } else {
                s0 = RES[h - 2][2];
                if (rj > 0 && (h >> 1) == rj) {
                    m0 = par ? C.ro0 : C.re0;
                    m1 = par ? C.ro1 : C.re1;
                } else {
                    m0 = LV0[h - 2][2];
                    m1 = LV1[h - 2][2];
                }
            }
            const uint64_t nb[6] = {nxp, nxm, nyp, nym, nzp, nzm};
            long long a = 0, b = 0;
            const uint64_t Sn = msc_move(s0, nb, jb, m0, m1, a, b);
            RES[h][0] = Sn;
            LV0[h][0] = m0;
            LV1[h][0] = m1;
            if (h + 1 < H) SB(buf, h + 1)[me] = Sn;
            const bool own_plane = zh_u >= z0 && zh_u < z0 + f.TZ;
            if (own_row && own_plane) {
                so += a;
                sn += b;
                if (h >= H - 2) {
                    const uint32_t ho = zoff(zh) + rY;
                    const int64_t pp = lp + (par ? m.plane : 0);
                    st8(spin_out + pp, ho, Sn);
                    st8(d0_out + pp, ho, m0);
                    st8(d1_out + pp, ho, m1);
                }
            }
        }
        O_prev = O_cur;
        O_cur = O_next;
#pragma unroll
        for (int h = 0; h < H; ++h) {
            RES[h][2] = RES[h][1];
            RES[h][1] = RES[h][0];
            LV0[h][2] = LV0[h][1];
            LV0[h][1] = LV0[h][0];
            LV1[h][2] = LV1[h][1];
            LV1[h][1] = LV1[h][0];
        }
    };
    Msc2Stage SA = {}, SBs = {};
    load(0, SA);
    for (int st = 0; st < steps; st += 2) {
        step(st, SA, SBs);
        if (st + 1 < steps) step(st + 1, SBs, SA);
    }
    block_add(tally + (int64_t)l * kSlots, 4 * (so - sn));
}

}  // namespace micsa
