// Two MicSA sweeps per pass over memory (temporal blocking of the fused
// sweep in fused_kernels.hpp): sweeps A = k and B = k + 1 of one lattice in
// one launch, reading the state once and writing it once.
//
// A work-group owns TY rows x TZ planes and marches along z.  At step st,
// with p = zstart + dz st, it applies
//     A-even to plane p,   A-odd to plane p - dz,
//     B-even to plane p - 2dz,   B-odd to plane p - 3dz,
// each half seeing exactly the neighbour values the checkerboard order
// prescribes (Sec. 2.8): A-odd on p - dz needs A-even on p - 2dz .. p, B-even
// on p - 2dz needs A-odd on p - 3dz .. p - dz, B-odd on p - 3dz needs B-even
// on p - 4dz .. p - 2dz -- all computed at this or earlier steps.
//
// Rings: B-odd runs on the owned rows/planes, B-even on one ring around
// them, A-odd on two, A-even on three, and the old odd spins are read on
// four; so no tile needs another tile's new values, and every recomputed
// value equals the owner's (all of them are functions of the old state).
// Only owned sites are stored and counted.  The lanes cover TY + 8 rows of
// 16-site chunks.  In-plane neighbours come through four double-buffered
// LDS planes (old odd spins; A's even view; A's new odd spins; B's even
// view), z-neighbours from per-lane registers: one barrier per step.
//
// Refresh (Sec. 2.7): RA draws A's daemons instead of loading them; RB
// draws B's instead of taking A's new ones (the drawn levels of plane q are
// made at the even half of q and the odd ones kept for the odd half of q one
// step later).
//
// Walkers (WALK, gamma = 1, Sec. 2.6): the forward-X wandering that ends a
// timestep moves daemons between a row's parity arrays by 0 or 1 site.  A
// wandering owed from before the launch (wanderA >= 0) is applied as A
// loads its daemons, as in the one-sweep kernel; the wandering of A's own
// timestep (parity wanderAB) is applied in registers: B-even takes A's final
// odd levels of its plane and B-odd A's final even levels, byte-shifted,
// the edge byte coming from the neighbouring chunk's lane by a wave
// shuffle (a row's NC lanes lie in one wave when NC divides 64).  B's own
// wandering is left owed to the next sweep.
#pragma once
#include "fused_kernels.hpp"

namespace micsa {

constexpr int kSweep2Lanes = 640;  // (TY + 8) * NC lanes at most: TY <= 32 for Lx = 512

// Even half on one 16-site chunk: spins W (spin bit 0, bond d in bit 1 + d),
// levels M, the four in-plane odd neighbours A (same k), B (k +- 1), Yp, Ym
// and the two z neighbours.  Returns the even view of the new spins and
// updates W, M and the level sums.
__device__ __forceinline__ V4 even_chunk(V4& W, V4& M, const V4& A, const V4& B, const V4& Yp, const V4& Ym,
                                         const V4& Zup, const V4& Zdn, int q, uint32_t& so, uint32_t& sn)
{
    const int dA = q ? kMx : kPx, dB = q ? kPx : kMx;
    V4 X;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t m1 = 0x01010101u;
        const uint32_t w = W.w[i];
        uint32_t S = w & m1;
        const uint32_t v = xor_and(times63(S), w >> 1, 0x3F3F3F3Fu);
        const uint32_t u = xor_and(A.w[i], v >> dA, m1) + xor_and(B.w[i], v >> dB, m1) +
                           xor_and(Yp.w[i], v >> kPy, m1) + xor_and(Ym.w[i], v >> kMy, m1) +
                           xor_and(Zup.w[i], v >> kPz, m1) + xor_and(Zdn.w[i], v >> kMz, m1);
        const uint32_t S0 = S;
        creutz4(S, M.w[i], u, so, sn);
        const uint32_t flip = S ^ S0;
        W.w[i] = w ^ flip;
        X.w[i] = v ^ times63(flip);  // even view: bit d = new spin ^ j_d
    }
    return X;
}

// Odd half on one chunk: old odd spins S (clean), levels M, and the even
// views of the six neighbours.
__device__ __forceinline__ void odd_chunk(V4& S, V4& M, const V4& A, const V4& B, const V4& Yp, const V4& Ym,
                                          const V4& Zup, const V4& Zdn, int q, uint32_t& so, uint32_t& sn)
{
    const int dA = q ? kMx : kPx, dB = q ? kPx : kMx;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t m1 = 0x01010101u;
        uint32_t s = S.w[i];
        const uint32_t u = xor_and(s, A.w[i] >> dA, m1) + xor_and(s, B.w[i] >> dB, m1) +
                           xor_and(s, Yp.w[i] >> kMy, m1) + xor_and(s, Ym.w[i] >> kPy, m1) +
                           xor_and(s, Zup.w[i] >> kMz, m1) + xor_and(s, Zdn.w[i] >> kPz, m1);
        creutz4(s, M.w[i], u, so, sn);
        S.w[i] = s;
    }
}

template <bool RA, bool RB, bool WALK>
__global__ void __launch_bounds__(kSweep2Lanes) k_micsa_sweep2_fused(
    Geom g, FusedTile f, const uint8_t* __restrict__ spin_in, const uint8_t* __restrict__ dem_in,
    uint8_t* __restrict__ spin_out, uint8_t* __restrict__ dem_out, unsigned long long* __restrict__ tally,
    uint32_t rhoA, DaemonThresholds thA, uint32_t rhoB, DaemonThresholds thB, int wanderA, int wanderAB)
{
    extern __shared__ uint4 lds[];
    const int rows_slots = f.TY + 8;
    const int plane_slots = rows_slots * f.NC;
    uint4* SoO = lds;                    // [2][TY+8][NC] old odd spins of plane p
    uint4* XA = lds + 2 * plane_slots;   // [2][..] A's even view of plane p - dz (written a step earlier)
    uint4* SoA = lds + 4 * plane_slots;  // [2][..] A's new odd spins of plane p - 2dz
    uint4* XB = lds + 6 * plane_slots;   // [2][..] B's even view of plane p - 3dz

    const int l = blockIdx.y;
    const int s = l / g.R, r = l % g.R;
    int ty, tz;
    tile_of(f, blockIdx.x, ty, tz);
    const int y0 = ty * f.TY, z0 = tz * f.TZ;
    const int dz = (tz & 1) ? -1 : 1;  // odd z-tiles march downwards (shared halo planes read together)
    const int zstart = dz > 0 ? z0 - 3 : z0 + f.TZ + 2;
    const int ry = threadIdx.x / f.NC, c = threadIdx.x - ry * f.NC;
    const bool active = ry < rows_slots;
    // rings reach 4 rows / planes out: wrap with a full modulo (sides may be 2)
    auto wrap = [](int v, int L) { v %= L; return v < 0 ? v + L : v; };
    const int y = wrap(y0 - 4 + ry, g.Ly);
    const bool rowA_e = active && ry >= 1 && ry <= f.TY + 6;
    const bool rowA_o = active && ry >= 2 && ry <= f.TY + 5;
    const bool rowB_e = active && ry >= 3 && ry <= f.TY + 4;
    const bool rowB_o = active && ry >= 4 && ry <= f.TY + 3;  // the rows the tile owns
    auto owned_plane = [&](int st_plane) {  // plane index st_plane in march order -> owned?
        const int zz = zstart + dz * st_plane;
        return zz >= z0 && zz < z0 + f.TZ;
    };

    const uint8_t* ev_in = spin_in + ((int64_t)l * 2 + 0) * g.Nh;
    const uint8_t* od_in = spin_in + ((int64_t)l * 2 + 1) * g.Nh;
    const uint8_t* me_in = dem_in + ((int64_t)l * 2 + 0) * g.Nh;
    const uint8_t* mo_in = dem_in + ((int64_t)l * 2 + 1) * g.Nh;
    uint8_t* ev_out = spin_out + ((int64_t)l * 2 + 0) * g.Nh;
    uint8_t* od_out = spin_out + ((int64_t)l * 2 + 1) * g.Nh;
    uint8_t* me_out = dem_out + ((int64_t)l * 2 + 0) * g.Nh;
    uint8_t* mo_out = dem_out + ((int64_t)l * 2 + 1) * g.Nh;
    const uint32_t sw = stream_word(kStreamDaemon, (uint32_t)s);

    auto zof = [&](int st_plane) { return wrap(zstart + dz * st_plane, g.Lz); };
    const int64_t lane_off = (int64_t)y * g.Kx + 16 * c;
    const int64_t plane = (int64_t)g.Ly * g.Kx;
    auto hof = [&](int z) { return lane_off + plane * z; };  // z is uniform: the product is scalar
    const int cn = c + 1 == f.NC ? 0 : c + 1, cp = c == 0 ? f.NC - 1 : c - 1;
    const int steps = f.TZ + 6;

    // registers carried along the march (index 0 = newest plane)
    V4 Oo_prev{}, Oo_cur{}, Oo_next{};  // old odd spins at p - dz, p, p + dz
    V4 XA0{}, XA1{}, XA2{};             // A even views at p, p - dz, p - 2dz
    V4 WA1{}, WA2{}, MA1{}, MA2{};      // A's new even spins/levels at p - dz, p - 2dz
    V4 MA3{};                           // WALK: A's new even levels at p - 3dz
    V4 SA0{}, SA1{}, SA2{};             // A's new odd spins at p - dz, p - 2dz, p - 3dz
    V4 NA0{}, NA1{}, NA2{};             // A's new odd levels at the same planes
    V4 XB0{}, XB1{}, XB2{};             // B even views at p - 2dz, p - 3dz, p - 4dz
    V4 MoA_gen{};                       // RA: A's drawn odd levels of plane p - dz
    V4 MoB_gen{};                       // RB: B's drawn odd levels of plane p - 3dz
    V4 nSo{}, nSe{}, nMe{}, nMo{};      // loads for the next step
    uint32_t nMex = 0, nMox = 0;        // WALK: edge words of an owed wandering

    // shift of a row's even (odd) daemons in a wandering of parity w:
    // new[k] = other parity array[k + shift] (see shift_bytes)
    auto sh_even = [&](int w, int z) { return w == 0 ? ((y + z) & 1) : ((y + z) & 1) - 1; };
    auto sh_odd = [&](int w, int z) { return w == 0 ? -((y + z) & 1) : 1 - ((y + z) & 1); };
    auto row_of = [&](int z) { return (int64_t)y * g.Kx + plane * z; };
    // the loads of march step st2 at wrapped planes z2 = zof(st2), z2p =
    // zof(st2 + 1) and z2m = zof(st2 - 1)
    auto load_step = [&](int st2, int z2, int z2p, int z2m) {
        nMex = 0u;
        nMox = 0u;
        if (active) nSo = ldg16(od_in + hof(z2p));
        if (rowA_e) {
            const int64_t h2 = hof(z2);
            nSe = ldg16(ev_in + h2);
            if (!RA) {
                if (!WALK || wanderA < 0) {
                    nMe = ldg16(me_in + h2);
                } else {  // new even daemons come from the odd array
                    const uint8_t* row = mo_in + row_of(z2);
                    nMe = ldg16(row + 16 * c);
                    nMex = *reinterpret_cast<const uint32_t*>(shift_edge(row, cn, cp, sh_even(wanderA, z2)));
                }
            }
        }
        if (!RA && rowA_o && st2 >= 2) {
            const int zo2 = z2m;
            if (!WALK || wanderA < 0) {
                nMo = ldg16(mo_in + hof(zo2));
            } else {  // new odd daemons come from the even array
                const uint8_t* row = me_in + row_of(zo2);
                nMo = ldg16(row + 16 * c);
                nMox = *reinterpret_cast<const uint32_t*>(shift_edge(row, cn, cp, sh_odd(wanderA, zo2)));
            }
        }
    };
    // lanes of this row's neighbouring chunks (a row's lanes share a wave)
    const int lane_next = (ry * f.NC + cn) & 63, lane_prev = (ry * f.NC + cp) & 63;
    // the edge word a neighbour needs from v for a shift sh, taken from the lane it comes from
    auto edge_from = [&](const V4& v, int sh) {
        const uint32_t give = sh > 0 ? v.w[0] : v.w[3];
        return (uint32_t)__shfl((int)give, sh > 0 ? lane_next : lane_prev, 64);
    };
    // zr[k] = zof(st + 2 - k), k = 0 .. 5: the wrapped planes of the step's
    // loads and halves, moved by one plane per step (a compare, no division)
    int zr[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) zr[k] = zof(2 - k);
    if (active) {
        Oo_prev = ldg16(od_in + hof(zr[3]));
        Oo_cur = ldg16(od_in + hof(zr[2]));
    }
    load_step(0, zr[2], zr[1], zr[3]);
    uint32_t sum_old = 0, sum_new = 0;  // level sums before/after the owned moves of both sweeps
    for (int st = 0; st < steps; ++st) {
        const int buf = st & 1, pb = buf ^ 1;
        const int zA = zr[2];   // A-even plane p
        const int zAo = zr[3];  // A-odd plane p - dz
        const int zBe = zr[4];  // B-even plane p - 2dz
        const int zBo = zr[5];  // B-odd plane p - 3dz
        Oo_next = nSo;
        V4 Se = nSe, Me = nMe, Mo = nMo;
        if (WALK && !RA && wanderA >= 0) {
            Me = shift_bytes(Me, nMex, sh_even(wanderA, zA));
            Mo = shift_bytes(Mo, nMox, sh_odd(wanderA, zAo));
        }
        // WALK: B's daemons are A's final ones after the wandering of A's
        // timestep: even levels of zBe from A's odd levels (NA1), odd levels
        // of zBo from A's even levels (MA3); the edge bytes by shuffle, with
        // every lane taking part
        uint32_t edgeBe = 0, edgeBo = 0;
        if (WALK && !RB) {
            edgeBe = edge_from(NA1, sh_even(wanderAB, zBe));
            edgeBo = edge_from(MA3, sh_odd(wanderAB, zBo));
        }
        if (st + 1 < steps) load_step(st + 1, zr[1], zr[0], zr[2]);
        V4 MoA_next{}, MoB_next{};
        if (RA && rowA_e) refresh_chunk(g, y + g.Ly * zA, c, (y + zA) & 1, rhoA, (uint32_t)r, sw, thA, Me, MoA_next);
        if (active) sts16(&SoO[buf * plane_slots + ry * f.NC + c], Oo_cur);
        __syncthreads();

        // ---- A-even on plane p (old odd neighbours)
        if (rowA_e) {
            const int q = (y + zA) & 1;
            const int dir = q ? 1 : -1;
            const uint4* row = &SoO[buf * plane_slots + ry * f.NC];
            const uint32_t nbw = dir > 0 ? row[cn].x : row[cp].w;
            const V4 B = shift16(Oo_cur, nbw, dir);
            const V4 Yp = lds16(&SoO[buf * plane_slots + (ry + 1) * f.NC + c]);
            const V4 Ym = lds16(&SoO[buf * plane_slots + (ry - 1) * f.NC + c]);
            uint32_t so = 0, sn = 0;
            XA0 = even_chunk(Se, Me, Oo_cur, B, Yp, Ym, dz > 0 ? Oo_next : Oo_prev, dz > 0 ? Oo_prev : Oo_next, q,
                             so, sn);
            sts16(&XA[buf * plane_slots + ry * f.NC + c], XA0);
            if (rowB_o && owned_plane(st)) {
                sum_old += so;
                sum_new += sn;
            }
        }
        // ---- A-odd on plane p - dz (A's even views of p - 2dz .. p)
        if (rowA_o && st >= 2) {
            const int q = (y + zAo) & 1;
            const int dir = q ? -1 : 1;
            const uint4* row = &XA[pb * plane_slots + ry * f.NC];
            const uint32_t nbw = dir > 0 ? row[cn].x : row[cp].w;
            const V4 B = shift16(XA1, nbw, dir);
            const V4 Yp = lds16(&XA[pb * plane_slots + (ry + 1) * f.NC + c]);
            const V4 Ym = lds16(&XA[pb * plane_slots + (ry - 1) * f.NC + c]);
            if (RA) Mo = MoA_gen;
            V4 S = Oo_prev;
            uint32_t so = 0, sn = 0;
            odd_chunk(S, Mo, XA1, B, Yp, Ym, dz > 0 ? XA0 : XA2, dz > 0 ? XA2 : XA0, q, so, sn);
            SA0 = S;
            NA0 = Mo;
            sts16(&SoA[buf * plane_slots + ry * f.NC + c], SA0);
            if (rowB_o && owned_plane(st - 1)) {
                sum_old += so;
                sum_new += sn;
            }
        }
        // ---- B-even on plane p - 2dz (A's new odd spins of p - 3dz .. p - dz)
        if (rowB_e && st >= 4) {
            const int q = (y + zBe) & 1;
            const int dir = q ? 1 : -1;
            const uint4* row = &SoA[pb * plane_slots + ry * f.NC];
            const uint32_t nbw = dir > 0 ? row[cn].x : row[cp].w;
            const V4 B = shift16(SA1, nbw, dir);
            const V4 Yp = lds16(&SoA[pb * plane_slots + (ry + 1) * f.NC + c]);
            const V4 Ym = lds16(&SoA[pb * plane_slots + (ry - 1) * f.NC + c]);
            V4 W = WA2, M = MA2;
            if (WALK && !RB) M = shift_bytes(NA1, edgeBe, sh_even(wanderAB, zBe));
            if (RB) refresh_chunk(g, y + g.Ly * zBe, c, (y + zBe) & 1, rhoB, (uint32_t)r, sw, thB, M, MoB_next);
            uint32_t so = 0, sn = 0;
            XB0 = even_chunk(W, M, SA1, B, Yp, Ym, dz > 0 ? SA0 : SA2, dz > 0 ? SA2 : SA0, q, so, sn);
            sts16(&XB[buf * plane_slots + ry * f.NC + c], XB0);
            if (rowB_o && owned_plane(st - 2)) {
                const int64_t h = hof(zBe);
                stg16_nt(ev_out + h, W.w);
                stg16_nt(me_out + h, M.w);
                sum_old += so;
                sum_new += sn;
            }
        }
        // ---- B-odd on plane p - 3dz (B's even views of p - 4dz .. p - 2dz)
        if (rowB_o && st >= 6) {
            const int q = (y + zBo) & 1;
            const int dir = q ? -1 : 1;
            const uint4* row = &XB[pb * plane_slots + ry * f.NC];
            const uint32_t nbw = dir > 0 ? row[cn].x : row[cp].w;
            const V4 B = shift16(XB1, nbw, dir);
            const V4 Yp = lds16(&XB[pb * plane_slots + (ry + 1) * f.NC + c]);
            const V4 Ym = lds16(&XB[pb * plane_slots + (ry - 1) * f.NC + c]);
            V4 S = SA2, M = RB ? MoB_gen : NA2;
            if (WALK && !RB) M = shift_bytes(MA3, edgeBo, sh_odd(wanderAB, zBo));
            uint32_t so = 0, sn = 0;
            odd_chunk(S, M, XB1, B, Yp, Ym, dz > 0 ? XB0 : XB2, dz > 0 ? XB2 : XB0, q, so, sn);
            if (owned_plane(st - 3)) {
                const int64_t h = hof(zBo);
                stg16_nt(od_out + h, S.w);
                stg16_nt(mo_out + h, M.w);
                sum_old += so;
                sum_new += sn;
            }
        }
        // shift the per-lane plane histories by one plane
        Oo_prev = Oo_cur;
        Oo_cur = Oo_next;
        XA2 = XA1;
        XA1 = XA0;
        WA2 = WA1;
        if (WALK) MA3 = MA2;
        MA2 = MA1;
        WA1 = Se;
        MA1 = Me;
        SA2 = SA1;
        SA1 = SA0;
        NA2 = NA1;
        NA1 = NA0;
        XB2 = XB1;
        XB1 = XB0;
        MoA_gen = MoA_next;
        MoB_gen = MoB_next;
#pragma unroll
        for (int k = 5; k > 0; --k) zr[k] = zr[k - 1];
        zr[0] = zr[1] + dz == g.Lz ? 0 : (zr[1] + dz < 0 ? g.Lz - 1 : zr[1] + dz);
    }
    // dH = 4 (sum of old levels - sum of new levels) over the owned moves of both sweeps
    block_add(tally + (int64_t)l * kSlots, 4 * ((long long)sum_old - (long long)sum_new));
}

}  // namespace micsa
