// Fused MicSA sweep for the byte layout: one launch performs a whole sweep
// (even half, then odd half, Sec. 2.8) and, on refresh sweeps, the daemon
// refresh (Sec. 2.7) -- reading each state byte from HBM about once and
// writing it once.
//
// Decomposition.  A work-group owns a tile of TY full rows (all of x) and TZ
// planes of one lattice and marches along z.  At step z it performs the
// even half on plane z and the odd half on plane z-1: the odd sites of plane
// z-1 see new even spins on planes z-2, z-1 and z, all final by then.  The
// even half is also computed on one ring of rows/planes around the tile and
// the odd spins are read on two rings, so a tile never needs another tile's
// new values.  State is double-buffered (read "in", write "out"), so the
// ring recomputations read exactly the old state and agree bit for bit with
// the owning tile.
//
// Lanes.  Each lane owns one 16-site chunk of one row (16 even and 16 odd
// sites, uint4 loads and stores) for the whole march.  Its z-neighbours live
// in its registers; in-plane neighbours (y +- 1, and the byte-shifted x
// neighbour from the adjacent chunk) come through LDS, one plane of odd
// spins and one plane of "even view" bytes per step, double-buffered so one
// barrier per step suffices.
//
// Even view.  After an even site is updated its byte X holds, in bit d, the
// new even spin XOR the coupling bit of its bond in direction d (d = +x, -x,
// +y, -y, +z, -z).  The odd neighbour across that bond reads bit d of X: the
// spin and the coupling it needs, in one byte.
#pragma once
#include "byte_kernels.hpp"

namespace micsa {

struct FusedTile {
    int32_t TY, TZ;  // tile rows (divides Ly) and planes (divides Lz)
    int32_t NC;      // 16-site chunks per row = Lx / 32
    int32_t nty;     // tiles along y = Ly / TY
    int32_t ntz;     // tiles along z = Lz / TZ
    int32_t xcd;     // 1: map blocks to tiles XCD by XCD (tiles per lattice divisible by 8)
};

// Tile of block b.  Work-groups are dispatched round-robin over the 8 XCDs
// (block b on XCD b % 8), each XCD with its own L2.  Tiles are numbered
// z-fastest and, with xcd set, XCD x receives the contiguous tile range
// [x T/8, (x+1) T/8): a band of whole y-tiles, so most y- and z-neighbour
// tiles, which read each other's halo rows and planes, share an L2.
__device__ __forceinline__ void tile_of(const FusedTile& f, int b, int& ty, int& tz)
{
    int t = b;
    if (f.xcd) {
        const int per = f.nty * f.ntz / 8;
        t = (b & 7) * per + (b >> 3);
    }
    tz = t % f.ntz;
    ty = t / f.ntz;
}

using v4u = unsigned int __attribute__((ext_vector_type(4)));

// Streaming 16-byte store that does not allocate in L2 (the written state is
// not read again in this sweep), leaving L2 to the halo reads.
__device__ __forceinline__ void stg16_nt(uint8_t* __restrict__ p, const uint32_t w[4])
{
    v4u v = {w[0], w[1], w[2], w[3]};
    __builtin_nontemporal_store(v, reinterpret_cast<v4u*>(p));
}

struct V4 {
    uint32_t w[4];
};

__device__ __forceinline__ V4 ldg16(const uint8_t* __restrict__ p)
{
    const uint4 v = *reinterpret_cast<const uint4*>(p);
    return {{v.x, v.y, v.z, v.w}};
}

// A row chunk of 16 daemon bytes shifted by sh sites, new[k] = src[k + sh]
// (sh in {-1, 0, 1}), from the chunk v and the edge word x of the adjacent
// chunk of the same row (the first word of the next chunk for sh = 1, the
// last word of the previous one for sh = -1), so the shift wraps around the
// row as the lattice does.  Branch-free (rows of both shifts share a wave):
// each word is alignbyte((hi:lo) >> 8 * shift).
__device__ __forceinline__ const uint8_t* shift_edge(const uint8_t* row, int cn, int cp, int sh)
{
    return sh < 0 ? row + 16 * cp + 12 : row + 16 * cn;
}

__device__ __forceinline__ V4 shift_bytes(const V4& v, uint32_t x, int sh)
{
    const uint32_t b = sh > 0 ? 1u : (sh < 0 ? 3u : 0u);
    V4 o;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const uint32_t up = i < 3 ? v.w[i + 1] : x;  // the word after w[i]
        const uint32_t dn = i > 0 ? v.w[i - 1] : x;  // the word before w[i]
        o.w[i] = __builtin_amdgcn_alignbyte(sh > 0 ? up : v.w[i], sh < 0 ? dn : v.w[i], b);
    }
    return o;
}

__device__ __forceinline__ void stg16(uint8_t* __restrict__ p, const V4& v)
{
    *reinterpret_cast<uint4*>(p) = make_uint4(v.w[0], v.w[1], v.w[2], v.w[3]);
}

__device__ __forceinline__ V4 lds16(const uint4* s)
{
    const uint4 v = *s;
    return {{v.x, v.y, v.z, v.w}};
}

__device__ __forceinline__ void sts16(uint4* s, const V4& v) { *s = make_uint4(v.w[0], v.w[1], v.w[2], v.w[3]); }

// The 16 sites k+1 .. k+16 (dir > 0, nbw = first word of the next chunk) or
// k-1 .. k+14 (dir < 0, nbw = last word of the previous chunk).
__device__ __forceinline__ V4 shift16(const V4& a, uint32_t nbw, int dir)
{
    V4 r;
    if (dir > 0) {
        r.w[0] = __builtin_amdgcn_alignbyte(a.w[1], a.w[0], 1);
        r.w[1] = __builtin_amdgcn_alignbyte(a.w[2], a.w[1], 1);
        r.w[2] = __builtin_amdgcn_alignbyte(a.w[3], a.w[2], 1);
        r.w[3] = __builtin_amdgcn_alignbyte(nbw, a.w[3], 1);
    } else {
        r.w[0] = __builtin_amdgcn_alignbyte(a.w[0], nbw, 3);
        r.w[1] = __builtin_amdgcn_alignbyte(a.w[1], a.w[0], 3);
        r.w[2] = __builtin_amdgcn_alignbyte(a.w[2], a.w[1], 3);
        r.w[3] = __builtin_amdgcn_alignbyte(a.w[3], a.w[2], 3);
    }
    return r;
}

// x * 0x3F for x with at most bit 0 of each byte set (each byte becomes 0x3F
// or 0), as one packed 16-bit multiply: a 16-bit half holds two such bytes,
// 0x0101 * 0x3F < 2^16, so no half carries into the next.  (Written as a
// shift and a subtraction it compiles to a quarter-rate 32-bit multiply.)
__device__ __forceinline__ uint32_t times63(uint32_t x)
{
    typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
    u16x2 v = __builtin_bit_cast(u16x2, x);
    v = v * (u16x2){63, 63};
    return __builtin_bit_cast(uint32_t, v);
}

// Three-input bit operations in one v_bitop3: the truth table indexes the
// bits as (a << 2) | (b << 1) | c.
__device__ __forceinline__ uint32_t xor_and(uint32_t a, uint32_t b, uint32_t c)  // a ^ (b & c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x78);
}
__device__ __forceinline__ uint32_t and_andn(uint32_t a, uint32_t b, uint32_t c)  // a & ~b & c
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x20);
}
__device__ __forceinline__ uint32_t bitsel(uint32_t a, uint32_t b, uint32_t c)  // a ? b : c, bitwise
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0xCA);
}

// Creutz move on 4 byte-sites given their unsatisfied-bond counts u (see
// micsa_word): legal iff t = m + u + 5 lies in 8..11, new level t & 3.
// Energy: an accepted move changes H by dH = 4 (m - m') exactly (eq.
// Creutz), a rejected one leaves m' = m, so the tally needs only the byte
// sums of the old and new levels (v_sad_u8 accumulates them).
__device__ __forceinline__ void creutz4(uint32_t& S, uint32_t& M, uint32_t u, uint32_t& sum_old, uint32_t& sum_new)
{
    const uint32_t t = M + u + 0x05050505u;
    const uint32_t acc = and_andn(t >> 3, t >> 2, 0x01010101u);
    const uint32_t low2 = (acc << 1) + acc;  // 0x03 in accepted bytes
    S ^= acc;
    sum_old = __builtin_amdgcn_sad_u8(M, 0u, sum_old);
    M = bitsel(low2, t, M);
    sum_new = __builtin_amdgcn_sad_u8(M, 0u, sum_new);
}

// Daemon levels of the 16 even and 16 odd sites of chunk c of a row from the
// refresh draws: natural sites x = 32c .. 32c+31 of the row use the 8 Philox
// calls with counters (i >> 2) = row*Lx/4 + 8c + j, one value per site.
__device__ __forceinline__ void refresh_chunk(const Geom& g, int row, int c, int q, uint32_t rho, uint32_t r,
                                              uint32_t sw, const DaemonThresholds& th, V4& Me, V4& Mo)
{
    const uint32_t base = (uint32_t)row * (uint32_t)(g.Lx / 4) + 8u * (uint32_t)c;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const u32x4 a = philox10(base + 2u * i, rho, r, sw, g.key0, g.key1);
        const u32x4 b = philox10(base + 2u * i + 1u, rho, r, sw, g.key0, g.key1);
        // even site t = 8i + q + {0,2,4,6} of the 32; odd site t = 8i + (1-q) + {0,2,4,6}
        const uint32_t da[4] = {a.v0, a.v1, a.v2, a.v3};
        const uint32_t db[4] = {b.v0, b.v1, b.v2, b.v3};
        auto lvl = [&](uint32_t u) { return daemon_level(u, th); };
        const int qe = q, qo = 1 - q;
        Me.w[i] = lvl(da[qe]) | (lvl(da[qe + 2]) << 8) | (lvl(db[qe]) << 16) | (lvl(db[qe + 2]) << 24);
        Mo.w[i] = lvl(da[qo]) | (lvl(da[qo + 2]) << 8) | (lvl(db[qo]) << 16) | (lvl(db[qo + 2]) << 24);
    }
}

// Inputs of one step of the march (global loads issued ahead of use).
struct StepIn {
    V4 So, Se, Me, Mo;
    uint32_t mex, mox;  // edge words of a pending walker wandering (see load_step)
};

// PF = steps of loads in flight: 1, or 2 with two input sets used
// alternately (the march unrolled by two, so no register copy has to wait
// for a load still in flight).
// The two-step variant holds a second input set: it is built for
// work-groups of at most kPf2Lanes lanes (up to 170 VGPRs per lane).
constexpr int kPf2Lanes = 640;

template <bool REFRESH, int PF>
__global__ void __launch_bounds__(PF == 2 ? kPf2Lanes : 1024) k_micsa_sweep_fused(
    Geom g, FusedTile f, const uint8_t* __restrict__ spin_in, const uint8_t* __restrict__ dem_in,
    uint8_t* __restrict__ spin_out, uint8_t* __restrict__ dem_out, unsigned long long* __restrict__ tally,
    uint32_t rho, DaemonThresholds th, int wander)
{
    extern __shared__ uint4 lds[];
    const int rows_slots = f.TY + 4;
    const int plane_slots = rows_slots * f.NC;
    uint4* So = lds;                    // [2][TY+4][NC] odd spins of the current plane
    uint4* Xs = lds + 2 * plane_slots;  // [2][TY+4][NC] even views of the previous plane

    const int l = blockIdx.y;
    const int s = l / g.R, r = l % g.R;
    int ty, tz;
    tile_of(f, blockIdx.x, ty, tz);
    const int y0 = ty * f.TY, z0 = tz * f.TZ;
    // Odd z-tiles march downwards: the tiles on both sides of a z boundary
    // then reach its halo planes at the same time (both first or both last),
    // so the second read of those planes is an L2 hit.
    const int dz = (tz & 1) ? -1 : 1;
    const int zstart = dz > 0 ? z0 - 1 : z0 + f.TZ;
    const int ry = threadIdx.x / f.NC, c = threadIdx.x - ry * f.NC;
    const bool active = ry < rows_slots;
    int y = y0 - 2 + ry;
    y = y < 0 ? y + g.Ly : (y >= g.Ly ? y - g.Ly : y);
    const bool do_even = active && ry >= 1 && ry <= f.TY + 2;
    const bool do_odd = active && ry >= 2 && ry <= f.TY + 1;  // also the rows the tile owns

    const uint8_t* ev_in = spin_in + ((int64_t)l * 2 + 0) * g.Nh;
    const uint8_t* od_in = spin_in + ((int64_t)l * 2 + 1) * g.Nh;
    const uint8_t* me_in = dem_in + ((int64_t)l * 2 + 0) * g.Nh;
    const uint8_t* mo_in = dem_in + ((int64_t)l * 2 + 1) * g.Nh;
    uint8_t* ev_out = spin_out + ((int64_t)l * 2 + 0) * g.Nh;
    uint8_t* od_out = spin_out + ((int64_t)l * 2 + 1) * g.Nh;
    uint8_t* me_out = dem_out + ((int64_t)l * 2 + 0) * g.Nh;
    uint8_t* mo_out = dem_out + ((int64_t)l * 2 + 1) * g.Nh;
    const uint32_t sw = stream_word(kStreamDaemon, (uint32_t)s);

    auto wrapz = [&](int z) { return z < 0 ? z + g.Lz : (z >= g.Lz ? z - g.Lz : z); };
    auto hof = [&](int z) { return ((int64_t)y + (int64_t)g.Ly * z) * g.Kx + 16 * c; };
    const int cn = c + 1 == f.NC ? 0 : c + 1, cp = c == 0 ? f.NC - 1 : c - 1;
    const int steps = f.TZ + 2;

    // Step st works on plane z = zstart + dz st (even half) and z - dz (odd
    // half).  Global loads are issued PF steps ahead.
    V4 So_prev{}, So_cur{}, So_next{};  // odd spins (old) at planes z-dz, z, z+dz
    V4 X_prev2{}, X_prev{}, X_cur{};    // even views at planes z-2dz, z-dz, z
    V4 Mo_gen{};                        // refreshed odd levels of plane z-dz
    // Walkers (Sec. 2.6): with wander = p >= 0 the stored daemons have not yet
    // made the forward-X wandering of the sites of parity p that ended the
    // previous timestep; it is applied here, on load.  In a row with
    // q = (y + z) & 1 the even site k pairs with odd site k + q (p = 0), and
    // odd site k with even site k + 1 - q (p = 1).
    // The loads only fetch (the chunk and an edge word); the byte shift is
    // applied when the step uses them, so the prefetch stays asynchronous.
    auto row_of = [&](int z) { return ((int64_t)y + (int64_t)g.Ly * z) * g.Kx; };
    auto sh_even = [&](int z) { return wander == 0 ? ((y + z) & 1) : ((y + z) & 1) - 1; };
    auto sh_odd = [&](int z) { return wander == 0 ? -((y + z) & 1) : 1 - ((y + z) & 1); };
    auto load_step = [&](StepIn& in, int st2) {  // inputs of step st2 (plane z2 = zstart + dz st2)
        const int z2 = wrapz(zstart + dz * st2);
        in.mex = 0u;
        in.mox = 0u;
        if (active) in.So = ldg16(od_in + hof(wrapz(z2 + dz)));
        if (do_even) {
            const int64_t h2 = hof(z2);
            in.Se = ldg16(ev_in + h2);  // even spins with their bond bits
            if (!REFRESH) {
                if (wander < 0) {
                    in.Me = ldg16(me_in + h2);
                } else {  // new even daemons come from the odd array
                    const uint8_t* row = mo_in + row_of(z2);
                    in.Me = ldg16(row + 16 * c);
                    in.mex = *reinterpret_cast<const uint32_t*>(shift_edge(row, cn, cp, sh_even(z2)));
                }
            }
        }
        if (!REFRESH && do_odd && st2 >= 2) {
            const int zo2 = wrapz(z2 - dz);
            if (wander < 0) {
                in.Mo = ldg16(mo_in + hof(zo2));
            } else {  // new odd daemons come from the even array
                const uint8_t* row = me_in + row_of(zo2);
                in.Mo = ldg16(row + 16 * c);
                in.mox = *reinterpret_cast<const uint32_t*>(shift_edge(row, cn, cp, sh_odd(zo2)));
            }
        }
    };
    if (active) {
        So_prev = ldg16(od_in + hof(wrapz(zstart - dz)));
        So_cur = ldg16(od_in + hof(wrapz(zstart)));
    }
    StepIn inA{}, inB{};
    load_step(inA, 0);
    if (PF == 2 && steps > 1) load_step(inB, 1);
    uint32_t sum_old = 0, sum_new = 0;  // daemon level sums before/after owned moves
    auto step = [&](const int st, StepIn& in) {
        const int buf = st & 1;
        const int z = wrapz(zstart + dz * st);
        const int64_t h = hof(z);
        So_next = in.So;
        V4 Se = in.Se, Me = in.Me, Mo = in.Mo;
        if (!REFRESH && wander >= 0) {
            Me = shift_bytes(Me, in.mex, sh_even(z));
            Mo = shift_bytes(Mo, in.mox, sh_odd(wrapz(z - dz)));
        }
        V4 Mo_next{};
        if (st + PF < steps) load_step(in, st + PF);
        if (REFRESH && do_even) refresh_chunk(g, y + g.Ly * z, c, (y + z) & 1, rho, (uint32_t)r, sw, th, Me, Mo_next);
        const bool odd_now = do_odd && st >= 2;
        const int zo = wrapz(z - dz);
        if (active) sts16(&So[buf * plane_slots + ry * f.NC + c], So_cur);
        __syncthreads();
        // odd spins on planes z + 1 and z - 1 (old), even views on zo + 1 and zo - 1 (new)
        const V4& Sz_up = dz > 0 ? So_next : So_prev;
        const V4& Sz_dn = dz > 0 ? So_prev : So_next;
        const V4& Xz_up = dz > 0 ? X_cur : X_prev2;
        const V4& Xz_dn = dz > 0 ? X_prev2 : X_cur;

        if (do_even) {
            // ---- even half on plane z
            const int q = (y + z) & 1;
            const int dir = q ? 1 : -1;
            const uint4* row = &So[buf * plane_slots + ry * f.NC];
            const uint32_t nbw = dir > 0 ? row[cn].x : row[cp].w;
            const V4 A = So_cur;
            const V4 B = shift16(A, nbw, dir);
            const V4 Yp = lds16(&So[buf * plane_slots + (ry + 1) * f.NC + c]);
            const V4 Ym = lds16(&So[buf * plane_slots + (ry - 1) * f.NC + c]);
            // the same-k odd neighbour is across +x (q = 0) or -x (q = 1)
            const int dA = q ? kMx : kPx, dB = q ? kPx : kMx;
            const bool owned = do_odd && st >= 1 && st <= f.TZ;
            uint32_t so = 0, sn = 0;
            V4 Xn;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                // bit d of v = old spin ^ j_d: the bond term for neighbour nb is nb ^ ((v >> d) & 1)
                const uint32_t m1 = 0x01010101u;
                const uint32_t W = Se.w[i];  // spin in bit 0, bond d in bit 1 + d
                uint32_t S = W & m1;
                const uint32_t v = xor_and(times63(S), W >> 1, 0x3F3F3F3Fu);
                const uint32_t u = xor_and(A.w[i], v >> dA, m1) + xor_and(B.w[i], v >> dB, m1) +
                                   xor_and(Yp.w[i], v >> kPy, m1) + xor_and(Ym.w[i], v >> kMy, m1) +
                                   xor_and(Sz_up.w[i], v >> kPz, m1) + xor_and(Sz_dn.w[i], v >> kMz, m1);
                const uint32_t S0 = S;
                creutz4(S, Me.w[i], u, so, sn);
                const uint32_t flip = S ^ S0;
                Se.w[i] = W ^ flip;
                Xn.w[i] = v ^ times63(flip);  // even view: bit d = new spin ^ j_d
            }
            X_cur = Xn;
            sts16(&Xs[buf * plane_slots + ry * f.NC + c], Xn);
            if (owned) {  // ring rows and halo planes are recomputed, not owned
                stg16_nt(ev_out + h, Se.w);
                stg16_nt(me_out + h, Me.w);
                sum_old += so;
                sum_new += sn;
            }
        }
        if (odd_now) {
            // ---- odd half on plane zo = z - dz (its even neighbours are all final)
            const int q = (y + zo) & 1;
            const int dir = q ? -1 : 1;
            const int pb = buf ^ 1;
            const uint4* row = &Xs[pb * plane_slots + ry * f.NC];
            const uint32_t nbw = dir > 0 ? row[cn].x : row[cp].w;
            const V4 A = X_prev;
            const V4 B = shift16(A, nbw, dir);
            const V4 Yp = lds16(&Xs[pb * plane_slots + (ry + 1) * f.NC + c]);
            const V4 Ym = lds16(&Xs[pb * plane_slots + (ry - 1) * f.NC + c]);
            const int dA = q ? kMx : kPx, dB = q ? kPx : kMx;
            if (REFRESH) Mo = Mo_gen;
            V4 So_new;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                uint32_t S = So_prev.w[i];
                const uint32_t m1 = 0x01010101u;
                const uint32_t u = xor_and(S, A.w[i] >> dA, m1) + xor_and(S, B.w[i] >> dB, m1) +
                                   xor_and(S, Yp.w[i] >> kMy, m1) + xor_and(S, Ym.w[i] >> kPy, m1) +
                                   xor_and(S, Xz_up.w[i] >> kMz, m1) + xor_and(S, Xz_dn.w[i] >> kPz, m1);
                creutz4(S, Mo.w[i], u, sum_old, sum_new);
                So_new.w[i] = S;
            }
            const int64_t ho = hof(zo);
            stg16_nt(od_out + ho, So_new.w);
            stg16_nt(mo_out + ho, Mo.w);
        }
        So_prev = So_cur;
        So_cur = So_next;
        X_prev2 = X_prev;
        X_prev = X_cur;
        Mo_gen = Mo_next;
    };
    for (int st = 0; st < steps; st += PF) {
        step(st, inA);
        if (PF == 2 && st + 1 < steps) step(st + 1, inB);
    }
    // dH = 4 (sum of old levels - sum of new levels) over the owned moves
    block_add(tally + (int64_t)l * kSlots, 4 * ((long long)sum_old - (long long)sum_new));
}

// Fused sweep of the random-number-greedy baselines (ALG 0 heat bath, ALG 1
// Metropolis; canonical4): same z-march, tiles, rings and LDS exchange as
// k_micsa_sweep_fused, with one 32-bit uniform per visited site,
// u = Philox(h>>2, 2k+p, r, stream | s)[h & 3] for its parity-split index h.
// No daemons.
template <int ALG>
__global__ void __launch_bounds__(1024) k_heatbath_sweep_fused(
    Geom g, FusedTile f, const uint8_t* __restrict__ spin_in, uint8_t* __restrict__ spin_out,
    unsigned long long* __restrict__ tally, uint32_t time0, HeatBathThresholds th)
{
    extern __shared__ uint4 lds[];
    __shared__ uint64_t tau[8];
    if (threadIdx.x < 7) tau[threadIdx.x] = th.tau[threadIdx.x];
    const int rows_slots = f.TY + 4;
    const int plane_slots = rows_slots * f.NC;
    uint4* So = lds;
    uint4* Xs = lds + 2 * plane_slots;

    const int l = blockIdx.y;
    const int s = l / g.R, r = l % g.R;
    int ty, tz;
    tile_of(f, blockIdx.x, ty, tz);
    const int y0 = ty * f.TY, z0 = tz * f.TZ;
    const int ry = threadIdx.x / f.NC, c = threadIdx.x - ry * f.NC;
    const bool active = ry < rows_slots;
    int y = y0 - 2 + ry;
    y = y < 0 ? y + g.Ly : (y >= g.Ly ? y - g.Ly : y);
    const bool do_even = active && ry >= 1 && ry <= f.TY + 2;
    const bool do_odd = active && ry >= 2 && ry <= f.TY + 1;

    const uint8_t* ev_in = spin_in + ((int64_t)l * 2 + 0) * g.Nh;
    const uint8_t* od_in = spin_in + ((int64_t)l * 2 + 1) * g.Nh;
    uint8_t* ev_out = spin_out + ((int64_t)l * 2 + 0) * g.Nh;
    uint8_t* od_out = spin_out + ((int64_t)l * 2 + 1) * g.Nh;
    const uint32_t sw = canonical_stream<ALG>((uint32_t)s);

    auto wrapz = [&](int z) { return z < 0 ? z + g.Lz : (z >= g.Lz ? z - g.Lz : z); };
    auto hof = [&](int z) { return ((int64_t)y + (int64_t)g.Ly * z) * g.Kx + 16 * c; };
    const int cn = c + 1 == f.NC ? 0 : c + 1, cp = c == 0 ? f.NC - 1 : c - 1;
    const int steps = f.TZ + 2;

    V4 So_prev{}, So_cur{}, So_next{};
    V4 X_prev2{}, X_prev{}, X_cur{};
    V4 nSo{}, nSe{};
    auto load_step = [&](int st2) {
        const int z2 = wrapz(z0 - 1 + st2);
        if (active) nSo = ldg16(od_in + hof(wrapz(z2 + 1)));
        if (do_even) {
            const int64_t h2 = hof(z2);
            nSe = ldg16(ev_in + h2);
        }
    };
    if (active) {
        So_prev = ldg16(od_in + hof(wrapz(z0 - 2)));
        So_cur = ldg16(od_in + hof(wrapz(z0 - 1)));
    }
    load_step(0);
    int dE = 0;
    for (int st = 0; st < steps; ++st) {
        const int buf = st & 1;
        const int z = wrapz(z0 - 1 + st);
        const int64_t h = hof(z);
        So_next = nSo;
        V4 Se = nSe;
        if (st + 1 < steps) load_step(st + 1);
        const bool odd_now = do_odd && st >= 2;
        const int zo = wrapz(z - 1);
        if (active) sts16(&So[buf * plane_slots + ry * f.NC + c], So_cur);
        __syncthreads();

        if (do_even) {
            const int q = (y + z) & 1;
            const int dir = q ? 1 : -1;
            const uint4* row = &So[buf * plane_slots + ry * f.NC];
            const uint32_t nbw = dir > 0 ? row[cn].x : row[cp].w;
            const V4 A = So_cur;
            const V4 B = shift16(A, nbw, dir);
            const V4 Yp = lds16(&So[buf * plane_slots + (ry + 1) * f.NC + c]);
            const V4 Ym = lds16(&So[buf * plane_slots + (ry - 1) * f.NC + c]);
            const int dA = q ? kMx : kPx, dB = q ? kPx : kMx;
            const bool owned = do_odd && st >= 1 && st <= f.TZ;
            int dEe = 0;
            V4 Xn;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t m1 = 0x01010101u;
                const uint32_t W = Se.w[i];  // spin in bit 0, bond d in bit 1 + d
                const uint32_t jw = (W >> 1) & 0x3F3F3F3Fu;
                const uint32_t v = xor_and(A.w[i], jw >> dA, m1) + xor_and(B.w[i], jw >> dB, m1) +
                                   xor_and(Yp.w[i], jw >> kPy, m1) + xor_and(Ym.w[i], jw >> kMy, m1) +
                                   xor_and(So_next.w[i], jw >> kPz, m1) + xor_and(So_prev.w[i], jw >> kMz, m1);
                const uint32_t ctr = (uint32_t)((h >> 2) + i);
                const u32x4 rnd = philox10(ctr, time0, (uint32_t)r, sw, g.key0, g.key1);
                const uint32_t S = canonical4<ALG>(W, v, rnd, tau, dEe);
                Se.w[i] = S | (W & ~m1);
                Xn.w[i] = times63(S) ^ jw;
            }
            X_cur = Xn;
            sts16(&Xs[buf * plane_slots + ry * f.NC + c], Xn);
            if (owned) {
                stg16(ev_out + h, Se);
                dE += dEe;
            }
        }
        if (odd_now) {
            const int q = (y + zo) & 1;
            const int dir = q ? -1 : 1;
            const int pb = buf ^ 1;
            const uint4* row = &Xs[pb * plane_slots + ry * f.NC];
            const uint32_t nbw = dir > 0 ? row[cn].x : row[cp].w;
            const V4 A = X_prev;
            const V4 B = shift16(A, nbw, dir);
            const V4 Yp = lds16(&Xs[pb * plane_slots + (ry + 1) * f.NC + c]);
            const V4 Ym = lds16(&Xs[pb * plane_slots + (ry - 1) * f.NC + c]);
            const int dA = q ? kMx : kPx, dB = q ? kPx : kMx;
            const int64_t ho = hof(zo);
            V4 So_new;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const uint32_t m1 = 0x01010101u;
                const uint32_t v = ((A.w[i] >> dA) & m1) + ((B.w[i] >> dB) & m1) + ((Yp.w[i] >> kMy) & m1) +
                                   ((Ym.w[i] >> kPy) & m1) + ((X_cur.w[i] >> kMz) & m1) +
                                   ((X_prev2.w[i] >> kPz) & m1);
                const uint32_t ctr = (uint32_t)((ho >> 2) + i);
                const u32x4 rnd = philox10(ctr, time0 + 1u, (uint32_t)r, sw, g.key0, g.key1);
                So_new.w[i] = canonical4<ALG>(So_prev.w[i], v, rnd, tau, dE);
            }
            stg16(od_out + ho, So_new);
        }
        So_prev = So_cur;
        So_cur = So_next;
        X_prev2 = X_prev;
        X_prev = X_cur;
    }
    block_add(tally + (int64_t)l * kSlots, dE);
}

}  // namespace micsa
