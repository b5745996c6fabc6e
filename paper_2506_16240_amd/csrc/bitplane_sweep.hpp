// One launch per MicSA sweep in the bit-plane layout (multispin coding
// across lattices, Sec. 2.5 and App. B): the 64 bits of a word are the same
// site of 64 lattices, so one Creutz move on a word updates 64 lattices.
//
// A work-group owns TZ consecutive planes of one word lattice (all rows and
// all words of each plane).  Both halves of the sweep (Sec. 2.8: even
// sublattice, then odd) run inside the work-group:
//   1. the old odd spins of planes z0 - 2 .. z0 + TZ + 1 are staged in LDS;
//   2. the even half runs on planes z0 - 1 .. z0 + TZ (one ring plane on
//      each side that another work-group owns, recomputed here from the same
//      old values, so no work-group waits for another) and leaves the new
//      even spins in LDS;
//   3. barrier; the odd half runs on the owned planes with its neighbours'
//      new even spins from LDS.
// State is read from the "in" arrays and written to the "out" arrays (the
// host swaps them after the launch), so ring reads always see old values.
// The levels are read from the level arrays passed in: the state's own
// levels, or at a refresh point the freshly drawn ones.
//
// Word layout (bitplane_kernels.hpp): spin/dm0/dm1 [WL][2][Nh], coupling
// words Jw [NJ][6][Nh] of the even sites; the parity split of the byte layout
// puts the x neighbours of word k at k and k +- 1 of the other parity's row,
// the y and z neighbours at the same k of the adjacent rows.
//
// Move (Sec. 2.3, eq. flip-OK with the capacity of Sec. 2.5), bit-sliced on
// 64 lanes: the six unsatisfied-bond bits s ^ neighbour ^ j are counted into
// u = (u2 u1 u0) by two carry-save adders, w = m + u, the flip is taken iff
// 3 <= w <= 6 and then m' = w - 3 -- the same boolean algebra as the
// multispin sweep (msc_move), three-input XOR and majority as v_bitop3.
//
// Incremental energy tally per lane (TALLY): energy plus daemon energy is
// conserved by every move (eq. H-total), so the lattice energy changes by
// 4 (sum m - sum m') over the moves.  Each thread adds m + (3 - m') of every
// word it owns into a vertical counter (bit plane b holds bit b of the
// per-lane count); half the waves take the other half's counters through
// LDS and sum them over their lanes by a butterfly of bit-sliced adders;
// each lane then reads its lattice's count, and the counts are summed in
// LDS and added to the lane's lattice (bp_tally_counts).
#pragma once
#include "bitplane_kernels.hpp"
#include "msc_kernels.hpp"

namespace micsa {

struct BpTile {
    int32_t TZ;   // planes a work-group owns (divides Lz)
    int32_t ntz;  // Lz / TZ
    int32_t P;    // words of one parity per plane = Ly * Kx
    int32_t TY;   // kb_sweep_rows: rows a work-group owns (the last tile along y what is left of Ly)
    int32_t nty;  // kb_sweep_rows: tiles along y
};

constexpr int kBpLanes = 1024;  // largest work-group
constexpr int kBpPlanes = 5;    // vertical counter planes per thread: counts up to 31 (a thread owns at
                                // most 4 words, each adding at most 6)

// The move on 64 lanes (a[] the six unsatisfied-bond bits); returns the new
// spins, updates the levels.
__device__ __forceinline__ uint64_t bp_move(uint64_t s, const uint64_t (&a)[6], uint64_t& m0, uint64_t& m1)
{
    const uint64_t s1 = xor3(a[0], a[1], a[2]), c1 = maj3w(a[0], a[1], a[2]);
    const uint64_t s2 = xor3(a[3], a[4], a[5]), c2 = maj3w(a[3], a[4], a[5]);
    const uint64_t u0 = s1 ^ s2, k0 = s1 & s2;
    const uint64_t u1 = xor3(c1, c2, k0), u2 = maj3w(c1, c2, k0);
    const uint64_t w0 = m0 ^ u0, cw0 = m0 & u0;
    const uint64_t w1 = xor3(m1, u1, cw0), cw1 = maj3w(m1, u1, cw0);
    const uint64_t w2 = u2 ^ cw1, w3 = u2 & cw1;
    const uint64_t acc = ~w3 & (w2 ^ (w1 & w0));
    const uint64_t n0 = (acc & ~w0) | (~acc & m0);
    const uint64_t n1 = (acc & (w2 & (w1 | w0))) | (~acc & m1);
    m0 = n0;
    m1 = n1;
    return s ^ acc;
}

// Vertical counter: add the bit plane v at weight 2^from.
template <int NP>
__device__ __forceinline__ void vc_add(uint64_t (&c)[NP], uint64_t v, int from)
{
#pragma unroll
    for (int b = 0; b < NP; ++b)
        if (b >= from) {
            const uint64_t t = c[b] & v;
            c[b] ^= v;
            v = t;
        }
}

// 64-bit lane move by DPP (32-bit halves); lanes of rows outside ROWMASK read 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ uint64_t dpp64(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, ROWMASK, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, ROWMASK, 0xF, false);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

// One level of the wave reduction: add the counter of the lane the DPP
// control names (bit-sliced ripple adder over the first NP planes).
template <int CTRL, int ROWMASK, int NP, int NW>
__device__ __forceinline__ void vc_dpp_level(uint64_t (&c)[NW])
{
    uint64_t carry = 0;
#pragma unroll
    for (int b = 0; b < NP; ++b) {
        const uint64_t o = dpp64<CTRL, ROWMASK>(c[b]);
        const uint64_t sum = xor3(c[b], o, carry);
        carry = maj3w(c[b], o, carry);
        c[b] = sum;
    }
}

// Per lane: m_old + (3 - m_new) of one word into the counter.
template <int NP>
__device__ __forceinline__ void vc_word(uint64_t (&c)[NP], uint64_t o0, uint64_t o1, uint64_t n0, uint64_t n1)
{
    // (o1 o0) + (~n1 ~n0): bit 0 sum and carry, then bit 1 with the carry
    const uint64_t a0 = ~n0, a1 = ~n1;
    const uint64_t s0 = o0 ^ a0, k0 = o0 & a0;
    const uint64_t s1 = xor3(o1, a1, k0), k1 = maj3w(o1, a1, k0);
    vc_add(c, s0, 0);
    vc_add(c, s1, 1);
    vc_add(c, k1, 2);
}

// Per-lane tally counts of a work-group.  Waves w >= H (H: half the waves,
// rounded up) hand their vertical counters to wave w - H through LDS; the H
// waves (one or two per SIMD) add them and sum their counters over the 64
// lanes into lane 63 by bit-sliced adders over DPP lane moves (within rows of
// 16: swap neighbours, swap pairs, rotate by 4 and by 8; then the last lane
// of row 0 into row 1, of rows 2 / 3 ... as row broadcasts); each lane reads
// its lattice's count out of lane 63's planes; the H waves' counts meet in
// LDS.  Returns the lane's total in threads < 64 (0 elsewhere).  Starts with
// a barrier, after which the caller's LDS is reused.
__device__ __forceinline__ long long bp_tally_counts(const uint64_t (&cnt)[kBpPlanes], uint64_t* lds)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwaves = (blockDim.x + 63) >> 6, H = (nwaves + 1) >> 1;
    __syncthreads();  // the caller's LDS planes are no longer read
    if (wave >= H) {
#pragma unroll
        for (int b = 0; b < kBpPlanes; ++b) lds[((wave - H) * kBpPlanes + b) * 64 + lane] = cnt[b];
    }
    __syncthreads();
    long long mine = 0;
    if (wave < H) {  // uniform per wave: DPP moves see every lane
        constexpr int NP0 = kBpPlanes + 1;  // a wave's counter plus its partner's
        constexpr int NW = NP0 + 6;
        uint64_t c[NW];
#pragma unroll
        for (int b = 0; b < NW; ++b) c[b] = b < kBpPlanes ? cnt[b] : 0;
        if (wave + H < nwaves) {
            uint64_t carry = 0;
#pragma unroll
            for (int b = 0; b < NP0; ++b) {
                const uint64_t x = b < kBpPlanes ? lds[(wave * kBpPlanes + b) * 64 + lane] : 0;
                const uint64_t sum = xor3(c[b], x, carry);
                carry = maj3w(c[b], x, carry);
                c[b] = sum;
            }
        }
        vc_dpp_level<0xB1, 0xF, NP0 + 1>(c);   // quad_perm [1,0,3,2]
        vc_dpp_level<0x4E, 0xF, NP0 + 2>(c);   // quad_perm [2,3,0,1]
        vc_dpp_level<0x124, 0xF, NP0 + 3>(c);  // row_ror:4
        vc_dpp_level<0x128, 0xF, NP0 + 4>(c);  // row_ror:8
        vc_dpp_level<0x142, 0xA, NP0 + 5>(c);  // row_bcast:15 into rows 1, 3
        vc_dpp_level<0x143, 0xC, NP0 + 6>(c);  // row_bcast:31 into rows 2, 3
#pragma unroll
        for (int b = 0; b < NW; ++b) {
            const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)c[b], 63);
            const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(c[b] >> 32), 63);
            const uint32_t bit = lane < 32 ? (lo >> lane) & 1u : (hi >> (lane - 32)) & 1u;
            mine += (long long)bit << b;
        }
    }
    __syncthreads();  // the handed-over counters are no longer read
    long long* part = reinterpret_cast<long long*>(lds);
    if (wave < H) part[wave * 64 + lane] = mine;
    __syncthreads();
    long long total = 0;
    if (threadIdx.x < 64)
        for (int w = 0; w < H; ++w) total += part[w * 64 + threadIdx.x];
    return total;
}

// One thread per word position of a plane (P <= block); every global load of
// the sweep is issued at the start (old odd spins of the TZ + 4 ring-extended
// planes, the even words with their couplings and levels of TZ + 2 planes,
// the odd levels and their even neighbours' couplings of the TZ owned planes),
// so the work-group waits for memory once.
template <bool TALLY, int TZ>
__global__ __launch_bounds__(TZ == 1 ? 1024 : 512) void kb_sweep(GeomB gb, BpTile f,
                                                                const uint64_t* __restrict__ spin_in,
                                                                const uint64_t* __restrict__ d0_in,
                                                                const uint64_t* __restrict__ d1_in,
                                                                const uint64_t* __restrict__ Jw,
                                                                uint64_t* __restrict__ spin_out,
                                                                uint64_t* __restrict__ d0_out,
                                                                uint64_t* __restrict__ d1_out,
                                                                unsigned long long* __restrict__ tally)
{
    extern __shared__ uint64_t lds_bp[];
    uint64_t* lds = lds_bp;
    const Geom& g = gb.g;
    // One-dimensional grid over (word lattice, z tile).  Work-groups go round
    // robin over the 8 XCDs (block b on XCD b % 8), each with its own L2; when
    // the tile count divides by 8, XCD x takes the contiguous tiles [x T/8,
    // (x + 1) T/8) -- consecutive z tiles of one word lattice, whose ring
    // planes its L2 then serves.
    const int ntiles = gridDim.x;
    int t = blockIdx.x;
    if ((ntiles & 7) == 0) t = (t & 7) * (ntiles >> 3) + (t >> 3);
    const int wl = t / f.ntz;
    const int z0 = (t - wl * f.ntz) * TZ;
    const int P = f.P;
    const int64_t Nh = g.Nh;
    uint64_t* LO = lds;                        // old odd spins, planes z0 - 2 .. z0 + TZ + 1
    uint64_t* LE = lds + (size_t)(TZ + 4) * P;  // new even spins, planes z0 - 1 .. z0 + TZ
    const uint64_t* ev_in = spin_in + (int64_t)wl * 2 * Nh;
    const uint64_t* od_in = ev_in + Nh;
    const uint64_t* m0e = d0_in + (int64_t)wl * 2 * Nh;
    const uint64_t* m1e = d1_in + (int64_t)wl * 2 * Nh;
    uint64_t* ev_out = spin_out + (int64_t)wl * 2 * Nh;
    uint64_t* n0e = d0_out + (int64_t)wl * 2 * Nh;
    uint64_t* n1e = d1_out + (int64_t)wl * 2 * Nh;
    const uint64_t* J = Jw + (int64_t)bp_cset(gb, wl) * 6 * Nh;
    auto wrapz = [&](int z) { return z < 0 ? z + g.Lz : (z >= g.Lz ? z - g.Lz : z); };
    const int pos = threadIdx.x;
    const bool live = pos < P;
    const int pq = live ? pos : 0;  // idle lanes read position 0 (in bounds) and store nothing
    const int y = pq / g.Kx, k = pq - y * g.Kx;
    const int yp = y + 1 == g.Ly ? 0 : y + 1, ym = y == 0 ? g.Ly - 1 : y - 1;
    const int kp = k + 1 == g.Kx ? 0 : k + 1, km = k == 0 ? g.Kx - 1 : k - 1;

    // ---- every load of the sweep
    uint64_t Od[TZ + 4];
#pragma unroll
    for (int e = 0; e < TZ + 4; ++e) Od[e] = od_in[(int64_t)wrapz(z0 - 2 + e) * P + pq];
    uint64_t Es[TZ + 2], Ej[TZ + 2][6], Em0[TZ + 2], Em1[TZ + 2];
#pragma unroll
    for (int e = 0; e < TZ + 2; ++e) {
        const int z = wrapz(z0 - 1 + e);
        const int64_t h = (int64_t)z * P + pq;
        const int q = (y + z) & 1;
        const int dA = q ? kMx : kPx, dB = q ? kPx : kMx;
        Es[e] = ev_in[h];
        Ej[e][0] = J[dA * Nh + h];
        Ej[e][1] = J[dB * Nh + h];
        Ej[e][2] = J[kPy * Nh + h];
        Ej[e][3] = J[kMy * Nh + h];
        Ej[e][4] = J[kPz * Nh + h];
        Ej[e][5] = J[kMz * Nh + h];
        Em0[e] = m0e[h];
        Em1[e] = m1e[h];
    }
    uint64_t Oj[TZ][6], Om0[TZ], Om1[TZ];
#pragma unroll
    for (int e = 0; e < TZ; ++e) {
        // an odd site's coupling is its even neighbour's in the opposite direction
        const int z = wrapz(z0 + e), zp = wrapz(z0 + e + 1), zm = wrapz(z0 + e - 1);
        const int64_t h = (int64_t)z * P + pq;
        const int q = (y + z) & 1;
        const int ks = q ? km : kp;
        const int dA = q ? kMx : kPx, dB = q ? kPx : kMx;
        Oj[e][0] = J[dA * Nh + h];
        Oj[e][1] = J[dB * Nh + (int64_t)z * P + y * g.Kx + ks];
        Oj[e][2] = J[kMy * Nh + (int64_t)z * P + yp * g.Kx + k];
        Oj[e][3] = J[kPy * Nh + (int64_t)z * P + ym * g.Kx + k];
        Oj[e][4] = J[kMz * Nh + (int64_t)zp * P + pq];
        Oj[e][5] = J[kPz * Nh + (int64_t)zm * P + pq];
        Om0[e] = m0e[Nh + h];
        Om1[e] = m1e[Nh + h];
    }

    // ---- old odd spins of the ring-extended slab into LDS
    if (live) {
#pragma unroll
        for (int e = 0; e < TZ + 4; ++e) LO[(size_t)e * P + pos] = Od[e];
    }
    __syncthreads();

    uint64_t cnt[kBpPlanes];
#pragma unroll
    for (int b = 0; b < kBpPlanes; ++b) cnt[b] = 0;

    // ---- even half on planes z0 - 1 .. z0 + TZ (the first and last recomputed ring planes)
#pragma unroll
    for (int e = 0; e < TZ + 2; ++e) {
        const int z = wrapz(z0 - 1 + e);
        const int q = (y + z) & 1;
        const int ks = q ? kp : km;
        const uint64_t* Oz = LO + (size_t)(e + 1) * P;  // odd plane z0 - 1 + e
        const uint64_t S = Es[e];
        const uint64_t nb[6] = {Oz[pq], Oz[y * g.Kx + ks], Oz[yp * g.Kx + k], Oz[ym * g.Kx + k], (Oz + P)[pq],
                                (Oz - P)[pq]};
        const uint64_t a[6] = {xor3(S, nb[0], Ej[e][0]), xor3(S, nb[1], Ej[e][1]), xor3(S, nb[2], Ej[e][2]),
                               xor3(S, nb[3], Ej[e][3]), xor3(S, nb[4], Ej[e][4]), xor3(S, nb[5], Ej[e][5])};
        uint64_t M0 = Em0[e], M1 = Em1[e];
        const uint64_t Sn = bp_move(S, a, M0, M1);
        if (live) {
            LE[(size_t)e * P + pos] = Sn;
            if (e >= 1 && e <= TZ) {  // a plane this work-group owns
                const int64_t h = (int64_t)z * P + pos;
                ev_out[h] = Sn;
                n0e[h] = M0;
                n1e[h] = M1;
                if (TALLY) vc_word(cnt, Em0[e], Em1[e], M0, M1);
            }
        }
    }
    __syncthreads();

    // ---- odd half on the owned planes, with the new even spins
#pragma unroll
    for (int e = 0; e < TZ; ++e) {
        const int z = wrapz(z0 + e);
        const int q = (y + z) & 1;
        const int ks = q ? km : kp;
        const uint64_t* Ez = LE + (size_t)(e + 1) * P;  // new even plane z0 + e
        const uint64_t S = Od[e + 2];
        const uint64_t nb[6] = {Ez[pq], Ez[y * g.Kx + ks], Ez[yp * g.Kx + k], Ez[ym * g.Kx + k], (Ez + P)[pq],
                                (Ez - P)[pq]};
        const uint64_t a[6] = {xor3(S, nb[0], Oj[e][0]), xor3(S, nb[1], Oj[e][1]), xor3(S, nb[2], Oj[e][2]),
                               xor3(S, nb[3], Oj[e][3]), xor3(S, nb[4], Oj[e][4]), xor3(S, nb[5], Oj[e][5])};
        uint64_t M0 = Om0[e], M1 = Om1[e];
        const uint64_t Sn = bp_move(S, a, M0, M1);
        if (live) {
            const int64_t h = (int64_t)z * P + pos;
            ev_out[Nh + h] = Sn;
            n0e[Nh + h] = M0;
            n1e[Nh + h] = M1;
            if (TALLY) vc_word(cnt, Om0[e], Om1[e], M0, M1);
        }
    }
    if (TALLY) {
        // 4. per-lane tally: the work-group's counts per lane (bp_tally_counts)
        const long long sum = bp_tally_counts(cnt, lds);
        if (threadIdx.x < 64) {
            // every lane counted m + (3 - m') over the 2 TZ P words the group owns
            const long long dE = 4 * (sum - 3ll * 2 * TZ * P);
            int s, r;
            if (dE != 0 && bp_lattice(gb, wl, (int)threadIdx.x, s, r))
                atomicAdd(&tally[((int64_t)s * g.R + r) * kSlots + (t % kSlots)], (unsigned long long)dE);
        }
    }
}


// Planes of more than 1024 words: a work-group owns TY rows (f.TY; the last
// tile along y what is left of Ly) of one plane of one word lattice, with two
// ring rows on each side.  The old odd spins are staged on the TY + 4 rows
// of planes z - 2 .. z + 2; the even half runs on planes z - 1 .. z + 1 and
// on the TY + 2 rows whose results the odd half reads (ring rows and planes
// recomputed from the same old values as their owners, so no work-group
// waits for another); the odd half runs on the owned rows of plane z.  One
// thread per word position of the TY + 4 rows; every global load is issued
// at the start, as in kb_sweep.  Lanes of a ragged last tile beyond its rows
// load their tile's last row and store nothing.
template <bool TALLY>
__global__ __launch_bounds__(1024) void kb_sweep_rows(GeomB gb, BpTile f, const uint64_t* __restrict__ spin_in,
                                                      const uint64_t* __restrict__ d0_in,
                                                      const uint64_t* __restrict__ d1_in,
                                                      const uint64_t* __restrict__ Jw,
                                                      uint64_t* __restrict__ spin_out,
                                                      uint64_t* __restrict__ d0_out,
                                                      uint64_t* __restrict__ d1_out,
                                                      unsigned long long* __restrict__ tally)
{
    extern __shared__ uint64_t lds_bp[];
    const Geom& g = gb.g;
    // one-dimensional grid over (word lattice, plane, y tile), y tiles
    // fastest; XCD x takes a contiguous run of tiles when their count divides by 8
    const int ntiles = gridDim.x;
    int t = blockIdx.x;
    if ((ntiles & 7) == 0) t = (t & 7) * (ntiles >> 3) + (t >> 3);
    const int per_wl = f.ntz * f.nty;
    const int wl = t / per_wl;
    const int rem = t - wl * per_wl;
    const int z = rem / f.nty, ty = rem - z * f.nty;
    const int y0 = ty * f.TY;
    const int own = min(f.TY, g.Ly - y0);
    const int Kx = g.Kx;
    const int PT = (f.TY + 4) * Kx;  // words of one LDS plane
    const int P = f.P;
    const int64_t Nh = g.Nh;
    uint64_t* LO = lds_bp;           // old odd spins, planes z - 2 .. z + 2, rows y0 - 2 .. y0 + TY + 1
    uint64_t* LE = lds_bp + 5 * PT;  // new even spins, planes z - 1 .. z + 1
    const uint64_t* ev_in = spin_in + (int64_t)wl * 2 * Nh;
    const uint64_t* od_in = ev_in + Nh;
    const uint64_t* m0e = d0_in + (int64_t)wl * 2 * Nh;
    const uint64_t* m1e = d1_in + (int64_t)wl * 2 * Nh;
    uint64_t* ev_out = spin_out + (int64_t)wl * 2 * Nh;
    uint64_t* n0e = d0_out + (int64_t)wl * 2 * Nh;
    uint64_t* n1e = d1_out + (int64_t)wl * 2 * Nh;
    const uint64_t* J = Jw + (int64_t)bp_cset(gb, wl) * 6 * Nh;
    auto wrapz = [&](int v) { return v < 0 ? v + g.Lz : (v >= g.Lz ? v - g.Lz : v); };
    auto wrapy = [&](int v) {
        v %= g.Ly;
        return v < 0 ? v + g.Ly : v;
    };
    const int pos = threadIdx.x;
    const int r0 = pos / Kx, k = pos - r0 * Kx;
    const bool active = r0 < own + 4;
    const int r = active ? r0 : own + 3;  // tile row
    const int me = r * Kx + k;
    const int rup = min(r + 1, own + 3), rdn = max(r - 1, 0);  // in-tile rows r +- 1 (clamped at the ring's edge)
    const int y = wrapy(y0 - 2 + r), yp = wrapy(y0 - 1 + r), ym = wrapy(y0 - 3 + r);
    const int kp = k + 1 == Kx ? 0 : k + 1, km = k == 0 ? Kx - 1 : k - 1;
    const bool own_row = active && r >= 2 && r <= own + 1;
    const int yw = y * Kx;

    // ---- every load of the sweep
    uint64_t Od[5];
#pragma unroll
    for (int e = 0; e < 5; ++e) Od[e] = od_in[(int64_t)wrapz(z - 2 + e) * P + yw + k];
    uint64_t Es[3], Ej[3][6], Em0[3], Em1[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int zz = wrapz(z - 1 + e);
        const int64_t h = (int64_t)zz * P + yw + k;
        const int q = (y + zz) & 1;
        const int dA = q ? kMx : kPx, dB = q ? kPx : kMx;
        Es[e] = ev_in[h];
        Ej[e][0] = J[dA * Nh + h];
        Ej[e][1] = J[dB * Nh + h];
        Ej[e][2] = J[kPy * Nh + h];
        Ej[e][3] = J[kMy * Nh + h];
        Ej[e][4] = J[kPz * Nh + h];
        Ej[e][5] = J[kMz * Nh + h];
        Em0[e] = m0e[h];
        Em1[e] = m1e[h];
    }
    uint64_t Oj[6], Om0, Om1;
    {
        // an odd site's coupling is its even neighbour's in the opposite direction
        const int zp = wrapz(z + 1), zm = wrapz(z - 1);
        const int64_t h = (int64_t)z * P + yw + k;
        const int q = (y + z) & 1;
        const int ks = q ? km : kp;
        const int dA = q ? kMx : kPx, dB = q ? kPx : kMx;
        Oj[0] = J[dA * Nh + h];
        Oj[1] = J[dB * Nh + (int64_t)z * P + yw + ks];
        Oj[2] = J[kMy * Nh + (int64_t)z * P + yp * Kx + k];
        Oj[3] = J[kPy * Nh + (int64_t)z * P + ym * Kx + k];
        Oj[4] = J[kMz * Nh + (int64_t)zp * P + yw + k];
        Oj[5] = J[kPz * Nh + (int64_t)zm * P + yw + k];
        Om0 = m0e[Nh + h];
        Om1 = m1e[Nh + h];
    }

    // ---- old odd spins of the ring-extended tile into LDS
    if (active) {
#pragma unroll
        for (int e = 0; e < 5; ++e) LO[(size_t)e * PT + me] = Od[e];
    }
    __syncthreads();

    uint64_t cnt[kBpPlanes];
#pragma unroll
    for (int b = 0; b < kBpPlanes; ++b) cnt[b] = 0;

    // ---- even half on planes z - 1 .. z + 1 (rows 1 .. own + 2 are read by the odd half)
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int zz = wrapz(z - 1 + e);
        const int q = (y + zz) & 1;
        const int ks = q ? kp : km;
        const uint64_t* Oz = LO + (size_t)(e + 1) * PT;  // odd plane z - 1 + e
        const uint64_t S = Es[e];
        const uint64_t nb[6] = {Oz[me], Oz[r * Kx + ks], Oz[rup * Kx + k], Oz[rdn * Kx + k], (Oz + PT)[me],
                                (Oz - PT)[me]};
        const uint64_t a[6] = {xor3(S, nb[0], Ej[e][0]), xor3(S, nb[1], Ej[e][1]), xor3(S, nb[2], Ej[e][2]),
                               xor3(S, nb[3], Ej[e][3]), xor3(S, nb[4], Ej[e][4]), xor3(S, nb[5], Ej[e][5])};
        uint64_t M0 = Em0[e], M1 = Em1[e];
        const uint64_t Sn = bp_move(S, a, M0, M1);
        if (active) LE[(size_t)e * PT + me] = Sn;
        if (e == 1 && own_row) {  // the owned plane and rows
            const int64_t h = (int64_t)z * P + yw + k;
            ev_out[h] = Sn;
            n0e[h] = M0;
            n1e[h] = M1;
            if (TALLY) vc_word(cnt, Em0[e], Em1[e], M0, M1);
        }
    }
    __syncthreads();

    // ---- odd half on the owned rows of plane z, with the new even spins
    {
        const int q = (y + z) & 1;
        const int ks = q ? km : kp;
        const uint64_t* Ez = LE + (size_t)PT;  // new even plane z
        const uint64_t S = Od[2];
        const uint64_t nb[6] = {Ez[me], Ez[r * Kx + ks], Ez[rup * Kx + k], Ez[rdn * Kx + k], (Ez + PT)[me],
                                (Ez - PT)[me]};
        const uint64_t a[6] = {xor3(S, nb[0], Oj[0]), xor3(S, nb[1], Oj[1]), xor3(S, nb[2], Oj[2]),
                               xor3(S, nb[3], Oj[3]), xor3(S, nb[4], Oj[4]), xor3(S, nb[5], Oj[5])};
        uint64_t M0 = Om0, M1 = Om1;
        const uint64_t Sn = bp_move(S, a, M0, M1);
        if (own_row) {
            const int64_t h = (int64_t)z * P + yw + k;
            ev_out[Nh + h] = Sn;
            n0e[Nh + h] = M0;
            n1e[Nh + h] = M1;
            if (TALLY) vc_word(cnt, Om0, Om1, M0, M1);
        }
    }

    if (TALLY) {
        const long long sum = bp_tally_counts(cnt, lds_bp);
        if (threadIdx.x < 64) {
            // every lane counted m + (3 - m') over the 2 own Kx words the group owns
            const long long dE = 4 * (sum - 3ll * 2 * own * Kx);
            int s, rr;
            if (dE != 0 && bp_lattice(gb, wl, (int)threadIdx.x, s, rr))
                atomicAdd(&tally[((int64_t)s * g.R + rr) * kSlots + (t % kSlots)], (unsigned long long)dE);
        }
    }
}

}  // namespace micsa
