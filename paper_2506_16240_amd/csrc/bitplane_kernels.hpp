// Bit-plane (multispin-coded) layout: 64 lattices per 64-bit word (Sec. 2.5
// and App. B pack 64 spins per word; here the 64 bits of a word are the same
// site of 64 different lattices).  Two lane modes (enum micsa_lane_mode):
//   samples:  word lattice wl = G r-major: wl = group * R + r; lane l is
//             sample 64 group + l, replica r; the coupling words of a group
//             (coupling set = group) serve all its replicas;
//   replicas: wl = s * G + group; lane l is replica 64 group + l of sample s;
//             the couplings of sample s (coupling set = s) are broadcast to
//             every lane (each coupling word is 0 or ~0).
//
//   spin [WL][p][h]     uint64   bit l = spin bit of the lane's lattice
//   dm0, dm1 [WL][p][h]          bits 0 and 1 of the daemon level m
//   Jw [NJ][d][h]       uint64   coupling bit of bond d of even site h
//
// with the same parity split h as the byte layout (geometry.hpp): site
// words of one row are contiguous, so the x neighbours of site k are words
// k and k +- 1 of the other parity in the same row.
//
// The Creutz move is evaluated for all 64 lanes with Boolean operations
// only (Sec. 2.5): the six unsatisfied-bond bits are added by a bit-sliced
// adder into u = (u2 u1 u0), the two-bit daemon added to it, the legality
// window 3 <= m + u <= 6 tested and the new level m + u - 3 formed, each as
// a handful of 64-bit logic operations.
#pragma once
#include <type_traits>
#include <utility>
#include "geometry.hpp"
#include "philox.hpp"

namespace micsa {

struct GeomB {
    Geom g;
    int32_t G;     // lane groups: ceil(S / 64) (samples mode) or ceil(R / 64) per sample (replicas mode)
    int32_t mode;  // 0: lanes are samples, 1: lanes are the replicas of one sample
};

__host__ __device__ __forceinline__ int bp_word_lattices(const GeomB& b) { return b.mode ? b.g.S * b.G : b.G * b.g.R; }
__host__ __device__ __forceinline__ int bp_coupling_sets(const GeomB& b) { return b.mode ? b.g.S : b.G; }
// coupling set of word lattice wl
__host__ __device__ __forceinline__ int bp_cset(const GeomB& b, int wl) { return b.mode ? wl / b.G : wl / b.g.R; }

// Lattice (s, r) of lane l of word lattice wl; false for a lane beyond the counts.
__host__ __device__ __forceinline__ bool bp_lattice(const GeomB& b, int wl, int l, int& s, int& r)
{
    if (b.mode) {
        s = wl / b.G;
        r = 64 * (wl - s * b.G) + l;
    } else {
        const int grp = wl / b.g.R;
        s = 64 * grp + l;
        r = wl - grp * b.g.R;
    }
    return s < b.g.S && r < b.g.R;
}

// Word lattice and lane of lattice (s, r).
__host__ __device__ __forceinline__ int bp_word_of(const GeomB& b, int s, int r, int& lane)
{
    if (b.mode) {
        lane = r & 63;
        return s * b.G + (r >> 6);
    }
    lane = s & 63;
    return (s >> 6) * b.g.R + r;
}

// Full adder on 64 lanes.
__device__ __forceinline__ void fadd(uint64_t a, uint64_t b, uint64_t c, uint64_t& s, uint64_t& carry)
{
    const uint64_t t = a ^ b;
    s = t ^ c;
    carry = (a & b) | (c & t);
}

// MicSA move on 64 lanes: a[0..5] are the unsatisfied-bond bits.
__device__ __forceinline__ void creutz64(const uint64_t a[6], uint64_t& S, uint64_t& M0, uint64_t& M1)
{
    uint64_t s1, c1, s2, c2;
    fadd(a[0], a[1], a[2], s1, c1);
    fadd(a[3], a[4], a[5], s2, c2);
    const uint64_t u0 = s1 ^ s2;
    const uint64_t c3 = s1 & s2;
    uint64_t u1, u2;
    fadd(c1, c2, c3, u1, u2);
    // w = m + u (4 bits)
    const uint64_t w0 = M0 ^ u0;
    const uint64_t k0 = M0 & u0;
    uint64_t w1, k1;
    fadd(M1, u1, k0, w1, k1);
    const uint64_t w2 = u2 ^ k1;
    const uint64_t w3 = u2 & k1;
    // legal iff w in {3,4,5,6} = {0011, 0100, 0101, 0110}
    const uint64_t acc = ~w3 & (w2 ^ (w1 & w0));
    // new level w - 3 = (w + 1) mod 4 on the legal window
    S ^= acc;
    M0 = (M0 & ~acc) | (~w0 & acc);
    M1 = (M1 & ~acc) | ((w1 ^ w0) & acc);
}

// ---------------------------------------------------------------- init
// One wave per (lane group, site group): lane l draws for sample 64G + l and
// __ballot assembles the 64-lane words.
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Thread = (even site h, lane); block of 256 = 4 even sites x 64 lanes.
// Grid y: coupling sets; lane l draws for sample 64 set + l (samples mode)
// or every lane for sample `set` (replicas mode: broadcast words).
__global__ void __launch_bounds__(256) kb_init_couplings(GeomB b, uint64_t* __restrict__ Jw)
{
    const Geom& g = b.g;
    const int G = blockIdx.y;
    const int64_t h = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = lane_id();
    const uint32_t s = (uint32_t)(b.mode ? G : 64 * G + lane);
    const bool live = h < g.Nh;
    uint32_t bits[6] = {0, 0, 0, 0, 0, 0};
    if (live && s < (uint32_t)g.S) {
        const int k = (int)(h % g.Kx);
        const int row = (int)(h / g.Kx);
        const int y = row % g.Ly, z = row / g.Ly;
        const int x = 2 * k + ((y + z) & 1);
        const uint32_t sw = stream_word(kStreamCoupling, s);
        auto fwd = [&](int xx, int yy, int zz) {
            xx = (xx + g.Lx) % g.Lx;
            yy = (yy + g.Ly) % g.Ly;
            zz = (zz + g.Lz) % g.Lz;
            const uint32_t i = (uint32_t)(xx + (int64_t)g.Lx * (yy + (int64_t)g.Ly * zz));
            return philox10(i, 0u, 0u, sw, g.key0, g.key1);
        };
        const u32x4 o = fwd(x, y, z);
        bits[0] = o.v0 >> 31;
        bits[1] = fwd(x - 1, y, z).v0 >> 31;
        bits[2] = o.v1 >> 31;
        bits[3] = fwd(x, y - 1, z).v1 >> 31;
        bits[4] = o.v2 >> 31;
        bits[5] = fwd(x, y, z - 1).v2 >> 31;
    }
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        const uint64_t w = __ballot(bits[d] != 0);
        if (live && lane == 0) Jw[((int64_t)G * 6 + d) * g.Nh + h] = w;
    }
}

// Thread = (4 consecutive natural sites, lane), one Philox call per thread;
// the 4 sites are 2 even and 2 odd (Lx % 4 == 0), stored at h = i0/2, i0/2+1.
template <typename F>
__device__ __forceinline__ void ballot4(const Geom& g, int64_t i0, const u32x4& o, F&& planes_of,
                                        uint64_t* __restrict__ arr0, uint64_t* __restrict__ arr1, bool live)
{
    const int x0 = (int)(i0 % g.Lx);
    const int64_t row = i0 / g.Lx;
    const int y = (int)(row % g.Ly), z = (int)(row / g.Ly);
    const uint32_t d[4] = {o.v0, o.v1, o.v2, o.v3};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        uint32_t b0, b1;
        planes_of(d[t], b0, b1);
        const uint64_t w0 = __ballot(b0 != 0);
        const uint64_t w1 = __ballot(b1 != 0);
        if (live && lane_id() == 0) {
            const int p = (x0 + t + y + z) & 1;
            const int64_t h = (i0 + t) >> 1;
            arr0[p * g.Nh + h] = w0;
            if (arr1) arr1[p * g.Nh + h] = w1;
        }
    }
}

__global__ void __launch_bounds__(256) kb_init_spins(GeomB b, uint64_t* __restrict__ spin)
{
    const Geom& g = b.g;
    const int wl = blockIdx.y;  // word lattice
    const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const bool live = t < g.Nh / 2;
    int si, r;
    const bool lane_ok = bp_lattice(b, wl, lane_id(), si, r);
    const uint32_t s = (uint32_t)si;
    u32x4 o = {0, 0, 0, 0};
    const int64_t i0 = 4 * t;
    if (live && lane_ok)
        o = philox10((uint32_t)t, 0u, (uint32_t)r, stream_word(kStreamSpin, s), g.key0, g.key1);
    ballot4(g, live ? i0 : 0, o, [](uint32_t u, uint32_t& b0, uint32_t& b1) { b0 = u >> 31; b1 = 0; },
            spin + (int64_t)wl * 2 * g.Nh, nullptr, live);
}

// Refresh draws: a wave draws kRefreshCounters consecutive Philox counters
// (4 sites each) for its 64 lattices, one per lane; the levels of site j of
// the wave's run are gathered into lane j by ballots, so each lane stores
// the two level-plane words of one site (consecutive sites, coalesced).
constexpr int kRefreshCounters = 16;

// v with lane J replaced by the wave-uniform value w (v_writelane_b32, lane
// select an inline constant).
template <int J>
__device__ __forceinline__ uint64_t put_lane(uint64_t v, uint64_t w)
{
    static_assert(J >= 0 && J < 64, "lane");
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    asm volatile("v_writelane_b32 %0, %1, %2" : "+v"(lo) : "s"((uint32_t)w), "i"(J));
    asm volatile("v_writelane_b32 %0, %1, %2" : "+v"(hi) : "s"((uint32_t)(w >> 32)), "i"(J));
    return ((uint64_t)hi << 32) | lo;
}
constexpr int kRefreshSites = 4 * kRefreshCounters;  // one per lane
static_assert(kRefreshSites == 64, "one site per lane");

// f(integral_constant<int, C>) for C = C0 .. kRefreshCounters - 1, unrolled.
template <int C, class F>
__device__ __forceinline__ void for_counters(F& f)
{
    if constexpr (C < kRefreshCounters) {
        f(std::integral_constant<int, C>{});
        for_counters<C + 1>(f);
    }
}

__device__ __forceinline__ void bp_draw_levels(const GeomB& b, int wl, uint32_t rho, const DaemonThresholds& th,
                                               uint64_t* __restrict__ dm0, uint64_t* __restrict__ dm1)
{
    const Geom& g = b.g;
    // first counter of this wave (wave-uniform)
    const int64_t tb = ((int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) *
                       kRefreshCounters;
    const int64_t nt = g.Nh / 2;  // counters per lattice
    if (tb >= nt) return;         // whole waves only
    int si, r;
    const int lane = lane_id();
    const bool lane_ok = bp_lattice(b, wl, lane, si, r);
    const uint32_t sw = stream_word(kStreamDaemon, (uint32_t)si);
    uint64_t W0 = 0, W1 = 0;  // level planes of site 4 tb + lane
    const uint32_t u0 = (uint32_t)(th.t0 - 1u), u1 = (uint32_t)(th.t1 - 1u), u2 = (uint32_t)(th.t2 - 1u);
    // m = [u >= t0] + [u >= t1] + [u >= t2] with t0 <= t1 <= t2, so the high
    // bit of m is [u >= t1] and the low bit the XOR of the three
    auto site = [&](uint32_t u, auto J) {
        const uint64_t a0 = __ballot(u > u0), a1 = __ballot(u > u1), a2 = __ballot(u > u2);
        W0 = put_lane<decltype(J)::value>(W0, a0 ^ a1 ^ a2);
        W1 = put_lane<decltype(J)::value>(W1, a1);
    };
    auto counter = [&](auto C) {
        constexpr int c = decltype(C)::value;
        const int64_t t = tb + c;
        u32x4 o = {0, 0, 0, 0};  // counters past the lattice: sites that are not stored
        if (lane_ok && t < nt) o = philox10((uint32_t)t, rho, (uint32_t)r, sw, g.key0, g.key1);
        site(o.v0, std::integral_constant<int, 4 * c>{});
        site(o.v1, std::integral_constant<int, 4 * c + 1>{});
        site(o.v2, std::integral_constant<int, 4 * c + 2>{});
        site(o.v3, std::integral_constant<int, 4 * c + 3>{});
    };
    for_counters<0>(counter);
    const int64_t i = 4 * tb + lane;
    if (i < 4 * nt) {
        const int x = (int)(i % g.Lx);
        const int64_t row = i / g.Lx;
        const int y = (int)(row % g.Ly), z = (int)(row / g.Ly);
        const int64_t at = (int64_t)((x + y + z) & 1) * g.Nh + (i >> 1);
        dm0[(int64_t)wl * 2 * g.Nh + at] = W0;
        dm1[(int64_t)wl * 2 * g.Nh + at] = W1;
    }
}

// Work-groups of the refresh draw along x (4 waves of kRefreshCounters counters each).
__host__ __device__ inline unsigned bp_refresh_blocks(const Geom& g)
{
    return (unsigned)((g.Nh / 2 + 4 * kRefreshCounters - 1) / (4 * kRefreshCounters));
}

__global__ void __launch_bounds__(256) kb_refresh(GeomB b, uint64_t* __restrict__ dm0, uint64_t* __restrict__ dm1,
                                                  uint32_t rho, DaemonThresholds th)
{
    bp_draw_levels(b, blockIdx.y, rho, th, dm0, dm1);
}

// kb_refresh with the sweep index in device memory (replayable graphs).
__global__ void __launch_bounds__(256) kb_refresh_dev(GeomB b, uint64_t* __restrict__ dm0, uint64_t* __restrict__ dm1,
                                                      const int64_t* __restrict__ dk, int32_t period,
                                                      const DaemonThresholds* __restrict__ dth)
{
    const int64_t k = *dk;
    if (!(period >= 1 ? (k % period == 0) : (((k + 1) & k) == 0))) return;
    const int64_t rho = period >= 1 ? k / period : 63 - __clzll((unsigned long long)(k + 1));
    bp_draw_levels(b, blockIdx.y, (uint32_t)rho, dth[rho], dm0, dm1);
}

// ------------------------------------------------------------- half sweep
// Thread per site word (64 lanes) of parity P.
template <int P>
__global__ void __launch_bounds__(256) kb_micsa_half(GeomB b, uint64_t* __restrict__ spin,
                                                     uint64_t* __restrict__ dm0, uint64_t* __restrict__ dm1,
                                                     const uint64_t* __restrict__ Jw)
{
    const Geom& g = b.g;
    const int wl = blockIdx.y;
    const int G = bp_cset(b, wl);
    const uint32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= (uint32_t)g.Nh) return;
    const int row = (int)(h / (uint32_t)g.Kx), k = (int)(h - (uint32_t)row * (uint32_t)g.Kx);
    const int z = row / g.Ly, y = row - z * g.Ly;
    const int q = (y + z) & 1;
    const int dir = (q ^ P) ? 1 : -1;
    const int ks = dir > 0 ? (k + 1 == g.Kx ? 0 : k + 1) : (k == 0 ? g.Kx - 1 : k - 1);
    const int yp = y + 1 == g.Ly ? 0 : y + 1, ym = y == 0 ? g.Ly - 1 : y - 1;
    const int zp = z + 1 == g.Lz ? 0 : z + 1, zm = z == 0 ? g.Lz - 1 : z - 1;
    const int64_t K = g.Kx;
    const int64_t hA = h, hB = (int64_t)row * K + ks, hYp = (int64_t)(yp + g.Ly * z) * K + k,
                  hYm = (int64_t)(ym + g.Ly * z) * K + k, hZp = (int64_t)(y + g.Ly * zp) * K + k,
                  hZm = (int64_t)(y + g.Ly * zm) * K + k;
    const int64_t base = (int64_t)wl * 2 * g.Nh;
    const uint64_t* oth = spin + base + (1 - P) * g.Nh;
    const uint64_t* Jg = Jw + (int64_t)G * 6 * g.Nh;
    const int dA = q ? kMx : kPx, dB = q ? kPx : kMx;
    uint64_t j[6];
    if (P == 0) {
        j[0] = Jg[dA * g.Nh + hA];
        j[1] = Jg[dB * g.Nh + hA];
        j[2] = Jg[kPy * g.Nh + hA];
        j[3] = Jg[kMy * g.Nh + hA];
        j[4] = Jg[kPz * g.Nh + hA];
        j[5] = Jg[kMz * g.Nh + hA];
    } else {
        j[0] = Jg[dA * g.Nh + hA];
        j[1] = Jg[dB * g.Nh + hB];
        j[2] = Jg[kMy * g.Nh + hYp];
        j[3] = Jg[kPy * g.Nh + hYm];
        j[4] = Jg[kMz * g.Nh + hZp];
        j[5] = Jg[kPz * g.Nh + hZm];
    }
    const int64_t own = base + P * g.Nh + h;
    uint64_t S = spin[own], M0 = dm0[own], M1 = dm1[own];
    const uint64_t a[6] = {S ^ oth[hA] ^ j[0], S ^ oth[hB] ^ j[1], S ^ oth[hYp] ^ j[2],
                           S ^ oth[hYm] ^ j[3], S ^ oth[hZp] ^ j[4], S ^ oth[hZm] ^ j[5]};
    creutz64(a, S, M0, M1);
    spin[own] = S;
    dm0[own] = M0;
    dm1[own] = M1;
}

// ------------------------------------------------------------ reductions
// Per-lane counts: one wave per block; lane l owns the lattice of its bit
// and counts its bit of every word the wave reads (the same word for all
// lanes).  kind 0: unsatisfied bonds U (H = 2U - 3N); 1: daemon levels sum
// m; 2: sites where replicas a and b differ (samples mode: grid y over the
// lane groups, lane l = sample; replicas mode: grid y over the samples, the
// lanes splitting the words and the wave summing one count per sample).
template <int KIND>
__global__ void __launch_bounds__(64) kb_lane_count(GeomB b, const uint64_t* __restrict__ spin,
                                                   const uint64_t* __restrict__ dm0,
                                                   const uint64_t* __restrict__ dm1,
                                                   const uint64_t* __restrict__ Jw, int ra, int rb,
                                                   int64_t sites_per_block, unsigned long long* __restrict__ out)
{
    const Geom& g = b.g;
    const int wl = blockIdx.y;  // KIND 2: lane group (samples) or sample (replicas); otherwise word lattice
    const int G = KIND == 2 ? wl : bp_cset(b, wl);
    const int lane = lane_id();
    const int64_t h0 = (int64_t)blockIdx.x * sites_per_block;
    const int64_t h1 = h0 + sites_per_block < g.Nh ? h0 + sites_per_block : g.Nh;
    long long cnt = 0;
    if (KIND == 2 && b.mode) {
        int la, lb;
        const uint64_t* sa = spin + (int64_t)bp_word_of(b, wl, ra, la) * 2 * g.Nh;
        const uint64_t* sb = spin + (int64_t)bp_word_of(b, wl, rb, lb) * 2 * g.Nh;
        for (int64_t h = h0 + lane; h < h1; h += 64)
            for (int p = 0; p < 2; ++p)
                cnt += (long long)(((sa[p * g.Nh + h] >> la) ^ (sb[p * g.Nh + h] >> lb)) & 1u);
        cnt = wave_sum64(cnt);
        if (lane == 0 && cnt != 0) atomicAdd(&out[(int64_t)wl * kSlots + (blockIdx.x % kSlots)], (unsigned long long)cnt);
        return;
    }
    if (KIND == 0) {
        const uint64_t* ev = spin + (int64_t)wl * 2 * g.Nh;
        const uint64_t* od = ev + g.Nh;
        const uint64_t* Jg = Jw + (int64_t)G * 6 * g.Nh;
        for (int64_t h = h0; h < h1; ++h) {
            const int row = (int)(h / g.Kx), k = (int)(h - (int64_t)row * g.Kx);
            const int z = row / g.Ly, y = row - z * g.Ly;
            const int q = (y + z) & 1;
            const int ks = q ? (k + 1 == g.Kx ? 0 : k + 1) : (k == 0 ? g.Kx - 1 : k - 1);
            const int yp = y + 1 == g.Ly ? 0 : y + 1, ym = y == 0 ? g.Ly - 1 : y - 1;
            const int zp = z + 1 == g.Lz ? 0 : z + 1, zm = z == 0 ? g.Lz - 1 : z - 1;
            const int64_t K = g.Kx;
            const uint64_t S = ev[h];
            const int dA = q ? kMx : kPx, dB = q ? kPx : kMx;
            const uint64_t w[6] = {S ^ od[h] ^ Jg[dA * g.Nh + h], S ^ od[(int64_t)row * K + ks] ^ Jg[dB * g.Nh + h],
                                   S ^ od[(int64_t)(yp + g.Ly * z) * K + k] ^ Jg[kPy * g.Nh + h],
                                   S ^ od[(int64_t)(ym + g.Ly * z) * K + k] ^ Jg[kMy * g.Nh + h],
                                   S ^ od[(int64_t)(y + g.Ly * zp) * K + k] ^ Jg[kPz * g.Nh + h],
                                   S ^ od[(int64_t)(y + g.Ly * zm) * K + k] ^ Jg[kMz * g.Nh + h]};
#pragma unroll
            for (int d = 0; d < 6; ++d) cnt += (long long)((w[d] >> lane) & 1u);
        }
    } else if (KIND == 1) {
        const uint64_t* m0 = dm0 + (int64_t)wl * 2 * g.Nh;
        const uint64_t* m1 = dm1 + (int64_t)wl * 2 * g.Nh;
        for (int64_t h = h0; h < h1; ++h)
            for (int p = 0; p < 2; ++p)
                cnt += (long long)((m0[p * g.Nh + h] >> lane) & 1u) + 2 * (long long)((m1[p * g.Nh + h] >> lane) & 1u);
    } else {
        const uint64_t* sa = spin + ((int64_t)G * g.R + ra) * 2 * g.Nh;
        const uint64_t* sb = spin + ((int64_t)G * g.R + rb) * 2 * g.Nh;
        for (int64_t h = h0; h < h1; ++h)
            for (int p = 0; p < 2; ++p) cnt += (long long)(((sa[p * g.Nh + h] ^ sb[p * g.Nh + h]) >> lane) & 1u);
    }
    int s, r;
    const bool ok = KIND == 2 ? ((s = 64 * G + lane) < g.S) : bp_lattice(b, wl, lane, s, r);
    if (ok && cnt != 0) {
        const int64_t ent = KIND == 2 ? s : (int64_t)s * g.R + r;
        atomicAdd(&out[ent * kSlots + (blockIdx.x % kSlots)], (unsigned long long)cnt);
    }
}

}  // namespace micsa
