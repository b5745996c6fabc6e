// Kernels of the equilibrium workload of App. C: one Gaussian sample, runs x
// 2 replicas x M temperatures, continuous walkers (gamma = 1) refreshed every
// EMCS, Houdayer cluster moves between the replicas and parallel tempering.
//
// Energy mesh: couplings, energies and walkers are integers in units of
// 2^-17 (the paper allows walkers on a fine energy mesh, Sec. 2.3), so the
// Creutz move is exact integer arithmetic.
//
// Exponential on the mesh: P(n) = (1 - q) q^n, q = exp(-lambda 2^-17), drawn
// as four independent base-256 digits, digit d by inverse CDF on word d of
// one Philox output: c_d = #{v : w_d >= t_d[v]} with the table t_d[0..254]
// computed on the host.  Every t_d[v] lies in [2^24, 2^32] (the most likely
// value of a digit has probability >= 1/256), so the device holds
// t_d[v] - 1 in 32 bits (w >= t <=> w > t - 1), plus an indexed-search guide
// (Chen and Asau, 1974): for each top byte b of w the range [lo, hi] of
// counts the words of that bucket can have, so a draw costs one guide read
// and, in most buckets, no or one threshold compare.  The walkers use
// lambda = beta_t; the Metropolis update (a fresh walker per attempt,
// Sec. 2.3) and the tempering swaps (lambda = beta_t - beta_{t+1}) only
// need "n >= k", which is decided digit by digit from the top with at most
// two table reads per digit.
//
// Layout in HBM (per run u, replica a, slot c of the replica group):
//   rows[u][a][c][r]   one 64-bit word per lattice row r = y + Ly z: bit x
//                      is the spin bit sigma of site x + Lx r (Lx <= 64)
//   perm[u][a][t]      slot holding the configuration at temperature t
//   E[u][a][c]         energy of slot c (units of 2^-17), refreshed every EMCS
//   rec[x * R0 + r]    per-site coupling record (x-major so that the threads
//                      of consecutive rows read consecutive records):
//                      J+x, J+y, J+z, J-x, J-y, J-z, their sum, 0
// Tempering exchanges slots in perm; configurations never move.
//
// Work split of k_pt_emcs: one work-group per (temperature, run) holds both
// replicas of that temperature (Houdayer needs the pair); thread rr owns
// lattice row rr % R0 of replica rr / R0, so the x-neighbours of a site are
// bits of the thread's own word and the y/z-neighbours are the same bit of
// four other row words.  Forward-X wandering moves walkers within a row
// only, so every walker stays with the thread that owns its row.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "philox.hpp"

namespace micsa {

constexpr int kPtBlock = 256;
// u32 words per exponential table: [d * 256 + v] = t_d[v] - 1 (v < 255),
// then 4 x 256 guides as u16 lo | hi << 8 at byte offset 4096 + 2 (d * 256 + b)
constexpr int kPtTable = 1536;
enum : uint32_t { kStreamPtWalker = 6u, kStreamPtMetropolis = 7u, kStreamPtHoudayer = 8u, kStreamPtSwap = 9u,
                  kStreamPtSpin = 10u };

struct PtGeom {
    int32_t Lx, Ly, Lz;
    int32_t R0;  // rows per lattice
    int32_t N;
    int32_t M;     // temperatures
    int32_t runs;
    int32_t S;     // sweeps per EMCS
    uint32_t key0, key1;
    uint64_t xmask;  // the low Lx bits
};

__device__ __forceinline__ int32_t bit_mask(uint64_t w, int x) { return -(int32_t)((w >> x) & 1u); }

__device__ __forceinline__ uint64_t rot_up(uint64_t m, const PtGeom& g)  // bit x <- bit x - 1
{
    return ((m << 1) | (m >> (g.Lx - 1))) & g.xmask;
}
__device__ __forceinline__ uint64_t rot_down(uint64_t m, const PtGeom& g)  // bit x <- bit x + 1
{
    return ((m >> 1) | (m << (g.Lx - 1))) & g.xmask;
}

// Digit d of a draw: the number of thresholds <= w, found between the
// guide's bounds for the bucket of w by bisection.
__device__ __forceinline__ int32_t digit_draw(const uint32_t* tab, int d, uint32_t w)
{
    const uint32_t gb = ((const uint16_t*)(tab + 1024))[d * 256 + (w >> 24)];
    int32_t lo = (int32_t)(gb & 255u), hi = (int32_t)(gb >> 8);
    const uint32_t* t = tab + d * 256;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (w > t[mid])
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int32_t exp_draw4(const uint32_t* tab, const u32x4& w)
{
    return digit_draw(tab, 0, w.v0) + (digit_draw(tab, 1, w.v1) << 8) + (digit_draw(tab, 2, w.v2) << 16) +
           (digit_draw(tab, 3, w.v3) << 24);
}

// n >= k for the mesh exponential n drawn from words w.  Digit d of n
// exceeds k_d iff w_d >= t_d[k_d] (k_d <= 254) and falls below k_d iff
// w_d < t_d[k_d - 1] (k_d >= 1); equal digits pass to the next one.
__device__ __forceinline__ bool exp_at_least(const uint32_t* tab, const u32x4& w, int64_t k)
{
    if (k <= 0) return true;
    if (k >= (int64_t)1 << 32) return false;
    const uint32_t ws[4] = {w.v0, w.v1, w.v2, w.v3};
#pragma unroll
    for (int d = 3; d >= 0; --d) {
        const int32_t kd = (int32_t)((k >> (8 * d)) & 255);
        const uint32_t* td = tab + d * 256;
        if (kd <= 254 && ws[d] > td[kd]) return true;
        if (kd >= 1 && ws[d] <= td[kd - 1]) return false;
    }
    return true;
}

// Energy of one row's forward bonds: -sum J s_x s_y = sum J (2 d - 1),
// d = sigma_x XOR sigma_y.
template <bool JL>
__device__ __forceinline__ int32_t row_energy(const PtGeom& g, const int4* rec, int r, uint64_t row, uint64_t ryp,
                                              uint64_t rzp)
{
    const uint64_t dx = row ^ rot_down(row, g), dy = row ^ ryp, dz = row ^ rzp;
    int32_t e = 0;
    for (int x = 0; x < g.Lx; ++x) {
        const int4 a = rec[2 * (x * g.R0 + r)];
        e += (2 * (a.x & bit_mask(dx, x)) - a.x) + (2 * (a.y & bit_mask(dy, x)) - a.y) +
             (2 * (a.z & bit_mask(dz, x)) - a.z);
    }
    return e;
}

struct PtRowNb {
    int r, yp, ym, zp, zm;  // row indices of the row and its y/z neighbours
    int y, z;
};

__device__ __forceinline__ PtRowNb pt_row_nb(const PtGeom& g, int r)
{
    PtRowNb n;
    n.r = r;
    n.y = r % g.Ly;
    n.z = r / g.Ly;
    const int yp = n.y + 1 == g.Ly ? 0 : n.y + 1, ym = n.y == 0 ? g.Ly - 1 : n.y - 1;
    const int zp = n.z + 1 == g.Lz ? 0 : n.z + 1, zm = n.z == 0 ? g.Lz - 1 : n.z - 1;
    n.yp = yp + g.Ly * n.z;
    n.ym = ym + g.Ly * n.z;
    n.zp = n.y + g.Ly * zp;
    n.zm = n.y + g.Ly * zm;
    return n;
}

// LDS carve-up of k_pt_emcs (bytes): tables, coupling records (JL), spin
// rows of both replicas, walkers (ALGO 0), Houdayer rows and scan scratch.
struct PtLds {
    uint32_t tab, rec, rows, walk, mark, diff, scan, misc, total;
};

__host__ __device__ inline PtLds pt_lds_layout(const PtGeom& g, bool jl, bool walkers)
{
    PtLds l;
    uint32_t o = 0;
    l.tab = o;
    o += kPtTable * 4;
    l.rec = o;
    o += jl ? (uint32_t)g.N * 32u : 0u;
    l.rows = o;
    o += (uint32_t)g.R0 * 16u;
    l.walk = o;
    o += walkers ? (uint32_t)g.N * 8u : 0u;
    l.mark = o;
    o += (uint32_t)g.R0 * 8u;
    l.diff = o;
    o += (uint32_t)g.R0 * 8u;
    l.scan = o;
    o += kPtBlock * 4u;
    l.misc = o;
    o += 64u;
    l.total = o;
    return l;
}

// One EMCS of the fixed-temperature moves (walkers: ALGO 0; Metropolis:
// ALGO 1), then the Houdayer move (HOUD) and both replicas' energies.
// Grid (M, runs); block kPtBlock; dynamic LDS pt_lds_layout(g, JL, ALGO == 0).
template <int ALGO, bool HOUD, bool JL>
__global__ __launch_bounds__(kPtBlock) void k_pt_emcs(PtGeom g, const int4* __restrict__ grec,
                                                        uint64_t* __restrict__ spins,
                                                        const int32_t* __restrict__ perm, int64_t* __restrict__ E,
                                                        const uint32_t* __restrict__ wtab, uint32_t e)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const PtLds L = pt_lds_layout(g, JL, ALGO == 0);
    uint32_t* tab = (uint32_t*)(lds + L.tab);
    const int4* rec = JL ? (const int4*)(lds + L.rec) : grec;
    uint64_t* rows = (uint64_t*)(lds + L.rows);  // [2][R0]
    int32_t* walk = (int32_t*)(lds + L.walk);    // [2][Lx][R0]
    uint64_t* mark = (uint64_t*)(lds + L.mark);
    uint64_t* diff = (uint64_t*)(lds + L.diff);
    int32_t* scan = (int32_t*)(lds + L.scan);
    int32_t* misc = (int32_t*)(lds + L.misc);
    unsigned long long* esum = (unsigned long long*)(lds + L.misc + 16);

    const int t = blockIdx.x, run = blockIdx.y, tid = threadIdx.x;
    const int R0 = g.R0, nrow = 2 * R0;
    const int32_t slot0 = perm[((int64_t)run * 2 + 0) * g.M + t];
    const int32_t slot1 = perm[((int64_t)run * 2 + 1) * g.M + t];
    uint64_t* g0 = spins + (((int64_t)run * 2 + 0) * g.M + slot0) * R0;
    uint64_t* g1 = spins + (((int64_t)run * 2 + 1) * g.M + slot1) * R0;
    const uint32_t sw = (uint32_t)run;

    for (int k = tid; k < kPtTable; k += kPtBlock) tab[k] = wtab[(int64_t)t * kPtTable + k];
    if (JL)
        for (int k = tid; k < 2 * g.N; k += kPtBlock) ((int4*)(lds + L.rec))[k] = grec[k];
    for (int k = tid; k < R0; k += kPtBlock) {
        rows[k] = g0[k];
        rows[R0 + k] = g1[k];
    }
    if (tid < 2) esum[tid] = 0ull;
    __syncthreads();

    if (ALGO == 0) {  // walkers drawn at beta_t (one Philox output per site)
        for (int rr = tid; rr < nrow; rr += kPtBlock) {
            const int rep = rr >= R0, r = rr - rep * R0;
            for (int x = 0; x < g.Lx; ++x) {
                const uint32_t i = (uint32_t)(x + g.Lx * r);
                const u32x4 w = philox10(i, e, (uint32_t)(2 * t + rep), stream_word(kStreamPtWalker, sw), g.key0,
                                         g.key1);
                walk[(rep * g.Lx + x) * R0 + r] = exp_draw4(tab, w);
            }
        }
    }

    for (int s = 0; s < g.S; ++s) {
        for (int p = 0; p < 2; ++p) {
            for (int rr = tid; rr < nrow; rr += kPtBlock) {
                const int rep = rr >= R0, r = rr - rep * R0;
                const PtRowNb nb = pt_row_nb(g, r);
                const uint64_t* rw = rows + rep * R0;
                const uint64_t row = rw[r];
                const uint64_t xp = rot_down(row, g), xm = rot_up(row, g);
                const uint64_t yp = rw[nb.yp], ym = rw[nb.ym], zp = rw[nb.zp], zm = rw[nb.zm];
                uint64_t flips = 0;
                for (int x = (p + nb.y + nb.z) & 1; x < g.Lx; x += 2) {
                    const int4 a = rec[2 * (x * R0 + r)], b = rec[2 * (x * R0 + r) + 1];
                    // h = sum J s = Jsum - 2 sum over neighbours with sigma = 1
                    const int32_t up = (a.x & bit_mask(xp, x)) + (a.y & bit_mask(yp, x)) + (a.z & bit_mask(zp, x)) +
                                       (a.w & bit_mask(xm, x)) + (b.x & bit_mask(ym, x)) + (b.y & bit_mask(zm, x));
                    const int32_t h2 = 2 * (b.z - 2 * up);  // 2 h
                    const int32_t own = bit_mask(row, x);
                    const int32_t dH = (h2 ^ own) - own;    // 2 s h, s = -1 when sigma = 1
                    bool acc;
                    if (ALGO == 0) {
                        int32_t* wp = walk + (rep * g.Lx + x) * R0 + r;
                        const int32_t n = *wp;
                        acc = n - dH >= 0;
                        if (acc) *wp = n - dH;
                    } else {
                        const uint32_t i = (uint32_t)(x + g.Lx * r);
                        const u32x4 w = philox10(i, e * (uint32_t)g.S + (uint32_t)s, (uint32_t)(2 * t + rep),
                                                 stream_word(kStreamPtMetropolis, sw), g.key0, g.key1);
                        acc = exp_at_least(tab, w, dH);
                    }
                    flips |= (uint64_t)acc << x;
                }
                rows[rep * R0 + r] = row ^ flips;
            }
            __syncthreads();
        }
        if (ALGO == 0) {  // forward-X wandering of the sites of parity s & 1 (row-local)
            for (int rr = tid; rr < nrow; rr += kPtBlock) {
                const int rep = rr >= R0, r = rr - rep * R0;
                const int y = r % g.Ly, z = r / g.Ly;
                int32_t* wr = walk + rep * g.Lx * R0 + r;
                for (int x = ((s & 1) + y + z) & 1; x < g.Lx; x += 2) {
                    const int xn = x + 1 == g.Lx ? 0 : x + 1;
                    const int32_t tmp = wr[x * R0];
                    wr[x * R0] = wr[xn * R0];
                    wr[xn * R0] = tmp;
                }
            }
        }
    }

    if (HOUD) {
        // differing sites per row, in site order: prefix over contiguous row chunks
        const int chunk = (R0 + kPtBlock - 1) / kPtBlock;
        int32_t mine = 0;
        for (int r = tid * chunk; r < min(R0, (tid + 1) * chunk); ++r) {
            const uint64_t d = (rows[r] ^ rows[R0 + r]) & g.xmask;
            diff[r] = d;
            mark[r] = 0;
            mine += __popcll(d);
        }
        scan[tid] = mine;
        __syncthreads();
        for (int off = 1; off < kPtBlock; off <<= 1) {  // inclusive scan
            const int32_t v = tid >= off ? scan[tid - off] : 0;
            __syncthreads();
            scan[tid] += v;
            __syncthreads();
        }
        const int32_t count = scan[kPtBlock - 1];
        if (count > 0) {
            const uint32_t u = philox10((uint32_t)t, e, 0u, stream_word(kStreamPtHoudayer, sw), g.key0, g.key1).v0;
            const int32_t k = (int32_t)(((uint64_t)u * (uint64_t)count) >> 32);
            const int32_t before = scan[tid] - mine;
            if (k >= before && k < scan[tid]) {  // the chosen site is in this thread's chunk
                int32_t left = k - before;
                for (int r = tid * chunk; r < min(R0, (tid + 1) * chunk); ++r) {
                    uint64_t d = diff[r];
                    const int32_t c = __popcll(d);
                    if (left < c) {
                        for (; left > 0; --left) d &= d - 1;  // drop the lower set bits
                        mark[r] = d & (~d + 1);
                        break;
                    }
                    left -= c;
                }
            }
            // grow the cluster to the connected component of the chosen site
            for (;;) {
                __syncthreads();
                if (tid == 0) misc[0] = 0;
                __syncthreads();
                for (int r = tid; r < R0; r += kPtBlock) {
                    const PtRowNb nb = pt_row_nb(g, r);
                    const uint64_t d = diff[r], m = mark[r];
                    uint64_t m2 = d & (m | mark[nb.yp] | mark[nb.ym] | mark[nb.zp] | mark[nb.zm]);
                    for (;;) {  // close along the row
                        const uint64_t m3 = d & (m2 | rot_up(m2, g) | rot_down(m2, g));
                        if (m3 == m2) break;
                        m2 = m3;
                    }
                    if (m2 != m) {
                        mark[r] = m2;
                        misc[0] = 1;
                    }
                }
                __syncthreads();
                if (misc[0] == 0) break;
            }
            for (int r = tid; r < R0; r += kPtBlock) {
                rows[r] ^= mark[r];
                rows[R0 + r] ^= mark[r];
            }
            __syncthreads();
        }
    }

    // write back and energies
    for (int rr = tid; rr < nrow; rr += kPtBlock) {
        const int rep = rr >= R0, r = rr - rep * R0;
        const PtRowNb nb = pt_row_nb(g, r);
        const uint64_t* rw = rows + rep * R0;
        const int32_t er = row_energy<JL>(g, rec, r, rw[r], rw[nb.yp], rw[nb.zp]);
        atomicAdd(&esum[rep], (unsigned long long)(int64_t)er);
        (rep ? g1 : g0)[r] = rw[r];
    }
    __syncthreads();
    if (tid == 0) {
        E[((int64_t)run * 2 + 0) * g.M + slot0] = (int64_t)esum[0];
        E[((int64_t)run * 2 + 1) * g.M + slot1] = (int64_t)esum[1];
    }
}

// ---------------------------------------------------------------------------
// Register-resident variant for rows of LX <= 32 sites (LX a compile-time
// constant) and 2 * Ly * Lz <= 1024: a work-group holds G temperatures (both
// replicas each) and every thread owns exactly one row of one replica, so
// the walkers of a row live in VGPRs, split by parity class (wk0: the
// row's even sites x = 2j + ((y+z) & 1), wk1: its odd sites), and every bit
// test uses a constant offset.  Forward-X wandering pairs site j of the
// moving class with site j (or j + 1 when the class starts at x = 1) of the
// other class, all within the row.
// LDS: tables [G][1024] u64 | records [N][2] int4 | rows [G][2][R0] u32 |
//      mark, diff [G][R0] u32 | energies [G][2] u64 | flag.
struct PtRegLds {
    uint32_t tab, rec, rows, mark, diff, esum, flag, total;
};

__host__ __device__ inline PtRegLds pt_reg_layout(const PtGeom& g, int G)
{
    PtRegLds l;
    uint32_t o = 0;
    l.tab = o;
    o += (uint32_t)G * kPtTable * 4u;
    l.rec = o;
    o += (uint32_t)g.N * 32u;
    l.rows = o;
    o += (uint32_t)G * 2u * g.R0 * 4u;
    l.mark = o;
    o += (uint32_t)G * g.R0 * 4u;
    l.diff = o;
    o += (uint32_t)G * g.R0 * 4u;
    o = (o + 7u) & ~7u;
    l.esum = o;
    o += (uint32_t)G * 16u;
    l.flag = o;
    o += 16u;
    l.total = o;
    return l;
}

template <int LX>
__device__ __forceinline__ uint32_t rot_down32(uint32_t m)  // bit x <- bit x + 1
{
    constexpr uint32_t MASK = LX == 32 ? 0xFFFFFFFFu : ((1u << LX) - 1u);
    return ((m >> 1) | (m << (LX - 1))) & MASK;
}
template <int LX>
__device__ __forceinline__ uint32_t rot_up32(uint32_t m)  // bit x <- bit x - 1
{
    constexpr uint32_t MASK = LX == 32 ? 0xFFFFFFFFu : ((1u << LX) - 1u);
    return ((m << 1) | (m >> (LX - 1))) & MASK;
}

__device__ __forceinline__ int32_t sbit(uint32_t w, int pos)  // 0 or -1
{
    return __builtin_amdgcn_sbfe((int32_t)w, pos, 1);
}

template <int LX, int ALGO, int P>
__device__ __forceinline__ void reg_half(const PtGeom& g, const int4* rec, uint32_t* rows, int base, int r,
                                         const PtRowNb& nb, int32_t (&wk)[LX / 2], const uint32_t* tab, uint32_t e,
                                         int s, int t, int rep, uint32_t run)
{
    constexpr int K = LX / 2;
    const int R0 = g.R0;
    const int xs = (P + nb.y + nb.z) & 1;  // first x of this class in the row
    const uint32_t own = rows[base + r];
    const uint32_t wo = own >> xs, wxp = rot_down32<LX>(own) >> xs, wxm = rot_up32<LX>(own) >> xs;
    const uint32_t wyp = rows[base + nb.yp] >> xs, wym = rows[base + nb.ym] >> xs;
    const uint32_t wzp = rows[base + nb.zp] >> xs, wzm = rows[base + nb.zm] >> xs;
    const int4* rc = rec + 2 * (xs * R0 + r);
    uint32_t flips = 0;
    // the walker path unrolls (walkers in registers); the Metropolis path
    // keeps one generator output live at a time
    constexpr int kUnroll = ALGO == 0 ? K : 1;
#pragma unroll kUnroll
    for (int j = 0; j < K; ++j) {
        const int4 a = rc[4 * R0 * j], b = rc[4 * R0 * j + 1];
        const int32_t up = (a.x & sbit(wxp, 2 * j)) + (a.y & sbit(wyp, 2 * j)) + (a.z & sbit(wzp, 2 * j)) +
                           (a.w & sbit(wxm, 2 * j)) + (b.x & sbit(wym, 2 * j)) + (b.y & sbit(wzm, 2 * j));
        const int32_t h2 = 2 * (b.z - 2 * up);
        const int32_t m = sbit(wo, 2 * j);
        const int32_t dH = (h2 ^ m) - m;
        bool acc;
        if (ALGO == 0) {
            const int32_t n = wk[j], nn = n - dH;
            acc = nn >= 0;
            wk[j] = acc ? nn : n;
        } else {
            const uint32_t i = (uint32_t)(2 * j + xs + LX * r);
            const u32x4 w = philox10(i, e * (uint32_t)g.S + (uint32_t)s, (uint32_t)(2 * t + rep),
                                     stream_word(kStreamPtMetropolis, run), g.key0, g.key1);
            acc = exp_at_least(tab, w, dH);
        }
        flips |= acc ? (1u << (2 * j)) : 0u;
    }
    rows[base + r] = own ^ (flips << xs);
}

// Forward-X wandering of the sites of class PW: site j of class PW at
// x = 2j + xs swaps with site j + xs of the other class (periodic).
template <int K>
__device__ __forceinline__ void reg_wander(int32_t (&A)[K], int32_t (&B)[K], int xs)
{
    int32_t nA[K], nB[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        nA[j] = xs ? B[(j + 1) % K] : B[j];
        nB[j] = xs ? A[(j + K - 1) % K] : A[j];
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        A[j] = nA[j];
        B[j] = nB[j];
    }
}

// Grid (ceil(M / G), runs); block 64 * ceil(2 G R0 / 64) <= 1024 threads;
// dynamic LDS pt_reg_layout(g, G).
template <int LX, int ALGO, bool HOUD>
__global__ __launch_bounds__(1024) void k_pt_emcs_reg(PtGeom g, int G, const int4* __restrict__ grec,
                                                      uint64_t* __restrict__ spins, const int32_t* __restrict__ perm,
                                                      int64_t* __restrict__ E, const uint32_t* __restrict__ wtab,
                                                      uint32_t e)
{
    constexpr int K = LX / 2;
    constexpr uint32_t MASK = LX == 32 ? 0xFFFFFFFFu : ((1u << LX) - 1u);
    extern __shared__ __align__(16) unsigned char lds[];
    const PtRegLds L = pt_reg_layout(g, G);
    uint32_t* tabs = (uint32_t*)(lds + L.tab);
    int4* rec = (int4*)(lds + L.rec);
    uint32_t* rows = (uint32_t*)(lds + L.rows);
    uint32_t* mark = (uint32_t*)(lds + L.mark);
    uint32_t* diff = (uint32_t*)(lds + L.diff);
    unsigned long long* esum = (unsigned long long*)(lds + L.esum);
    int32_t* flag = (int32_t*)(lds + L.flag);

    const int R0 = g.R0, tid = threadIdx.x, nthr = blockDim.x;
    const int tl = tid / (2 * R0), rem = tid - tl * 2 * R0;
    const int rep = rem >= R0, r = rem - rep * R0;
    const int t0 = blockIdx.x * G, t = t0 + tl;
    const int run = blockIdx.y;
    const uint32_t sw = (uint32_t)run;
    const bool live = tl < G && t < g.M;
    const int base = (tl * 2 + rep) * R0;

    for (int k = tid; k < G * kPtTable; k += nthr) {
        const int tg = t0 + k / kPtTable;
        tabs[k] = tg < g.M ? wtab[(int64_t)tg * kPtTable + k % kPtTable] : 0u;
    }
    for (int k = tid; k < 2 * g.N; k += nthr) rec[k] = grec[k];
    int32_t slot = 0;
    uint64_t* grow = nullptr;
    if (live) {
        slot = perm[((int64_t)run * 2 + rep) * g.M + t];
        grow = spins + (((int64_t)run * 2 + rep) * g.M + slot) * R0 + r;
        rows[base + r] = (uint32_t)*grow;
    }
    if (tid < 2 * G) esum[tid] = 0ull;
    __syncthreads();

    const PtRowNb nb = pt_row_nb(g, live ? r : 0);
    const uint32_t* tab = tabs + (live ? tl : 0) * kPtTable;
    int32_t wk0[K], wk1[K];
#pragma unroll
    for (int j = 0; j < K; ++j) wk0[j] = wk1[j] = 0;
    if (ALGO == 0 && live) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int xs = (c + nb.y + nb.z) & 1;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const uint32_t i = (uint32_t)(2 * j + xs + LX * r);
                const u32x4 w = philox10(i, e, (uint32_t)(2 * t + rep), stream_word(kStreamPtWalker, sw), g.key0,
                                         g.key1);
                (c == 0 ? wk0 : wk1)[j] = exp_draw4(tab, w);
            }
        }
    }

    for (int s = 0; s < g.S; ++s) {
        if (live) reg_half<LX, ALGO, 0>(g, rec, rows, base, r, nb, wk0, tab, e, s, t, rep, sw);
        __syncthreads();
        if (live) reg_half<LX, ALGO, 1>(g, rec, rows, base, r, nb, wk1, tab, e, s, t, rep, sw);
        __syncthreads();
        if (ALGO == 0) {
            if ((s & 1) == 0)
                reg_wander<K>(wk0, wk1, (nb.y + nb.z) & 1);
            else
                reg_wander<K>(wk1, wk0, (1 + nb.y + nb.z) & 1);
        }
    }

    if (HOUD) {
        // one wave per temperature: differing sites per row, prefix in site order, chosen site
        const int wave = tid >> 6, lane = tid & 63, nwave = nthr >> 6;
        const int chunk = (R0 + 63) / 64;
        for (int q = wave; q < G; q += nwave) {
            if (t0 + q >= g.M) continue;
            const uint32_t* ra = rows + (q * 2 + 0) * R0;
            const uint32_t* rb = rows + (q * 2 + 1) * R0;
            int32_t mine = 0;
            for (int rr = lane * chunk; rr < min(R0, (lane + 1) * chunk); ++rr) {
                const uint32_t d = (ra[rr] ^ rb[rr]) & MASK;
                diff[q * R0 + rr] = d;
                mark[q * R0 + rr] = 0u;
                mine += __popc(d);
            }
            int32_t incl = mine;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int32_t v = __shfl_up(incl, off, 64);
                if (lane >= off) incl += v;
            }
            const int32_t count = __shfl(incl, 63, 64);
            if (count > 0) {
                const uint32_t u = philox10((uint32_t)(t0 + q), e, 0u, stream_word(kStreamPtHoudayer, sw), g.key0,
                                            g.key1).v0;
                const int32_t k = (int32_t)(((uint64_t)u * (uint64_t)count) >> 32);
                const int32_t before = incl - mine;
                if (k >= before && k < incl) {
                    int32_t left = k - before;
                    for (int rr = lane * chunk; rr < min(R0, (lane + 1) * chunk); ++rr) {
                        uint32_t d = diff[q * R0 + rr];
                        const int32_t c = __popc(d);
                        if (left < c) {
                            for (; left > 0; --left) d &= d - 1;
                            mark[q * R0 + rr] = d & (~d + 1u);
                            break;
                        }
                        left -= c;
                    }
                }
            }
        }
        // grow every temperature's cluster together until none changes
        const int q = tid / R0, rr = tid - q * R0;
        const bool grower = q < G && t0 + q < g.M;
        const PtRowNb gb = pt_row_nb(g, grower ? rr : 0);
        for (;;) {
            __syncthreads();
            if (tid == 0) flag[0] = 0;
            __syncthreads();
            if (grower) {
                const uint32_t* mq = mark + q * R0;
                const uint32_t d = diff[q * R0 + rr], m = mq[rr];
                uint32_t m2 = d & (m | mq[gb.yp] | mq[gb.ym] | mq[gb.zp] | mq[gb.zm]);
                for (;;) {
                    const uint32_t m3 = d & (m2 | rot_up32<LX>(m2) | rot_down32<LX>(m2));
                    if (m3 == m2) break;
                    m2 = m3;
                }
                if (m2 != m) {
                    mark[q * R0 + rr] = m2;
                    flag[0] = 1;
                }
            }
            __syncthreads();
            if (flag[0] == 0) break;
        }
        if (live) rows[base + r] ^= mark[tl * R0 + r];
        __syncthreads();
    }

    if (live) {
        const uint32_t own = rows[base + r];
        const uint32_t dx = own ^ rot_down32<LX>(own), dy = own ^ rows[base + nb.yp], dz = own ^ rows[base + nb.zp];
        int32_t en = 0;
#pragma unroll
        for (int x = 0; x < LX; ++x) {
            const int4 a = rec[2 * (x * R0 + r)];
            en += (2 * (a.x & sbit(dx, x)) - a.x) + (2 * (a.y & sbit(dy, x)) - a.y) + (2 * (a.z & sbit(dz, x)) - a.z);
        }
        atomicAdd(&esum[tl * 2 + rep], (unsigned long long)(int64_t)en);
        *grow = own;
    }
    __syncthreads();
    if (live && r == 0) E[((int64_t)run * 2 + rep) * g.M + slot] = (int64_t)esum[tl * 2 + rep];
}

// Tempering step: one wave per replica group (run, replica); lane t decides
// pair (t, t+1), first the pairs with t even, then those with t odd.
__global__ __launch_bounds__(256) void k_pt_swap(PtGeom g, int32_t* __restrict__ perm,
                                                 const int64_t* __restrict__ E, int64_t* __restrict__ swaps,
                                                 const uint32_t* __restrict__ ptab, uint32_t e)
{
    __shared__ int32_t sp[4][64];
    __shared__ int64_t se[4][64];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int grp = blockIdx.x * 4 + wv;
    const bool live = grp < 2 * g.runs;
    const int run = grp >> 1, rep = grp & 1;
    if (live && lane < g.M) {
        const int32_t c = perm[(int64_t)grp * g.M + lane];
        sp[wv][lane] = c;
        se[wv][lane] = E[(int64_t)grp * g.M + c];
    }
    const bool pair = live && lane + 1 < g.M;
    u32x4 w{0, 0, 0, 0};
    if (pair)
        w = philox10((uint32_t)lane, e, (uint32_t)rep, stream_word(kStreamPtSwap, (uint32_t)run), g.key0, g.key1);
    __syncthreads();
    for (int ph = 0; ph < 2; ++ph) {
        if (pair && (lane & 1) == ph) {
            const int64_t x = se[wv][lane] - se[wv][lane + 1];
            if (exp_at_least(ptab + (int64_t)lane * kPtTable, w, -x)) {
                const int32_t c = sp[wv][lane];
                sp[wv][lane] = sp[wv][lane + 1];
                sp[wv][lane + 1] = c;
                const int64_t v = se[wv][lane];
                se[wv][lane] = se[wv][lane + 1];
                se[wv][lane + 1] = v;
                swaps[(int64_t)grp * (g.M - 1) + lane] += 1;
            }
        }
        __syncthreads();
    }
    if (live && lane < g.M) perm[(int64_t)grp * g.M + lane] = sp[wv][lane];
}

// Initial spins sigma = bit 31 of word i & 3 of Philox (i >> 2, t, replica,
// 10 << 24 | run) into slot t.  One thread per row; grid covers runs*2*M*R0.
__global__ __launch_bounds__(256) void k_pt_init_spins(PtGeom g, uint64_t* __restrict__ spins)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)g.runs * 2 * g.M * g.R0;
    if (k >= total) return;
    const int r = (int)(k % g.R0);
    const int t = (int)((k / g.R0) % g.M);
    const int rep = (int)((k / ((int64_t)g.R0 * g.M)) % 2);
    const int run = (int)(k / ((int64_t)g.R0 * g.M * 2));
    uint64_t row = 0;
    for (int x = 0; x < g.Lx; ++x) {
        const uint32_t i = (uint32_t)(x + g.Lx * r);
        const u32x4 o = philox10(i >> 2, (uint32_t)t, (uint32_t)rep, stream_word(kStreamPtSpin, (uint32_t)run),
                                 g.key0, g.key1);
        const uint32_t ws[4] = {o.v0, o.v1, o.v2, o.v3};
        row |= (uint64_t)(ws[i & 3] >> 31) << x;
    }
    spins[k] = row;
}

// Energies of every slot from scratch: grid (M, runs * 2), one block per slot.
__global__ __launch_bounds__(256) void k_pt_energy(PtGeom g, const int4* __restrict__ rec,
                                                   const uint64_t* __restrict__ spins, int64_t* __restrict__ E)
{
    __shared__ unsigned long long acc;
    const int64_t lat = (int64_t)blockIdx.y * g.M + blockIdx.x;  // (run, replica, slot)
    const uint64_t* rw = spins + lat * g.R0;
    if (threadIdx.x == 0) acc = 0ull;
    __syncthreads();
    for (int r = threadIdx.x; r < g.R0; r += blockDim.x) {
        const PtRowNb nb = pt_row_nb(g, r);
        atomicAdd(&acc, (unsigned long long)(int64_t)row_energy<false>(g, rec, r, rw[r], rw[nb.yp], rw[nb.zp]));
    }
    __syncthreads();
    if (threadIdx.x == 0) E[lat] = (int64_t)acc;
}

}  // namespace micsa
