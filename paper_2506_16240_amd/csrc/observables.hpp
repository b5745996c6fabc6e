// Four-point correlation of the replica overlap field (Sec. 3).
//
// For a pair of replicas (a, b) of one sample the overlap field is
// q_x = s^a_x s^b_x, in bits w_x = sigma^a_x ^ sigma^b_x (q = 1 - 2w).  Along
// axis mu and distance r,
//     sum_x q_x q_{x + r e_mu} = N - 2 #{x : w_x != w_{x + r e_mu}},
// so the correlation reduces to popcounts of XORs of bit-packed w.
//
// Packed form (one pair): per parity p and row (y, z), the Kx sites of that
// parity, bit k = site x = 2k + ((p + y + z) & 1), stored as an "extended"
// row of E words whose bit j is w at k = j mod Kx, for j < 32 E; E covers
// Kx + 32 bits, so any cyclic 32-bit window starting at k < Kx is two
// adjacent words.  Partners of the parity-p site at k of row (y, z):
//   +r along y / z: the site at the same k of row (y + r, z) / (y, z + r),
//     parity p ^ (r & 1);
//   +r along x: parity p ^ (r & 1), index k + r/2 (r even) or
//     k + (r - 1)/2 + ((p + y + z) & 1) (r odd), cyclic in Kx.
#pragma once
#include "bitplane_kernels.hpp"

namespace micsa {

struct C4Geom {
    int32_t E;     // words per extended row
    int32_t Wv;    // words holding the Kx valid bits: ceil(Kx / 32)
    int32_t rmax;  // largest distance per axis: max side / 2
    int32_t npair; // replica pairs per sample: R (R - 1) / 2
};

// Extended overlap rows of the pairs sp0 .. sp0 + gridDim.y - 1 (sp = s * npair
// + pair): Q[sp - sp0][p][row][E].
// Thread per output word; the bits come from the spin bytes (byte layout) or
// from the lane of the sample in the bit-plane words.
template <bool BIT>
__global__ void __launch_bounds__(256) k_pack_overlap(GeomB gb, C4Geom cg, int sp0, const uint8_t* __restrict__ spin,
                                                      const uint64_t* __restrict__ bspin, uint32_t* __restrict__ Q)
{
    const Geom& g = gb.g;
    const int64_t per_pair = (int64_t)2 * g.rows * cg.E;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= per_pair) return;
    const int sp = sp0 + (int)blockIdx.y;  // s * npair + pair
    const int s = sp / cg.npair;
    int pair = sp - s * cg.npair, a = 0;
    while (pair >= g.R - 1 - a) {  // pair -> (a, b), a < b, in lexicographic order
        pair -= g.R - 1 - a;
        ++a;
    }
    const int b = a + 1 + pair;
    const int e = (int)(t % cg.E);
    const int64_t prow = t / cg.E;  // p * rows + row
    const int p = (int)(prow / g.rows);
    const int64_t row = prow - (int64_t)p * g.rows;
    uint32_t word = 0;
    for (int j = 0; j < 32; ++j) {
        const int k = (32 * e + j) % g.Kx;
        const int64_t h = row * g.Kx + k;
        uint32_t va, vb;
        if (BIT) {
            int la, lb;
            const int64_t wa = bp_word_of(gb, s, a, la), wb = bp_word_of(gb, s, b, lb);
            va = (uint32_t)(bspin[(wa * 2 + p) * g.Nh + h] >> la) & 1u;
            vb = (uint32_t)(bspin[(wb * 2 + p) * g.Nh + h] >> lb) & 1u;
        } else {
            va = spin[(((int64_t)s * g.R + a) * 2 + p) * g.Nh + h];
            vb = spin[(((int64_t)s * g.R + b) * 2 + p) * g.Nh + h];
        }
        word |= ((va ^ vb) & 1u) << j;
    }
    Q[(int64_t)blockIdx.y * per_pair + t] = word;
}

// Counts D[s][mu][r] += #{x : w_x != w_{x + r e_mu}} over the pairs of sample
// s.  grid.x over the valid words (p, row, v < Wv) of one pair, grid.y over
// (mu, r) flattened as mu * (rmax + 1) + r, grid.z over the packed pairs
// sp0 .. sp0 + gridDim.z - 1.
// Distances beyond L_mu / 2 are skipped (their slots stay 0).
__global__ void __launch_bounds__(256) k_c4_count(Geom g, C4Geom cg, int sp0, const uint32_t* __restrict__ Q,
                                                  unsigned long long* __restrict__ D)
{
    const int mu = blockIdx.y / (cg.rmax + 1), r = blockIdx.y - mu * (cg.rmax + 1);
    const int side = mu == 0 ? g.Lx : (mu == 1 ? g.Ly : g.Lz);
    if (2 * r > side) return;  // whole block: uniform
    const int s = (sp0 + (int)blockIdx.z) / cg.npair;
    const int64_t per_pair = (int64_t)2 * g.rows * cg.E;
    const uint32_t* Qp = Q + (int64_t)blockIdx.z * per_pair;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int cnt = 0;
    if (t < (int64_t)2 * g.rows * cg.Wv) {
        const int v = (int)(t % cg.Wv);
        const int64_t prow = t / cg.Wv;
        const int p = (int)(prow / g.rows);
        const int row = (int)(prow - (int64_t)p * g.rows);
        const int y = row % g.Ly, z = row / g.Ly;
        const int pp = p ^ (r & 1);
        const uint32_t own = Qp[((int64_t)p * g.rows + row) * cg.E + v];
        const int nvalid = min(32, g.Kx - 32 * v);
        const uint32_t mask = nvalid >= 32 ? 0xFFFFFFFFu : ((1u << nvalid) - 1u);
        uint32_t part;
        if (mu == 0) {
            const int q = (p + y + z) & 1;
            const int shift = (r & 1) ? (r - 1) / 2 + q : r / 2;
            const int b0 = (32 * v + shift) % g.Kx;  // window start in the partner's extended row
            const uint32_t* pr = Qp + ((int64_t)pp * g.rows + row) * cg.E;
            const int wi = b0 >> 5, sh = b0 & 31;
            const uint32_t lo = pr[wi], hi = pr[wi + 1];
            part = sh ? ((lo >> sh) | (hi << (32 - sh))) : lo;
        } else {
            const int y2 = mu == 1 ? (y + r) % g.Ly : y;
            const int z2 = mu == 2 ? (z + r) % g.Lz : z;
            part = Qp[((int64_t)pp * g.rows + (y2 + g.Ly * z2)) * cg.E + v];
        }
        cnt = __popc((own ^ part) & mask);
    }
    block_add(D + ((int64_t)(s * 3 + mu) * (cg.rmax + 1) + r) * kSlots, cnt);
}

// out[e] = sum of the kSlots accumulator slots of entity e (thread per entity).
__global__ void __launch_bounds__(256) k_sum_slots(const unsigned long long* __restrict__ slots, int64_t n,
                                                   long long* __restrict__ out)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n) return;
    unsigned long long t = 0;
    for (int k = 0; k < kSlots; ++k) t += slots[e * kSlots + k];
    out[e] = (long long)t;
}

// Device-pointer logging: one row of the energy and daemon logs from the
// slots of every lattice (thread per lattice): E = 2 U - 3 N from the
// unsatisfied-bond count U, D = 4 sum m.  A null output is skipped.
__global__ void __launch_bounds__(256) k_log_from_slots(const unsigned long long* __restrict__ U,
                                                        const unsigned long long* __restrict__ Ms, int L,
                                                        int64_t N, long long* __restrict__ E,
                                                        long long* __restrict__ D)
{
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= L) return;
    unsigned long long u = 0, m = 0;
    for (int k = 0; k < kSlots; ++k) {
        if (E) u += U[(int64_t)l * kSlots + k];
        if (D) m += Ms[(int64_t)l * kSlots + k];
    }
    if (E) E[l] = 2 * (long long)u - 3 * N;
    if (D) D[l] = 4 * (long long)m;
}

// The same from the resident kernel's log of (U, sum m) pairs, n = rows x L.
__global__ void __launch_bounds__(256) k_log_from_pairs(const long long* __restrict__ raw, int64_t n, int64_t N,
                                                        long long* __restrict__ E, long long* __restrict__ D)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= n) return;
    if (E) E[e] = 2 * raw[2 * e] - 3 * N;
    if (D) D[e] = 4 * raw[2 * e + 1];
}

}  // namespace micsa
