// Byte-layout kernels: initialisation, daemon refresh, one MicSA or
// heat-bath half sweep per launch, and the reductions (energy, daemon
// energy, overlap).  Layout and notation: geometry.hpp.
#pragma once
#include "geometry.hpp"
#include "philox.hpp"

namespace micsa {

// Neighbourhood of a 4-site word (sites h0 .. h0+3 of parity P in row (y,z)):
// the spin bits of the six opposite-parity neighbours and the coupling bits of
// the bonds to them, in matching order (A = same k, B = k +- 1 in the row),
// each as one bit per byte.  The coupling bits of a bond live in the spin
// byte of its even end (geometry.hpp): for P = 0 in `own`, the word being
// updated, for P = 1 in the neighbour words themselves.
struct Nbhd {
    uint32_t nb[6];
    uint32_t jb[6];
};

template <int P>
__device__ __forceinline__ Nbhd gather(const Geom& g, uint32_t own, const uint32_t* __restrict__ oth, int row,
                                       int c)
{
    const int z = (int)((uint32_t)row / (uint32_t)g.Ly), y = row - z * g.Ly;
    const int q = (y + z) & 1;
    const int dir = (q ^ P) ? 1 : -1;
    const int cs = dir > 0 ? (c + 1 == g.Wr ? 0 : c + 1) : (c == 0 ? g.Wr - 1 : c - 1);
    const int yp = y + 1 == g.Ly ? 0 : y + 1, ym = y == 0 ? g.Ly - 1 : y - 1;
    const int zp = z + 1 == g.Lz ? 0 : z + 1, zm = z == 0 ? g.Lz - 1 : z - 1;
    const int r_yp = yp + g.Ly * z, r_ym = ym + g.Ly * z, r_zp = y + g.Ly * zp, r_zm = y + g.Ly * zm;
    const int64_t wr = g.Wr;
    const uint32_t m1 = 0x01010101u;
    uint32_t w[6];
    w[0] = oth[row * wr + c];
    w[1] = shift_word(w[0], oth[row * wr + cs], dir);
    w[2] = oth[r_yp * wr + c];
    w[3] = oth[r_ym * wr + c];
    w[4] = oth[r_zp * wr + c];
    w[5] = oth[r_zm * wr + c];
    Nbhd n;
#pragma unroll
    for (int d = 0; d < 6; ++d) n.nb[d] = w[d] & m1;
    // The same-k neighbour A is across bond (q ? -x : +x) of the even site at
    // A's position, the shifted neighbour B across (q ? +x : -x); this holds
    // for both parities because the even site is at x = 2k + q.
    const int dA = q ? kMx : kPx, dB = q ? kPx : kMx;
    if (P == 0) {
        // even sites own all six of their bonds
        const uint32_t jw = own >> 1;
        n.jb[0] = jbits(jw, dA);
        n.jb[1] = jbits(jw, dB);
        n.jb[2] = jbits(jw, kPy);
        n.jb[3] = jbits(jw, kMy);
        n.jb[4] = jbits(jw, kPz);
        n.jb[5] = jbits(jw, kMz);
    } else {
        // odd sites read each bond from the even neighbour's opposite slot
        n.jb[0] = jbits(w[0] >> 1, dA);
        n.jb[1] = jbits(w[1] >> 1, dB);
        n.jb[2] = jbits(w[2] >> 1, kMy);
        n.jb[3] = jbits(w[3] >> 1, kPy);
        n.jb[4] = jbits(w[4] >> 1, kMz);
        n.jb[5] = jbits(w[5] >> 1, kPz);
    }
    return n;
}

// ------------------------------------------------------------------ init
// Thread per 4 even sites of lattice l: the six bond bits of each even site
// from the forward-bond draws j_mu(i) = Philox(i, 0, 0, stream J | s)[mu] >> 31,
// written into bits 1..6 of its spin byte (bit 0, the spin, is kept).  Every
// replica of a sample carries the same bits.
__global__ void k_init_couplings(Geom g, uint8_t* __restrict__ spin)
{
    const int l = blockIdx.y;
    const int s = l / g.R;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= g.Nh / 4) return;
    const uint32_t sw = stream_word(kStreamCoupling, (uint32_t)s);
    uint32_t word = 0;
    for (int b = 0; b < 4; ++b) {
        const int64_t h = 4 * t + b;
        const int k = (int)(h % g.Kx);
        const int row = (int)(h / g.Kx);
        const int y = row % g.Ly, z = row / g.Ly;
        const int x = 2 * k + ((y + z) & 1);
        auto fwd = [&](int xx, int yy, int zz) {
            xx = (xx + g.Lx) % g.Lx;
            yy = (yy + g.Ly) % g.Ly;
            zz = (zz + g.Lz) % g.Lz;
            const uint32_t i = (uint32_t)(xx + (int64_t)g.Lx * (yy + (int64_t)g.Ly * zz));
            return philox10(i, 0u, 0u, sw, g.key0, g.key1);
        };
        const u32x4 o = fwd(x, y, z);
        const uint32_t byte = (o.v0 >> 31) | ((fwd(x - 1, y, z).v0 >> 31) << kMx) | ((o.v1 >> 31) << kPy) |
                              ((fwd(x, y - 1, z).v1 >> 31) << kMy) | ((o.v2 >> 31) << kPz) |
                              ((fwd(x, y, z - 1).v2 >> 31) << kMz);
        word |= byte << (8 * b);
    }
    uint32_t* ev = reinterpret_cast<uint32_t*>(spin + (int64_t)l * 2 * g.Nh);
    ev[t] = (ev[t] & 0x01010101u) | (word << 1);
}

// Thread per 8 consecutive natural sites i0 .. i0+7 (same row since Lx % 8 == 0):
// two Philox calls give 8 draws; the 4 sites of each parity land in one word.
template <typename F>
__device__ __forceinline__ void split8q(int q, const u32x4& a, const u32x4& b, F&& val, uint32_t& w_even,
                                        uint32_t& w_odd)
{
    // q = (x0 + y + z) & 1 of the first of the eight sites: site t has the
    // parity of q + t, so sites 0, 2, 4, 6 form one word and 1, 3, 5, 7 the
    // other (values selected, not output addresses)
    const uint32_t d[8] = {a.v0, a.v1, a.v2, a.v3, b.v0, b.v1, b.v2, b.v3};
    uint32_t first = 0, second = 0;
#pragma unroll
    for (int t = 0; t < 8; t += 2) {
        first |= val(d[t]) << (8 * (t >> 1));
        second |= val(d[t + 1]) << (8 * (t >> 1));
    }
    w_even = q ? second : first;
    w_odd = q ? first : second;
}

template <class F>
__device__ __forceinline__ void split8(const Geom& g, int64_t i0, const u32x4& a, const u32x4& b, F&& val,
                                       uint32_t& w_even, uint32_t& w_odd)
{
    const int x0 = (int)(i0 % g.Lx);
    const int64_t row = i0 / g.Lx;
    const int y = (int)(row % g.Ly), z = (int)(row / g.Ly);
    split8q((x0 + y + z) & 1, a, b, val, w_even, w_odd);
}

__global__ void k_init_spins(Geom g, uint8_t* __restrict__ spin)
{
    const int l = blockIdx.y;
    const int s = l / g.R, r = l % g.R;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= g.Nh / 4) return;
    const int64_t i0 = 8 * t;
    const uint32_t sw = stream_word(kStreamSpin, (uint32_t)s);
    const u32x4 a = philox10((uint32_t)(i0 >> 2), 0u, (uint32_t)r, sw, g.key0, g.key1);
    const u32x4 b = philox10((uint32_t)(i0 >> 2) + 1u, 0u, (uint32_t)r, sw, g.key0, g.key1);
    uint32_t we, wo;
    split8(g, i0, a, b, [](uint32_t u) { return u >> 31; }, we, wo);
    reinterpret_cast<uint32_t*>(spin + ((int64_t)l * 2 + 0) * g.Nh)[t] = we;
    reinterpret_cast<uint32_t*>(spin + ((int64_t)l * 2 + 1) * g.Nh)[t] = wo;
}

// Daemon refresh (Sec. 2.7, eq. prob-daemons-walkers): m = #{k : u >= t_k}.
// Every family of every site is redrawn: grid.y runs over (lattice, family)
// pairs d = l * gamma + a, and daemon a of site i is number j = a*N + i of
// the lattice's daemon stream (N is a multiple of 8, so j & 3 = i & 3).
__global__ void k_refresh(Geom g, uint8_t* __restrict__ dem, uint32_t rho, DaemonThresholds th)
{
    const int d = blockIdx.y;
    const int l = d / g.gamma, fam = d - l * g.gamma;
    const int s = l / g.R, r = l % g.R;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= g.Nh / 4) return;
    const int64_t i0 = 8 * t;
    const uint32_t c0 = (uint32_t)(i0 >> 2) + (uint32_t)fam * (uint32_t)(g.Nh / 2);  // (a*N + i0) >> 2
    const uint32_t sw = stream_word(kStreamDaemon, (uint32_t)s);
    const u32x4 a = philox10(c0, rho, (uint32_t)r, sw, g.key0, g.key1);
    const u32x4 b = philox10(c0 + 1u, rho, (uint32_t)r, sw, g.key0, g.key1);
    uint32_t we, wo;
    split8(g, i0, a, b,
           [&](uint32_t u) { return daemon_level(u, th); },
           we, wo);
    reinterpret_cast<uint32_t*>(dem + ((int64_t)d * 2 + 0) * g.Nh)[t] = we;
    reinterpret_cast<uint32_t*>(dem + ((int64_t)d * 2 + 1) * g.Nh)[t] = wo;
}

__device__ __forceinline__ bool sweep_is_refresh(int64_t k, int32_t P)
{
    return P >= 1 ? (k % P == 0) : (((k + 1) & k) == 0);
}

__device__ __forceinline__ int64_t sweep_refresh_index(int64_t k, int32_t P)
{
    if (P >= 1) return k / P;
    return 63 - __clzll((unsigned long long)(k + 1));  // floor(log2(k + 1))
}

// Refresh whose sweep index comes from device memory (*dk), for replayable
// graphs (gamma = 1): does nothing unless sweep *dk is a refresh point;
// thresholds from the schedule's table.
__global__ void k_refresh_dev(Geom g, uint8_t* __restrict__ dem, const int64_t* __restrict__ dk, int32_t period,
                              const DaemonThresholds* __restrict__ dth)
{
    const int64_t k = *dk;
    if (!sweep_is_refresh(k, period)) return;
    const int64_t rho = sweep_refresh_index(k, period);
    const DaemonThresholds th = dth[rho];
    const int l = blockIdx.y;
    const int s = l / g.R, r = l % g.R;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= g.Nh / 4) return;
    const int64_t i0 = 8 * t;
    const uint32_t sw = stream_word(kStreamDaemon, (uint32_t)s);
    const u32x4 a = philox10((uint32_t)(i0 >> 2), (uint32_t)rho, (uint32_t)r, sw, g.key0, g.key1);
    const u32x4 b = philox10((uint32_t)(i0 >> 2) + 1u, (uint32_t)rho, (uint32_t)r, sw, g.key0, g.key1);
    uint32_t we, wo;
    split8(g, i0, a, b,
           [&](uint32_t u) { return daemon_level(u, th); },
           we, wo);
    reinterpret_cast<uint32_t*>(dem + ((int64_t)l * 2 + 0) * g.Nh)[t] = we;
    reinterpret_cast<uint32_t*>(dem + ((int64_t)l * 2 + 1) * g.Nh)[t] = wo;
}

// Advance the device sweep counter (one thread; launched after a sweep's
// last kernel in replayable graphs).
__global__ void k_count_sweep(int64_t* dk) { *dk += 1; }

__global__ void k_set_counter(int64_t* dk, int64_t k) { *dk = k; }

// --------------------------------------------------------- MicSA half sweep
// Creutz move with a 2-bit daemon (eqs. Creutz and flip-OK).  With u the
// number of unsatisfied bonds of the site (sigma ^ sigma_nb ^ j = 1),
// dH = 12 - 4u, so 0 <= 4m - dH <= 12  <=>  3 <= m + u <= 6, and then the
// new level is m + u - 3.  Per byte, t = m + u + 5 lies in 5..14 and the
// move is legal iff t is in 8..11, i.e. bit 3 set and bit 2 clear; the new
// level is then t & 3.
__device__ __forceinline__ void micsa_word(uint32_t& S, uint32_t& M, const Nbhd& n, int& dE)
{
    uint32_t u = 0;
#pragma unroll
    for (int d = 0; d < 6; ++d) u += xor3(S, n.nb[d], n.jb[d]);
    const uint32_t t = M + u + 0x05050505u;
    const uint32_t acc = (t >> 3) & ~(t >> 2) & 0x01010101u;
    const uint32_t mask = acc * 0xFFu;
    S ^= acc;
    M = (M & ~mask) | (t & 0x03030303u & mask);
    dE += 12 * (int)__popc(acc) - 4 * (int)bytesum(u & mask);
}

template <int P>
__global__ void __launch_bounds__(256) k_micsa_half(Geom g, uint8_t* __restrict__ spin,
                                                    uint8_t* __restrict__ dem,
                                                    unsigned long long* __restrict__ tally, int fam)
{
    const int l = blockIdx.y;
    const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    int dE = 0;
    if (w < (uint32_t)g.rows * (uint32_t)g.Wr) {
        const int row = (int)(w / (uint32_t)g.Wr), c = (int)(w - (uint32_t)row * (uint32_t)g.Wr);
        uint32_t* own = reinterpret_cast<uint32_t*>(spin + ((int64_t)l * 2 + P) * g.Nh);
        const uint32_t* oth = reinterpret_cast<const uint32_t*>(spin + ((int64_t)l * 2 + (1 - P)) * g.Nh);
        uint32_t* dm = reinterpret_cast<uint32_t*>(dem + (((int64_t)l * g.gamma + fam) * 2 + P) * g.Nh);
        const uint32_t W0 = own[w];
        const Nbhd n = gather<P>(g, W0, oth, row, c);
        const uint32_t S0 = W0 & 0x01010101u;  // spin bits (even bytes also hold their bonds)
        uint32_t S = S0, M = dm[w];
        micsa_word(S, M, n, dE);
        own[w] = W0 ^ S ^ S0;
        dm[w] = M;
    }
    block_add(tally + (int64_t)l * kSlots, dE);
}

// ------------------------------------------ canonical (random-number) updates
// The two baselines draw one 32-bit uniform u per visited site:
// u = Philox(h>>2, 2k+p, r, stream | s)[h & 3] for the parity-split index h.
//   ALG 0, heat bath: the new spin is +1 iff u < tau[v], where v counts the
//     neighbours with J s_nb = -1 (local field h = 6 - 2v).
//   ALG 1, Metropolis: the flip is taken iff u < theta[q], q = (dH + 12)/4;
//     dH = 2 s h, so q = 6 - v for s = +1 and q = v for s = -1.
// Four sites per word (byte b = site b); v holds the four counts bytewise.
// dE accumulates 2 s_old h for every spin that changed.
template <int ALG>
__device__ __forceinline__ uint32_t canonical4(uint32_t S, uint32_t v, const u32x4& rnd, const uint64_t* tab,
                                               int& dE)
{
    const uint32_t ru[4] = {rnd.v0, rnd.v1, rnd.v2, rnd.v3};
    uint32_t Sn = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const uint32_t vb = (v >> (8 * b)) & 0xFFu;
        const uint32_t old = (S >> (8 * b)) & 1u;
        uint32_t nw;
        if (ALG == 0) {
            nw = (uint64_t)ru[b] < tab[vb] ? 0u : 1u;
        } else {
            const uint32_t q = old ? vb : 6u - vb;
            nw = old ^ ((uint64_t)ru[b] < tab[q] ? 1u : 0u);
        }
        if (nw != old) dE += 2 * (1 - 2 * (int)old) * (6 - 2 * (int)vb);
        Sn |= nw << (8 * b);
    }
    return Sn;
}

template <int ALG>
__device__ __forceinline__ uint32_t canonical_stream(uint32_t s)
{
    return stream_word(ALG == 0 ? kStreamHeatBath : kStreamMetropolis, s);
}

// ------------------------------------------- heat-bath / Metropolis half sweep
// With dk != nullptr the sweep index k = *dk and the table of refresh rho(k)
// comes from device memory (replayable graphs); otherwise from the arguments.
template <int P, int ALG>
__global__ void __launch_bounds__(256) k_heatbath_half(Geom g, uint8_t* __restrict__ spin, uint32_t time,
                                                       HeatBathThresholds th,
                                                       unsigned long long* __restrict__ tally,
                                                       const int64_t* __restrict__ dk, int32_t period,
                                                       const HeatBathThresholds* __restrict__ hth)
{
    __shared__ uint64_t tau[8];
    if (dk) {
        const int64_t k = *dk;
        time = (uint32_t)(2 * k + P);
        if (threadIdx.x < 7) tau[threadIdx.x] = hth[sweep_refresh_index(k, period)].tau[threadIdx.x];
    } else if (threadIdx.x < 7) {
        tau[threadIdx.x] = th.tau[threadIdx.x];
    }
    __syncthreads();
    const int l = blockIdx.y;
    const int s = l / g.R, r = l % g.R;
    const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    int dE = 0;
    if (w < (uint32_t)g.rows * (uint32_t)g.Wr) {
        const int row = (int)(w / (uint32_t)g.Wr), c = (int)(w - (uint32_t)row * (uint32_t)g.Wr);
        uint32_t* own = reinterpret_cast<uint32_t*>(spin + ((int64_t)l * 2 + P) * g.Nh);
        const uint32_t* oth = reinterpret_cast<const uint32_t*>(spin + ((int64_t)l * 2 + (1 - P)) * g.Nh);
        const uint32_t W0 = own[w];
        const Nbhd n = gather<P>(g, W0, oth, row, c);
        uint32_t v = 0;
#pragma unroll
        for (int d = 0; d < 6; ++d) v += n.nb[d] ^ n.jb[d];
        const u32x4 rnd = philox10(w, time, (uint32_t)r, canonical_stream<ALG>((uint32_t)s), g.key0, g.key1);
        // new spin bits; the bond bits of even bytes are kept
        own[w] = canonical4<ALG>(W0, v, rnd, tau, dE) | (W0 & ~0x01010101u);
    }
    block_add(tally + (int64_t)l * kSlots, dE);
}

// ------------------------------------------------------------- wandering
// Walkers (Sec. 2.6): the wandering step along direction dir (+x, -x, +y,
// -y, +z, -z) exchanges the level of every site s of parity p with that of
// s + e_dir.  Written as two gathers into the other buffer: a site of parity
// p takes the level at s + e_dir, a site of parity 1-p the level at t - e_dir
// (both sites of the other parity).  Thread per word position (row, c) of
// both parity arrays; grid.y over (lattice, family) pairs d = l*gamma + a.
// Family a wanders along kWalkerDir[a] (Sec. 2.8: forward X, Y, Z, then
// backward X, Y, Z).
__constant__ const int kWalkerDir[6] = {kPx, kPy, kPz, kMx, kMy, kMz};

__global__ void __launch_bounds__(256) k_wander(Geom g, const uint8_t* __restrict__ dem_in,
                                                uint8_t* __restrict__ dem_out, int p)
{
    const int l = blockIdx.y;  // (lattice, family) pair
    const int dir = kWalkerDir[l % g.gamma];
    const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= (uint32_t)g.rows * (uint32_t)g.Wr) return;
    const int row = (int)(w / (uint32_t)g.Wr), c = (int)(w - (uint32_t)row * (uint32_t)g.Wr);
    const int z = row / g.Ly, y = row - z * g.Ly;
    const int sgn = (dir & 1) ? -1 : 1;  // even dir index: forward
    const int axis = dir >> 1;
    const int qp = (p + y + z) & 1;      // sites of parity p sit at x = 2k + qp
    const int64_t wr = g.Wr;
    for (int a = 0; a < 2; ++a) {  // destination parity array: a == 0 -> parity p
        const int par = a == 0 ? p : 1 - p;
        const uint32_t* src = reinterpret_cast<const uint32_t*>(dem_in + ((int64_t)l * 2 + (1 - par)) * g.Nh);
        uint32_t* dst = reinterpret_cast<uint32_t*>(dem_out + ((int64_t)l * 2 + par) * g.Nh);
        const int toward = a == 0 ? sgn : -sgn;  // partner offset along the axis
        uint32_t v;
        if (axis == 0) {
            // x +- 1 of a site at x = 2k + q of this parity is at index k + shift in the other array
            const int q = a == 0 ? qp : 1 - qp;
            const int shift = toward > 0 ? q : q - 1;  // 0 or +1, or -1 or 0
            const uint32_t A = src[row * wr + c];
            if (shift == 0) {
                v = A;
            } else {
                const int cs = shift > 0 ? (c + 1 == g.Wr ? 0 : c + 1) : (c == 0 ? g.Wr - 1 : c - 1);
                v = shift_word(A, src[row * wr + cs], shift);
            }
        } else if (axis == 1) {
            const int yy = toward > 0 ? (y + 1 == g.Ly ? 0 : y + 1) : (y == 0 ? g.Ly - 1 : y - 1);
            v = src[(int64_t)(yy + g.Ly * z) * wr + c];
        } else {
            const int zz = toward > 0 ? (z + 1 == g.Lz ? 0 : z + 1) : (z == 0 ? g.Lz - 1 : z - 1);
            v = src[(int64_t)(y + g.Ly * zz) * wr + c];
        }
        dst[w] = v;
    }
}

// -------------------------------------------------------------- reductions
// U = number of unsatisfied bonds, counted once each from the even end;
// H = 2U - 3N (eq. Hamiltonian).  Adds U to the slots of lattice l.
__global__ void __launch_bounds__(256) k_unsat_bonds(Geom g, const uint8_t* __restrict__ spin,
                                                     unsigned long long* __restrict__ out)
{
    const int l = blockIdx.y;
    const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
    int U = 0;
    if (w < (uint32_t)g.rows * (uint32_t)g.Wr) {
        const int row = (int)(w / (uint32_t)g.Wr), c = (int)(w - (uint32_t)row * (uint32_t)g.Wr);
        const uint32_t* ev = reinterpret_cast<const uint32_t*>(spin + ((int64_t)l * 2 + 0) * g.Nh);
        const uint32_t* od = reinterpret_cast<const uint32_t*>(spin + ((int64_t)l * 2 + 1) * g.Nh);
        const uint32_t W0 = ev[w];
        const Nbhd n = gather<0>(g, W0, od, row, c);
        const uint32_t S = W0 & 0x01010101u;
        uint32_t u = 0;
#pragma unroll
        for (int d = 0; d < 6; ++d) u += xor3(S, n.nb[d], n.jb[d]);
        U = (int)bytesum(u);
    }
    block_add(out + (int64_t)l * kSlots, U);
}

// Adds the sum of daemon levels of lattice l (both parities) to its slots.
__global__ void __launch_bounds__(256) k_level_sum(int64_t words_per_lattice, const uint32_t* __restrict__ dem,
                                                   unsigned long long* __restrict__ out)
{
    const int l = blockIdx.y;
    const int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int v = 0;
    if (w < words_per_lattice) v = (int)bytesum(dem[(int64_t)l * words_per_lattice + w]);
    block_add(out + (int64_t)l * kSlots, v);
}

// Adds the number of sites where replicas a and b of sample s differ to its slots.
__global__ void __launch_bounds__(256) k_differ_count(int64_t words_per_lattice, int R, int a, int b,
                                                      const uint32_t* __restrict__ spin,
                                                      unsigned long long* __restrict__ out)
{
    const int s = blockIdx.y;
    const int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int v = 0;
    if (w < words_per_lattice) {
        const uint32_t xa = spin[((int64_t)s * R + a) * words_per_lattice + w];
        const uint32_t xb = spin[((int64_t)s * R + b) * words_per_lattice + w];
        v = (int)__popc((xa ^ xb) & 0x01010101u);  // spin bits only
    }
    block_add(out + (int64_t)s * kSlots, v);
}

__global__ void k_fill_i64(unsigned long long* __restrict__ p, int64_t n, unsigned long long v)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace micsa
