/*
 * TEST INFRASTRUCTURE ONLY -- the CPU oracle for microcanonical simulated
 * annealing (MicSA) on the 3D Edwards-Anderson +-J spin glass.
 *
 * This file is the plain, slow, obviously correct reference that the HIP
 * product path is checked against.  It is used only by tests/, by the
 * smoke check and by the CPU-baseline leg of the benchmark; the product
 * library never links, loads or calls it, and it shares no code, header
 * or table with the GPU path.  Everything here is written from the paper
 * (Bernaschi et al., "Microcanonical simulated annealing", arXiv 2506.16240)
 * in its own notation: spins s = +-1, couplings J = +-1, daemons n = 4m.
 *
 * Storage (natural order, chosen for readability, not speed):
 *   site index     i = x + Lx*(y + Ly*z), N = Lx*Ly*Lz, periodic in all axes
 *   sigma[l][i]    spin bit, s = 1 - 2*sigma, l = sample*R + replica
 *   m[l][a][i]     level of daemon (or walker) a = 0..gamma-1 of site i,
 *                  n = 4*m, m in {0,1,2,3} (Sec. 2.2: gamma per spin)
 *   J[sample][i]   bits 0,1,2 = coupling bit j of the forward bonds
 *                  (i, i+e_x), (i, i+e_y), (i, i+e_z); J = 1 - 2*j
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11,
 * "Parallel random numbers: as easy as 1, 2, 3"), key = (lo32(seed),
 * hi32(seed)), with one counter per (stream, sample, replica, site, time):
 *   couplings  ctr = (i,      0,      0, 1<<24 | s)  j_mu(i) = out[mu] >> 31
 *   spins      ctr = (i>>2,   0,      r, 2<<24 | s)  sigma   = out[i&3] >> 31
 *   daemons    ctr = (j>>2,   rho,    r, 3<<24 | s)  u       = out[j&3], j = a*N + i
 *   heat bath  ctr = (h>>2,   2k+p,   r, 4<<24 | s)  u       = out[h&3], h = i>>1
 *   Metropolis ctr = (h>>2,   2k+p,   r, 5<<24 | s)  u       = out[h&3], h = i>>1
 * (rho = refresh index, k = sweep index, p = parity being updated).  The
 * paper leaves the generator unspecified; this map is the specification
 * both implementations follow.
 *
 * Parallelism: the only OpenMP use is a parallel loop over the sites of one
 * parity, which the paper's separability argument (Sec. 2.1, Sec. 2.3) makes
 * order-independent; integer reductions make the result deterministic.
 * The equilibrium workload of App. C (Gaussian couplings, continuous
 * walkers, parallel tempering, Houdayer moves) has its own section near
 * the end of the file, with its own storage and generator map; it runs
 * independent lattices in parallel.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Philox4x32-10, from its published definition (Salmon et al. 2011).  */
/* ------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; round++) {
        if (round > 0) { k0 += PHILOX_W0; k1 += PHILOX_W1; }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static uint32_t draw(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, int lane)
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    return out[lane];
}

enum { STREAM_J = 1, STREAM_SPIN = 2, STREAM_DAEMON = 3, STREAM_HEATBATH = 4, STREAM_METROPOLIS = 5 };

/* ------------------------------------------------------------------ */
/* Lattice geometry                                                    */
/* ------------------------------------------------------------------ */
typedef struct { int Lx, Ly, Lz; int64_t N; } geom;

static geom mk(int Lx, int Ly, int Lz)
{
    geom g = {Lx, Ly, Lz, (int64_t)Lx * Ly * Lz};
    return g;
}

static void coords(const geom *g, int64_t i, int *x, int *y, int *z)
{
    *x = (int)(i % g->Lx);
    *y = (int)((i / g->Lx) % g->Ly);
    *z = (int)(i / ((int64_t)g->Lx * g->Ly));
}

/* Site at (x, y, z) with periodic wrap; callers step at most one site
   outside the box. */
static int wrap(int a, int L) { return a < 0 ? a + L : (a >= L ? a - L : a); }

static int64_t site(const geom *g, int x, int y, int z)
{
    x = wrap(x, g->Lx);
    y = wrap(y, g->Ly);
    z = wrap(z, g->Lz);
    return x + (int64_t)g->Lx * (y + (int64_t)g->Ly * z);
}

static int parity_of(const geom *g, int64_t i)
{
    int x, y, z;
    coords(g, i, &x, &y, &z);
    return (x + y + z) & 1;
}

static int spin(uint8_t sigma_bit) { return 1 - 2 * (int)sigma_bit; }
static int coupling(uint8_t jbits, int mu) { return 1 - 2 * (int)((jbits >> mu) & 1u); }

/*
 * Local field h_x = sum over the 6 neighbours y of J_xy s_y (eq. Hamiltonian,
 * Sec. 2.1).  The forward bonds of x are stored at x, the backward bonds at
 * the neighbour behind x.
 */
static int local_field(const geom *g, const uint8_t *J, const uint8_t *sig, int64_t i)
{
    int x, y, z;
    coords(g, i, &x, &y, &z);
    int64_t fwd[3] = {site(g, x + 1, y, z), site(g, x, y + 1, z), site(g, x, y, z + 1)};
    int64_t bwd[3] = {site(g, x - 1, y, z), site(g, x, y - 1, z), site(g, x, y, z - 1)};
    int h = 0;
    for (int mu = 0; mu < 3; mu++) {
        h += coupling(J[i], mu) * spin(sig[fwd[mu]]);
        h += coupling(J[bwd[mu]], mu) * spin(sig[bwd[mu]]);
    }
    return h;
}

/* ------------------------------------------------------------------ */
/* Initial state (Sec. 3: J = +-1 with probability 1/2, eq. Hamiltonian; */
/* start from a fully disordered, infinite-temperature configuration).  */
/* ------------------------------------------------------------------ */
void oracle_init_couplings(int Lx, int Ly, int Lz, int S, uint64_t seed, uint8_t *J)
{
    geom g = mk(Lx, Ly, Lz);
    for (int s = 0; s < S; s++)
        for (int64_t i = 0; i < g.N; i++) {
            uint32_t ctr[4] = {(uint32_t)i, 0u, 0u, (uint32_t)(STREAM_J << 24) | (uint32_t)s};
            uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
            uint32_t o[4];
            oracle_philox4x32_10(ctr, key, o);
            J[(int64_t)s * g.N + i] = (uint8_t)((o[0] >> 31) | ((o[1] >> 31) << 1) | ((o[2] >> 31) << 2));
        }
}

void oracle_init_spins(int Lx, int Ly, int Lz, int S, int R, uint64_t seed, uint8_t *sigma)
{
    geom g = mk(Lx, Ly, Lz);
    for (int s = 0; s < S; s++)
        for (int r = 0; r < R; r++)
            for (int64_t i = 0; i < g.N; i++)
                sigma[((int64_t)s * R + r) * g.N + i] =
                    (uint8_t)(draw(seed, (uint32_t)(i >> 2), 0u, (uint32_t)r,
                                   (uint32_t)(STREAM_SPIN << 24) | (uint32_t)s, (int)(i & 3)) >> 31);
}

/* ------------------------------------------------------------------ */
/* Daemon refresh, eq. prob-daemons-walkers (Sec. 2.5):                */
/*   p(n = 4m) = exp(-4 m beta) (1 - exp(-4 beta)) / (1 - exp(-16 beta)) */
/* sampled by inverse CDF on a 32-bit uniform u:                       */
/*   m = #{k in 0..2 : u >= t_k},  t_k = floor(2^32 * P(m <= k))       */
/*   P(m <= k) = (1 - exp(-4 beta (k+1))) / (1 - exp(-16 beta))         */
/* held as 64-bit integers so that P = 1 (T -> 0) gives t_k = 2^32.    */
/* ------------------------------------------------------------------ */
void oracle_daemon_thresholds(double T, uint64_t t[3])
{
    double beta = 1.0 / T;
    for (int k = 0; k < 3; k++) {
        double cdf = expm1(-4.0 * beta * (double)(k + 1)) / expm1(-16.0 * beta);
        t[k] = (uint64_t)floor(cdf * 4294967296.0);
    }
}

/* A refresh redraws all gamma daemons of every site; daemon a of site i */
/* is drawn as number j = a*N + i of the lattice's daemon stream.        */
void oracle_refresh(int Lx, int Ly, int Lz, int S, int R, int gamma, uint64_t seed, int64_t rho,
                    double T, uint8_t *m)
{
    geom g = mk(Lx, Ly, Lz);
    uint64_t t[3];
    oracle_daemon_thresholds(T, t);
    for (int s = 0; s < S; s++)
        for (int r = 0; r < R; r++)
            for (int a = 0; a < gamma; a++)
                for (int64_t i = 0; i < g.N; i++) {
                    int64_t j = (int64_t)a * g.N + i;
                    uint64_t u = draw(seed, (uint32_t)(j >> 2), (uint32_t)rho, (uint32_t)r,
                                      (uint32_t)(STREAM_DAEMON << 24) | (uint32_t)s, (int)(j & 3));
                    int level = 0;
                    for (int k = 0; k < 3; k++) level += (u >= t[k]);
                    m[(((int64_t)s * R + r) * gamma + a) * g.N + i] = (uint8_t)level;
                }
}

/* ------------------------------------------------------------------ */
/* MicSA half sweep (Sec. 2.3 eq. Creutz, Sec. 2.5 eq. flip-OK,        */
/* procedure of Sec. 2.8.1): for every site x of the given parity,     */
/* dH = H(flipped) - H = 2 s_x h_x; with the site's daemon n = n_{x,a} */
/* of the family a in use, the flip is legal iff 0 <= n - dH <= 12,    */
/* and then n -> n - dH.  dE[l] accumulates the change of H^EA.        */
/* ------------------------------------------------------------------ */
static int micsa_site(const geom *g, const uint8_t *Js, uint8_t *sig, uint8_t *dm, int64_t i)
{
    int dH = 2 * spin(sig[i]) * local_field(g, Js, sig, i);
    int n = 4 * (int)dm[i];
    if (n - dH >= 0 && n - dH <= 12) {
        sig[i] ^= 1u;
        dm[i] = (uint8_t)((n - dH) / 4);
        return dH;
    }
    return 0;
}

/* One elementary move on site i of a single lattice; returns dH (0 if rejected). */
int oracle_micsa_site(int Lx, int Ly, int Lz, int64_t i, const uint8_t *J, uint8_t *sigma, uint8_t *m)
{
    geom g = mk(Lx, Ly, Lz);
    return micsa_site(&g, J, sigma, m, i);
}

void oracle_micsa_half(int Lx, int Ly, int Lz, int S, int R, int gamma, int alpha, int parity,
                       const uint8_t *J, uint8_t *sigma, uint8_t *m, int64_t *dE)
{
    geom g = mk(Lx, Ly, Lz);
    for (int s = 0; s < S; s++)
        for (int r = 0; r < R; r++) {
            const uint8_t *Js = J + (int64_t)s * g.N;
            uint8_t *sig = sigma + ((int64_t)s * R + r) * g.N;
            uint8_t *dm = m + (((int64_t)s * R + r) * gamma + alpha) * g.N;
            int64_t acc = 0;
#pragma omp parallel for reduction(+ : acc) schedule(static)
            for (int64_t i = 0; i < g.N; i++) {
                if (parity_of(&g, i) != parity) continue;
                acc += micsa_site(&g, Js, sig, dm, i);
            }
            dE[(int64_t)s * R + r] += acc;
        }
}

/* ------------------------------------------------------------------ */
/* Heat bath, the canonical baseline named in Sec. 2.1: the new spin is */
/* +1 with probability 1/(1 + exp(-2 beta h)) whatever its old value.  */
/* The probability is a 64-bit threshold tau(h) = floor(2^32 P(+1)) and */
/* the spin is +1 iff u < tau.  Index v = (6 - h)/2 in 0..6.           */
/* ------------------------------------------------------------------ */
void oracle_heatbath_thresholds(double T, uint64_t tau[7])
{
    double beta = 1.0 / T;
    for (int v = 0; v < 7; v++) {
        double h = (double)(6 - 2 * v);
        tau[v] = (uint64_t)floor(4294967296.0 / (1.0 + exp(-2.0 * beta * h)));
    }
}

void oracle_heatbath_half(int Lx, int Ly, int Lz, int S, int R, uint64_t seed, int64_t k, int parity,
                          double T, const uint8_t *J, uint8_t *sigma, int64_t *dE)
{
    geom g = mk(Lx, Ly, Lz);
    uint64_t tau[7];
    oracle_heatbath_thresholds(T, tau);
    uint32_t time = (uint32_t)(2 * k + parity);
    for (int s = 0; s < S; s++)
        for (int r = 0; r < R; r++) {
            const uint8_t *Js = J + (int64_t)s * g.N;
            uint8_t *sig = sigma + ((int64_t)s * R + r) * g.N;
            int64_t acc = 0;
#pragma omp parallel for reduction(+ : acc) schedule(static)
            for (int64_t i = 0; i < g.N; i++) {
                if (parity_of(&g, i) != parity) continue;
                int h = local_field(&g, Js, sig, i);
                int64_t hidx = i >> 1;
                uint64_t u = draw(seed, (uint32_t)(hidx >> 2), time, (uint32_t)r,
                                  (uint32_t)(STREAM_HEATBATH << 24) | (uint32_t)s, (int)(hidx & 3));
                int s_new = (u < tau[(6 - h) / 2]) ? +1 : -1;
                int s_old = spin(sig[i]);
                if (s_new != s_old) {
                    acc += 2 * s_old * h;
                    sig[i] = (uint8_t)(s_new < 0);
                }
            }
            dE[(int64_t)s * R + r] += acc;
        }
}

/* ------------------------------------------------------------------ */
/* Metropolis, the canonical comparison of Sec. 4 (Table 3): the flip   */
/* of s is proposed and accepted with probability min(1, exp(-beta dH)),*/
/* dH = 2 s h.  As a 64-bit threshold theta(dH) = floor(2^32 e^{-beta  */
/* dH}) for dH > 0 and 2^32 ("always") for dH <= 0; the flip happens   */
/* iff u < theta.  Index q = (dH + 12) / 4 in 0..6.                    */
/* ------------------------------------------------------------------ */
void oracle_metropolis_thresholds(double T, uint64_t th[7])
{
    double beta = 1.0 / T;
    for (int q = 0; q < 7; q++) {
        int dH = 4 * q - 12;
        th[q] = dH <= 0 ? 4294967296ull : (uint64_t)floor(exp(-beta * (double)dH) * 4294967296.0);
    }
}

void oracle_metropolis_half(int Lx, int Ly, int Lz, int S, int R, uint64_t seed, int64_t k, int parity,
                            double T, const uint8_t *J, uint8_t *sigma, int64_t *dE)
{
    geom g = mk(Lx, Ly, Lz);
    uint64_t th[7];
    oracle_metropolis_thresholds(T, th);
    uint32_t time = (uint32_t)(2 * k + parity);
    for (int s = 0; s < S; s++)
        for (int r = 0; r < R; r++) {
            const uint8_t *Js = J + (int64_t)s * g.N;
            uint8_t *sig = sigma + ((int64_t)s * R + r) * g.N;
            int64_t acc = 0;
#pragma omp parallel for reduction(+ : acc) schedule(static)
            for (int64_t i = 0; i < g.N; i++) {
                if (parity_of(&g, i) != parity) continue;
                int dH = 2 * spin(sig[i]) * local_field(&g, Js, sig, i);
                int64_t hidx = i >> 1;
                uint64_t u = draw(seed, (uint32_t)(hidx >> 2), time, (uint32_t)r,
                                  (uint32_t)(STREAM_METROPOLIS << 24) | (uint32_t)s, (int)(hidx & 3));
                if (u < th[(dH + 12) / 4]) {
                    sig[i] ^= 1;
                    acc += dH;
                }
            }
            dE[(int64_t)s * R + r] += acc;
        }
}

/* ------------------------------------------------------------------ */
/* Walkers (Sec. 2.6): a wandering step along direction dir (0..5 = +x, */
/* -x, +y, -y, +z, -z) exchanges walker `alpha` of every site x of the  */
/* given parity with walker `alpha` of its neighbour x + e_dir.  A      */
/* wandering cycle is two timesteps: sites of one parity at even        */
/* timesteps, of the other at odd ones.                                 */
/* ------------------------------------------------------------------ */
void oracle_wander(int Lx, int Ly, int Lz, int S, int R, int gamma, int alpha, int dir, int parity,
                   uint8_t *m)
{
    geom g = mk(Lx, Ly, Lz);
    static const int step[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    for (int l = 0; l < S * R; l++) {
        uint8_t *dm = m + ((int64_t)l * gamma + alpha) * g.N;
        for (int64_t i = 0; i < g.N; i++) {
            if (parity_of(&g, i) != parity) continue;
            int x, y, z;
            coords(&g, i, &x, &y, &z);
            int64_t j = site(&g, x + step[dir][0], y + step[dir][1], z + step[dir][2]);
            uint8_t t = dm[i];
            dm[i] = dm[j];
            dm[j] = t;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Observables                                                          */
/* ------------------------------------------------------------------ */
/* H^EA = - sum over bonds J_xy s_x s_y (eq. Hamiltonian), each bond once
   as the forward bond of its lower-coordinate end. */
void oracle_energy(int Lx, int Ly, int Lz, int S, int R, const uint8_t *J, const uint8_t *sigma,
                   int64_t *E)
{
    geom g = mk(Lx, Ly, Lz);
    for (int s = 0; s < S; s++)
        for (int r = 0; r < R; r++) {
            const uint8_t *Js = J + (int64_t)s * g.N;
            const uint8_t *sig = sigma + ((int64_t)s * R + r) * g.N;
            int64_t H = 0;
            for (int64_t i = 0; i < g.N; i++) {
                int x, y, z;
                coords(&g, i, &x, &y, &z);
                int64_t fwd[3] = {site(&g, x + 1, y, z), site(&g, x, y + 1, z), site(&g, x, y, z + 1)};
                for (int mu = 0; mu < 3; mu++)
                    H -= coupling(Js[i], mu) * spin(sig[i]) * spin(sig[fwd[mu]]);
            }
            E[(int64_t)s * R + r] = H;
        }
}

/* H^aux = sum_x sum_a n_{x,a} (eq. H-total); n counts every daemon of */
/* a lattice (N * gamma).                                              */
void oracle_daemon_energy(int64_t N, int L, const uint8_t *m, int64_t *D)
{
    for (int l = 0; l < L; l++) {
        int64_t sum = 0;
        for (int64_t i = 0; i < N; i++) sum += 4 * (int64_t)m[(int64_t)l * N + i];
        D[l] = sum;
    }
}

/* Q_ab = sum_x s^a_x s^b_x (replica overlap, q = Q/N, App. C). */
void oracle_overlap(int64_t N, int S, int R, int a, int b, const uint8_t *sigma, int64_t *Q)
{
    for (int s = 0; s < S; s++) {
        const uint8_t *sa = sigma + ((int64_t)s * R + a) * N;
        const uint8_t *sb = sigma + ((int64_t)s * R + b) * N;
        int64_t q = 0;
        for (int64_t i = 0; i < N; i++) q += spin(sa[i]) * spin(sb[i]);
        Q[s] = q;
    }
}

/* ------------------------------------------------------------------ */
/* Four-point correlation (Sec. 3): with the overlap field               */
/* q_x = s^a_x s^b_x of two replicas, the lattice sums                   */
/*   G_mu(r) = sum over pairs a < b of sum_x q_x q_{x + r e_mu}          */
/* for r = 0 .. L_mu/2 along each axis mu (periodic).  C4(r) is their    */
/* mean over the three axes divided by N * R(R-1)/2, so C4(0) = 1.       */
/* G[s][mu][r] is written for r <= L_mu/2, the rest of the row (up to    */
/* rmax + 1 entries) is set to 0.                                        */
/* ------------------------------------------------------------------ */
void oracle_c4_sums(int Lx, int Ly, int Lz, int S, int R, const uint8_t *sigma, int rmax, int64_t *G)
{
    geom g = mk(Lx, Ly, Lz);
    int side[3] = {Lx, Ly, Lz};
    for (int s = 0; s < S; s++)
        for (int mu = 0; mu < 3; mu++)
            for (int r = 0; r <= rmax; r++) {
                int64_t tot = 0;
                if (r <= side[mu] / 2)
                    for (int a = 0; a < R; a++)
                        for (int b = a + 1; b < R; b++) {
                            const uint8_t *sa = sigma + ((int64_t)s * R + a) * g.N;
                            const uint8_t *sb = sigma + ((int64_t)s * R + b) * g.N;
#pragma omp parallel for reduction(+ : tot) schedule(static)
                            for (int64_t i = 0; i < g.N; i++) {
                                int x, y, z;
                                coords(&g, i, &x, &y, &z);
                                int64_t j = site(&g, x + (mu == 0) * r, y + (mu == 1) * r, z + (mu == 2) * r);
                                tot += spin(sa[i]) * spin(sb[i]) * spin(sa[j]) * spin(sb[j]);
                            }
                        }
                G[((int64_t)s * 3 + mu) * (rmax + 1) + r] = tot;
            }
}

/* Coherence lengths (Sec. 3, eq. xi-def): I_n = sum_r r^n C4(r), the   */
/* integral over r >= 0 taken as the sum over the lattice distances     */
/* r = 0 .. rmax (rmax = half the smallest side: C4 of a periodic        */
/* lattice is symmetric about it); xi12 = I2 / I1, xi23 = I3 / I2.  C4   */
/* is given as C4[r], r = 0..rmax.  Returns -1 unless I1 and I2 > 0.     */
int oracle_xi_from_c4(const double *C4, int rmax, double *xi12, double *xi23)
{
    double I[4] = {0, 0, 0, 0};
    for (int r = 0; r <= rmax; r++) {
        double p = 1.0;
        for (int n = 0; n < 4; n++) {
            I[n] += p * C4[r];
            p *= (double)r;
        }
    }
    if (!(I[1] > 0.0) || !(I[2] > 0.0)) return -1;
    *xi12 = I[2] / I[1];
    *xi23 = I[3] / I[2];
    return 0;
}

/* ------------------------------------------------------------------ */
/* Schedule (Sec. 2.7, Sec. 2.8): when the daemons are refreshed and at */
/* which temperature.                                                  */
/*   period P >= 1 : refresh before sweep k iff k mod P == 0           */
/*   period P == 0 : logarithmic schedule of the procedure in Sec.     */
/*                   2.8.1 (refresh, 2^s steps, refresh, ...), i.e.    */
/*                   before sweep k iff k + 1 is a power of two        */
/* Temperature of refresh rho: CONST T0; LINEAR T0 -> T1 over the      */
/* refreshes that fall in [0, n_sweeps); TABLE table[rho].             */
/* ------------------------------------------------------------------ */
enum { SCHED_CONST = 0, SCHED_LINEAR = 1, SCHED_TABLE = 2 };

int oracle_is_refresh(int64_t k, int P)
{
    if (P >= 1) return k % P == 0;
    return ((k + 1) & k) == 0;
}

int64_t oracle_refresh_index(int64_t k, int P)
{
    if (P >= 1) return k / P;
    int64_t rho = -1;
    for (int64_t t = k + 1; t > 0; t >>= 1) rho++;
    return rho;
}

int64_t oracle_refresh_count(int64_t n_sweeps, int P)
{
    if (n_sweeps <= 0) return 0;
    return oracle_refresh_index(n_sweeps - 1, P) + 1;
}

double oracle_temperature(int kind, double T0, double T1, int64_t n_sweeps, int P,
                          const double *table, int64_t table_len, int64_t rho)
{
    if (kind == SCHED_CONST) return T0;
    if (kind == SCHED_LINEAR) {
        int64_t Rtot = oracle_refresh_count(n_sweeps, P);
        if (Rtot <= 1) return T0;
        double f = (double)rho / (double)(Rtot - 1);
        return T0 * (1.0 - f) + T1 * f;
    }
    if (kind == SCHED_TABLE && rho >= 0 && rho < table_len) return table[rho];
    return NAN;
}

/* ------------------------------------------------------------------ */
/* Driver: sweeps k0 .. k0+n-1 of one algorithm on the state in place. */
/* A sweep is the even half followed by the odd half (Sec. 2.8).  For  */
/* MicSA (daemons or, with ALGO_WALKERS, one forward-X walker per     */
/* site) the auxiliary variables are refreshed before sweep k when k   */
/* is a refresh point; the heat bath and Metropolis use the temperature*/
/* of the last refresh point at or before k.  After every `stride`     */
/* sweeps the from-scratch H^EA and H^aux of every lattice are logged. */
/* dE accumulates the tally.                                           */
/* ------------------------------------------------------------------ */
enum { ALGO_MICSA = 0, ALGO_HEATBATH = 1, ALGO_WALKERS = 2, ALGO_METROPOLIS = 3 };

/* Wandering direction of walker family a (Sec. 2.8): forward X, Y, Z, */
/* then backward X, Y, Z (direction codes as in oracle_wander).        */
static const int walker_dir[6] = {0, 2, 4, 1, 3, 5};

/* With gamma daemons or walkers per site (Sec. 2.8), a timestep is     */
/* gamma sweeps: sweep k is sweep a = k mod gamma of timestep           */
/* t = k / gamma and uses family a.  Refresh points and temperatures    */
/* are those of timestep t (a refresh happens before the first sweep of */
/* the timestep and redraws every family); the schedule's length counts */
/* sweeps, its refreshes the timesteps that start in it.  Walkers       */
/* wander once per timestep, after its last sweep, each family along    */
/* its own direction, the parity of t choosing the half of the cycle.   */
int oracle_run(int Lx, int Ly, int Lz, int S, int R, int gamma, uint64_t seed, int algo, int kind,
               double T0, double T1, int64_t n_sweeps, int P, const double *table, int64_t table_len,
               int64_t k0, int64_t n, int64_t stride, const uint8_t *J, uint8_t *sigma, uint8_t *m,
               int64_t *dE, int64_t *E_log, int64_t *D_log)
{
    int64_t N = (int64_t)Lx * Ly * Lz;
    int L = S * R;
    int64_t row = 0;
    if (gamma < 1 || gamma > 6) return -1;
    int64_t n_steps = (n_sweeps + gamma - 1) / gamma;
    for (int64_t k = k0; k < k0 + n; k++) {
        int64_t t = k / gamma;
        int a = (int)(k % gamma);
        int64_t rho = oracle_refresh_index(t, P);
        double T = oracle_temperature(kind, T0, T1, n_steps, P, table, table_len, rho);
        if (!(T > 0.0) || isinf(T)) return -1;
        if (algo == ALGO_MICSA || algo == ALGO_WALKERS) {
            if (a == 0 && oracle_is_refresh(t, P)) oracle_refresh(Lx, Ly, Lz, S, R, gamma, seed, rho, T, m);
            oracle_micsa_half(Lx, Ly, Lz, S, R, gamma, a, 0, J, sigma, m, dE);
            oracle_micsa_half(Lx, Ly, Lz, S, R, gamma, a, 1, J, sigma, m, dE);
            if (algo == ALGO_WALKERS && a == gamma - 1)
                for (int f = 0; f < gamma; f++)
                    oracle_wander(Lx, Ly, Lz, S, R, gamma, f, walker_dir[f], (int)(t & 1), m);
        } else if (algo == ALGO_HEATBATH) {
            oracle_heatbath_half(Lx, Ly, Lz, S, R, seed, k, 0, T, J, sigma, dE);
            oracle_heatbath_half(Lx, Ly, Lz, S, R, seed, k, 1, T, J, sigma, dE);
        } else if (algo == ALGO_METROPOLIS) {
            oracle_metropolis_half(Lx, Ly, Lz, S, R, seed, k, 0, T, J, sigma, dE);
            oracle_metropolis_half(Lx, Ly, Lz, S, R, seed, k, 1, T, J, sigma, dE);
        } else {
            return -1;
        }
        if (stride > 0 && (k - k0 + 1) % stride == 0) {
            if (E_log) oracle_energy(Lx, Ly, Lz, S, R, J, sigma, E_log + row * L);
            if (D_log) oracle_daemon_energy(N * gamma, L, m, D_log + row * L);
            row++;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Brute force: density of states g(H) of one sample by enumerating   */
/* all 2^N spin configurations (N <= 32), walking them in Gray-code   */
/* order so that consecutive states differ by one spin and H changes  */
/* by that spin's dH.  g has 3N+1 entries indexed by (H + 3N) / 2.    */
/* ------------------------------------------------------------------ */
int oracle_density_of_states(int Lx, int Ly, int Lz, const uint8_t *J, uint64_t *g)
{
    geom gm = mk(Lx, Ly, Lz);
    int N = (int)gm.N;
    if (N > 32 || N < 1) return -1;
    memset(g, 0, sizeof(uint64_t) * (size_t)(3 * N + 1));
    int split = N > 12 ? 8 : 0; /* top `split` bits are enumerated in parallel */
    int64_t chunks = (int64_t)1 << split;
    int low = N - split;
#pragma omp parallel
    {
        uint64_t *gl = calloc((size_t)(3 * N + 1), sizeof(uint64_t));
        uint8_t sig[32];
#pragma omp for schedule(dynamic)
        for (int64_t c = 0; c < chunks; c++) {
            for (int b = 0; b < N; b++) sig[b] = 0;
            for (int b = 0; b < split; b++) sig[low + b] = (uint8_t)((c >> b) & 1);
            int64_t H = 0;
            int64_t Ei[1];
            oracle_energy(Lx, Ly, Lz, 1, 1, J, sig, Ei);
            H = Ei[0];
            gl[(H + 3 * N) / 2]++;
            uint64_t nstates = (uint64_t)1 << low;
            for (uint64_t t = 1; t < nstates; t++) {
                int b = __builtin_ctzll(t); /* Gray code: flip bit b */
                int dH = 2 * spin(sig[b]) * local_field(&gm, J, sig, b);
                sig[b] ^= 1u;
                H += dH;
                gl[(H + 3 * N) / 2]++;
            }
        }
#pragma omp critical
        for (int e = 0; e <= 3 * N; e++) g[e] += gl[e];
        free(gl);
    }
    return 0;
}

/* ================================================================== */
/* Equilibrium workload of App. C: Gaussian couplings, continuous      */
/* walkers, parallel tempering with Houdayer cluster moves.            */
/*                                                                     */
/* Energy mesh.  The paper allows continuous walkers or walkers on a   */
/* fine energy mesh (Sec. 2.3).  Here every energy is an integer       */
/* multiple of eps = 2^-17: a coupling J is held as Jq = nearest       */
/* integer to J * 2^17 (ties to even), |J| <= 8, so H, dH and the      */
/* walkers are integers and the move is exact integer arithmetic.      */
/*   H = - sum over bonds Jq s_x s_y,   dH_x = 2 s_x sum_y Jq_xy s_y     */
/* Couplings are stored per site and axis: Jq[mu][i] is the bond       */
/* (i, i + e_mu).                                                      */
/*                                                                     */
/* Exponential on the mesh.  A walker refreshed at inverse temperature */
/* beta is exponentially distributed (Sec. 2.3); on the mesh this is   */
/* the geometric law P(n) = (1 - q) q^n, q = exp(-beta eps).  Its      */
/* base-256 digits c_0..c_3 (n = sum c_d 256^d) are independent, c_d   */
/* geometric with ratio r_d = q^(256^d), truncated to 0..255 for       */
/* d < 3; the top digit is untruncated and is required to stay below   */
/* 255 with probability 1 - 2^-32.  Each digit is an inverse CDF on    */
/* one 32-bit word w_d of a Philox output:                              */
/*   c_d = #{v in 0..254 : w_d >= t_d[v]},  t_d[v] = floor(2^32 F_d(v)) */
/*   F_d(v) = P(c_d <= v) = (1 - r_d^(v+1)) / (1 - r_d^256)  (d < 3)    */
/*   F_3(v) = 1 - r_3^(v+1)                                            */
/* The same law with rate beta drives the walkers; with a fresh draw   */
/* per attempt, accepting iff n >= dH is the Metropolis rule (Sec.     */
/* 2.3: a fresh walker per flip attempt is textbook Metropolis), and   */
/* with rate beta_t - beta_{t+1} it decides tempering swaps.           */
/*                                                                     */
/* Random numbers (Philox4x32-10, same key as above), per run u:       */
/*   spins      ctr = (i>>2, t,     rep,      10<<24 | u)  out[i&3] >> 31 */
/*   walkers    ctr = (i,    e,     2t + rep,  6<<24 | u)  w = out        */
/*   Metropolis ctr = (i,    e*S+s, 2t + rep,  7<<24 | u)  w = out        */
/*   Houdayer   ctr = (t,    e,     0,         8<<24 | u)  out[0]         */
/*   swap       ctr = (t,    e,     rep,       9<<24 | u)  w = out        */
/* (t = temperature index, rep = replica 0/1, e = EMCS index, s = sweep */
/* within the EMCS).                                                    */
/*                                                                     */
/* One EMCS (App. C), for every run:                                    */
/*  1. every (temperature t, replica): walkers drawn at beta_t, then S  */
/*     times a full sweep (even sites, odd sites) followed by a forward- */
/*     X wandering of the sites of parity s & 1.  The Creutz move is    */
/*     uncapped (App. C): flip iff n - dH >= 0, then n -= dH.  With the */
/*     Metropolis update instead, each visit draws a fresh n.           */
/*  2. Houdayer move at every temperature between the two replicas.     */
/*  3. one tempering step per replica: pairs (t, t+1) with t even, then */
/*     with t odd; configurations are exchanged iff n >= E_{t+1} - E_t,  */
/*     n drawn at rate beta_t - beta_{t+1}, i.e. with probability       */
/*     min(1, exp((beta_t - beta_{t+1}) (E_t - E_{t+1}))).             */
/* Temperatures are strictly increasing in t.                           */
/* Storage: sigma[u][rep][t][i], the configuration at temperature t.    */
/* ================================================================== */
enum { STREAM_PT_WALKER = 6, STREAM_PT_METROPOLIS = 7, STREAM_PT_HOUDAYER = 8, STREAM_PT_SWAP = 9,
       STREAM_PT_SPIN = 10 };
enum { PT_WALKERS = 0, PT_METROPOLIS = 1 };
#define PT_TABLE 1020 /* 4 digits x 255 thresholds */

int oracle_pt_quantise(int64_t n, const double *J, int32_t *Jq)
{
    for (int64_t k = 0; k < n; k++) {
        if (!(fabs(J[k]) <= 8.0)) return -1;
        Jq[k] = (int32_t)nearbyint(J[k] * 131072.0);
    }
    return 0;
}

/* Thresholds of the four digits for rate lam (per unit energy); returns
   0, or -1 if the top digit could reach 255. */
int oracle_pt_exp_table(double lam, uint64_t *t)
{
    for (int d = 0; d < 4; d++) {
        double a = -lam * ldexp(1.0, 8 * d - 17); /* log r_d */
        for (int v = 0; v < 255; v++) {
            double F = d < 3 ? expm1(a * (double)(v + 1)) / expm1(a * 256.0) : -expm1(a * (double)(v + 1));
            t[d * 255 + v] = (uint64_t)floor(F * 4294967296.0);
        }
    }
    return t[3 * 255 + 254] == 4294967296ull ? 0 : -1;
}

int64_t oracle_pt_exp_draw(const uint64_t *t, const uint32_t w[4])
{
    int64_t n = 0;
    for (int d = 3; d >= 0; d--) {
        int c = 0;
        for (int v = 0; v < 255; v++) c += (uint64_t)w[d] >= t[d * 255 + v];
        n = n * 256 + c;
    }
    return n;
}

static void philox_words(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t w[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, w);
}

/* dH of flipping site i: 2 s_i times the local field of the six bonds. */
int64_t oracle_pt_delta(int Lx, int Ly, int Lz, const int32_t *Jq, const uint8_t *sig, int64_t i)
{
    geom g = mk(Lx, Ly, Lz);
    int x, y, z;
    coords(&g, i, &x, &y, &z);
    int64_t fwd[3] = {site(&g, x + 1, y, z), site(&g, x, y + 1, z), site(&g, x, y, z + 1)};
    int64_t bwd[3] = {site(&g, x - 1, y, z), site(&g, x, y - 1, z), site(&g, x, y, z - 1)};
    int64_t h = 0;
    for (int mu = 0; mu < 3; mu++) {
        h += (int64_t)Jq[mu * g.N + i] * spin(sig[fwd[mu]]);
        h += (int64_t)Jq[mu * g.N + bwd[mu]] * spin(sig[bwd[mu]]);
    }
    return 2 * spin(sig[i]) * h;
}

int64_t oracle_pt_energy(int Lx, int Ly, int Lz, const int32_t *Jq, const uint8_t *sig)
{
    geom g = mk(Lx, Ly, Lz);
    int64_t H = 0;
    for (int64_t i = 0; i < g.N; i++) {
        int x, y, z;
        coords(&g, i, &x, &y, &z);
        int64_t fwd[3] = {site(&g, x + 1, y, z), site(&g, x, y + 1, z), site(&g, x, y, z + 1)};
        for (int mu = 0; mu < 3; mu++) H -= (int64_t)Jq[mu * g.N + i] * spin(sig[i]) * spin(sig[fwd[mu]]);
    }
    return H;
}

void oracle_pt_init_spins(int Lx, int Ly, int Lz, int runs, int M, uint64_t seed, uint8_t *sigma)
{
    geom g = mk(Lx, Ly, Lz);
    for (int u = 0; u < runs; u++)
        for (int rep = 0; rep < 2; rep++)
            for (int t = 0; t < M; t++)
                for (int64_t i = 0; i < g.N; i++)
                    sigma[(((int64_t)u * 2 + rep) * M + t) * g.N + i] =
                        (uint8_t)(draw(seed, (uint32_t)(i >> 2), (uint32_t)t, (uint32_t)rep,
                                       (uint32_t)(STREAM_PT_SPIN << 24) | (uint32_t)u, (int)(i & 3)) >> 31);
}

void oracle_pt_walker_refresh(int Lx, int Ly, int Lz, uint64_t seed, int run, int rep, int t, int64_t e,
                              const uint64_t *table, int64_t *n)
{
    geom g = mk(Lx, Ly, Lz);
    for (int64_t i = 0; i < g.N; i++) {
        uint32_t w[4];
        philox_words(seed, (uint32_t)i, (uint32_t)e, (uint32_t)(2 * t + rep),
                     (uint32_t)(STREAM_PT_WALKER << 24) | (uint32_t)run, w);
        n[i] = oracle_pt_exp_draw(table, w);
    }
}

/* Creutz move on every site of one parity (Sec. 2.3, uncapped); returns
   the summed dH of the accepted flips. */
int64_t oracle_pt_creutz_half(int Lx, int Ly, int Lz, const int32_t *Jq, int parity, uint8_t *sig, int64_t *n)
{
    geom g = mk(Lx, Ly, Lz);
    int64_t acc = 0;
    for (int64_t i = 0; i < g.N; i++) {
        if (parity_of(&g, i) != parity) continue;
        int64_t dH = oracle_pt_delta(Lx, Ly, Lz, Jq, sig, i);
        if (n[i] - dH >= 0) {
            sig[i] ^= 1u;
            n[i] -= dH;
            acc += dH;
        }
    }
    return acc;
}

/* Forward-X wandering (Sec. 2.6): the walker of each site of the given
   parity is exchanged with the walker of its +x neighbour. */
void oracle_pt_wander_x(int Lx, int Ly, int Lz, int parity, int64_t *n)
{
    geom g = mk(Lx, Ly, Lz);
    for (int64_t i = 0; i < g.N; i++) {
        if (parity_of(&g, i) != parity) continue;
        int x, y, z;
        coords(&g, i, &x, &y, &z);
        int64_t j = site(&g, x + 1, y, z);
        int64_t tmp = n[i];
        n[i] = n[j];
        n[j] = tmp;
    }
}

int64_t oracle_pt_metropolis_half(int Lx, int Ly, int Lz, const int32_t *Jq, uint64_t seed, int run, int rep,
                                  int t, int64_t k, int parity, const uint64_t *table, uint8_t *sig)
{
    geom g = mk(Lx, Ly, Lz);
    int64_t acc = 0;
    for (int64_t i = 0; i < g.N; i++) {
        if (parity_of(&g, i) != parity) continue;
        uint32_t w[4];
        philox_words(seed, (uint32_t)i, (uint32_t)k, (uint32_t)(2 * t + rep),
                     (uint32_t)(STREAM_PT_METROPOLIS << 24) | (uint32_t)run, w);
        int64_t dH = oracle_pt_delta(Lx, Ly, Lz, Jq, sig, i);
        if (oracle_pt_exp_draw(table, w) >= dH) {
            sig[i] ^= 1u;
            acc += dH;
        }
    }
    return acc;
}

/* Houdayer move: the sites where the replicas differ form a graph with
   the lattice bonds; the connected component of one of them, picked
   uniformly (the k-th in site order, k = floor(u * count / 2^32)), is
   flipped in both replicas.  Returns the cluster size (0: replicas equal). */
int64_t oracle_pt_houdayer(int Lx, int Ly, int Lz, uint32_t u, uint8_t *sa, uint8_t *sb)
{
    geom g = mk(Lx, Ly, Lz);
    int64_t count = 0;
    for (int64_t i = 0; i < g.N; i++) count += sa[i] != sb[i];
    if (count == 0) return 0;
    int64_t k = (int64_t)(((uint64_t)u * (uint64_t)count) >> 32);
    int64_t root = -1;
    for (int64_t i = 0, c = 0; i < g.N; i++)
        if (sa[i] != sb[i] && c++ == k) {
            root = i;
            break;
        }
    int64_t *queue = malloc(sizeof(int64_t) * (size_t)count);
    uint8_t *seen = calloc((size_t)g.N, 1);
    int64_t head = 0, tail = 0;
    queue[tail++] = root;
    seen[root] = 1;
    while (head < tail) {
        int64_t i = queue[head++];
        int x, y, z;
        coords(&g, i, &x, &y, &z);
        int64_t nb[6] = {site(&g, x + 1, y, z), site(&g, x - 1, y, z), site(&g, x, y + 1, z),
                         site(&g, x, y - 1, z), site(&g, x, y, z + 1), site(&g, x, y, z - 1)};
        for (int d = 0; d < 6; d++)
            if (!seen[nb[d]] && sa[nb[d]] != sb[nb[d]]) {
                seen[nb[d]] = 1;
                queue[tail++] = nb[d];
            }
    }
    for (int64_t q = 0; q < tail; q++) {
        sa[queue[q]] ^= 1u;
        sb[queue[q]] ^= 1u;
    }
    free(queue);
    free(seen);
    return tail;
}

/* Tempering step of one replica group: sig[t] is the configuration at
   temperature t; pair_tables[t] has rate beta_t - beta_{t+1}.  swaps[t]
   (may be NULL) counts accepted exchanges of pair t. */
void oracle_pt_swap_step(int Lx, int Ly, int Lz, const int32_t *Jq, int M, uint64_t seed, int run, int rep,
                         int64_t e, const uint64_t *pair_tables, uint8_t *sig, int64_t *swaps)
{
    geom g = mk(Lx, Ly, Lz);
    uint8_t *tmp = malloc((size_t)g.N);
    for (int ph = 0; ph < 2; ph++)
        for (int t = ph; t + 1 < M; t += 2) {
            uint8_t *a = sig + (int64_t)t * g.N, *b = sig + (int64_t)(t + 1) * g.N;
            int64_t x = oracle_pt_energy(Lx, Ly, Lz, Jq, a) - oracle_pt_energy(Lx, Ly, Lz, Jq, b);
            uint32_t w[4];
            philox_words(seed, (uint32_t)t, (uint32_t)e, (uint32_t)rep, (uint32_t)(STREAM_PT_SWAP << 24) | (uint32_t)run,
                         w);
            if (oracle_pt_exp_draw(pair_tables + (int64_t)t * PT_TABLE, w) >= -x) {
                memcpy(tmp, a, (size_t)g.N);
                memcpy(a, b, (size_t)g.N);
                memcpy(b, tmp, (size_t)g.N);
                if (swaps) swaps[t]++;
            }
        }
    free(tmp);
}

/* Tables of a temperature ladder: walker_tables[t] at rate beta_t,
   pair_tables[t] at rate beta_t - beta_{t+1}.  Returns -1 if T is not
   strictly increasing and positive, or a table's top digit could reach 255. */
int oracle_pt_tables(int M, const double *T, uint64_t *walker_tables, uint64_t *pair_tables)
{
    for (int t = 0; t < M; t++) {
        if (!(T[t] > 0.0) || (t > 0 && !(T[t] > T[t - 1]))) return -1;
        if (oracle_pt_exp_table(1.0 / T[t], walker_tables + (int64_t)t * PT_TABLE)) return -1;
    }
    for (int t = 0; t + 1 < M; t++)
        if (oracle_pt_exp_table(1.0 / T[t] - 1.0 / T[t + 1], pair_tables + (int64_t)t * PT_TABLE)) return -1;
    return 0;
}

/* n_emcs EMCS starting at index e0 on sigma[runs][2][M][N]; S sweeps per
   EMCS.  swaps (may be NULL) is [runs][2][M-1]. */
int oracle_pt_run(int Lx, int Ly, int Lz, int runs, int M, int S, int algo, int houdayer, uint64_t seed,
                  const int32_t *Jq, const double *T, int64_t e0, int64_t n_emcs, uint8_t *sigma, int64_t *swaps)
{
    geom g = mk(Lx, Ly, Lz);
    uint64_t *wt = malloc(sizeof(uint64_t) * PT_TABLE * (size_t)M);
    uint64_t *pt = malloc(sizeof(uint64_t) * PT_TABLE * (size_t)(M > 1 ? M - 1 : 1));
    if (oracle_pt_tables(M, T, wt, pt)) {
        free(wt);
        free(pt);
        return -1;
    }
    for (int64_t e = e0; e < e0 + n_emcs; e++) {
        /* 1. fixed-temperature moves, every lattice on its own */
#pragma omp parallel for schedule(dynamic)
        for (int64_t l = 0; l < (int64_t)runs * 2 * M; l++) {
            int u = (int)(l / (2 * M)), rep = (int)((l / M) % 2), t = (int)(l % M);
            uint8_t *sig = sigma + l * g.N;
            if (algo == PT_WALKERS) {
                int64_t *n = malloc(sizeof(int64_t) * (size_t)g.N);
                oracle_pt_walker_refresh(Lx, Ly, Lz, seed, u, rep, t, e, wt + (int64_t)t * PT_TABLE, n);
                for (int s = 0; s < S; s++) {
                    oracle_pt_creutz_half(Lx, Ly, Lz, Jq, 0, sig, n);
                    oracle_pt_creutz_half(Lx, Ly, Lz, Jq, 1, sig, n);
                    oracle_pt_wander_x(Lx, Ly, Lz, s & 1, n);
                }
                free(n);
            } else {
                for (int s = 0; s < S; s++)
                    for (int p = 0; p < 2; p++)
                        oracle_pt_metropolis_half(Lx, Ly, Lz, Jq, seed, u, rep, t, e * S + s, p,
                                                  wt + (int64_t)t * PT_TABLE, sig);
            }
        }
        for (int u = 0; u < runs; u++) {
            /* 2. Houdayer move at every temperature */
            if (houdayer)
                for (int t = 0; t < M; t++)
                    oracle_pt_houdayer(Lx, Ly, Lz,
                                       draw(seed, (uint32_t)t, (uint32_t)e, 0u,
                                            (uint32_t)(STREAM_PT_HOUDAYER << 24) | (uint32_t)u, 0),
                                       sigma + (((int64_t)u * 2 + 0) * M + t) * g.N,
                                       sigma + (((int64_t)u * 2 + 1) * M + t) * g.N);
            /* 3. tempering in each replica group */
            for (int rep = 0; rep < 2; rep++)
                oracle_pt_swap_step(Lx, Ly, Lz, Jq, M, seed, u, rep, e, pt,
                                    sigma + ((int64_t)u * 2 + rep) * M * g.N,
                                    swaps ? swaps + ((int64_t)u * 2 + rep) * (M - 1) : NULL);
        }
    }
    free(wt);
    free(pt);
    return 0;
}

int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
