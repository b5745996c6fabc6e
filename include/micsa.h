/*
 * micsa.h -- C ABI of libmicsa, microcanonical simulated annealing (MicSA)
 * for the 3D Edwards-Anderson +-J spin glass on AMD Instinct MI355X (gfx950).
 *
 * Method: Bernaschi et al., "Microcanonical simulated annealing: massively
 * parallel Monte Carlo simulations with sporadic random-number generation",
 * arXiv 2506.16240.  Section numbers below refer to that paper.
 *
 * Model (Sec. 2.1, eq. Hamiltonian): N = Lx*Ly*Lz Ising spins s = +-1 on a
 * periodic cubic lattice, H = -sum_<xy> J_xy s_x s_y with J = +-1 drawn with
 * probability 1/2 per bond.  Each site carries one daemon n = 4m, m in 0..3
 * (Sec. 2.4-2.5).  A MicSA sweep updates the even sublattice, then the odd
 * one (Sec. 2.8); a site flips iff 0 <= n - dH <= 12 (eq. flip-OK) and its
 * daemon absorbs the change (eq. Creutz).  Daemons are redrawn from eq.
 * prob-daemons-walkers only at refresh points (Sec. 2.7).  A heat-bath
 * sweep (Sec. 2.1) is provided as the random-number-greedy baseline.
 *
 * Conventions shared by every entry point
 *  - Every call returns an int status (enum micsa_status); no call aborts,
 *    throws or exits.  After a failure micsa_last_error() describes it.
 *  - Host arrays passed in are owned by the caller and only read or written
 *    during the call.  Device memory is owned by the context.
 *  - Site index in all host arrays: i = x + Lx*(y + Ly*z); lattice index
 *    l = sample*R + replica.  Spin bit sigma (s = 1 - 2 sigma); daemon level
 *    m (n = 4m); coupling bits j (J = 1 - 2j) of the forward bonds
 *    (i, i+e_x), (i, i+e_y), (i, i+e_z) in bits 0, 1, 2.
 *  - Random numbers are Philox4x32-10 keyed by the 64-bit seed with one
 *    counter per (stream, sample, replica, site, time); results are
 *    therefore independent of launch shapes, layouts and device count.
 *  - A context is not thread-safe.  Distinct contexts may run concurrently.
 */
#ifndef MICSA_H
#define MICSA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum micsa_status {
    MICSA_OK = 0,
    MICSA_EINVAL = -1, /* invalid argument; nothing was changed */
    MICSA_ENOMEM = -2, /* device allocation failed; nothing was changed */
    MICSA_EHIP = -3,   /* a HIP runtime call failed; the context must be destroyed */
    MICSA_ESTATE = -4, /* call not allowed in the current state (e.g. no schedule) */
    MICSA_ERANGE = -5  /* sweep index outside the schedule */
};

enum micsa_layout {
    MICSA_LAYOUT_BYTE = 0,    /* one byte per spin and per daemon; an even site's spin byte also
                                 holds the coupling bits of its six bonds */
    MICSA_LAYOUT_BITPLANE = 1 /* multispin coding: 64 lattices per 64-bit word (Sec. 2.5, App. B), the
                                 lanes set by micsa_params.lane_mode; one launch per sweep with both
                                 halves, ring planes recomputed, per-lane energy tally */
};

/* Bit-plane layout (multispin coding across lattices, Sec. 2.5 and App. B:
   the 64 bits of a word are the same site of 64 lattices). */
enum micsa_lane_mode {
    MICSA_LANES_SAMPLES = 0, /* bit l of lane group g is sample 64g + l; each replica has its own words,
                                and the coupling words of a group serve all its replicas */
    MICSA_LANES_REPLICAS = 1 /* bit l of lane group g is replica 64g + l of one sample; the couplings
                                of the sample are broadcast to every bit (0 or ~0 words) */
};

enum micsa_algo {
    MICSA_ALGO_MICSA = 0,    /* daemon update, Sec. 2.3-2.8 (gamma daemons per site) */
    MICSA_ALGO_HEATBATH = 1, /* canonical heat bath, Sec. 2.1 */
    MICSA_ALGO_WALKERS = 2,  /* gamma walkers per site with wandering (Sec. 2.6, 2.8): after the
                                last sweep of timestep t, walker family a of every site of
                                parity t mod 2 is exchanged with that of its neighbour along
                                +x, +y, +z, -x, -y, -z for a = 0..5 (byte layout) */
    MICSA_ALGO_METROPOLIS = 3 /* canonical Metropolis, the comparison of Sec. 4 (Table 3): the flip is
                                 accepted with probability min(1, exp(-beta dH)) (byte layout) */
};

enum micsa_sched_kind {
    MICSA_SCHED_CONST = 0,  /* T = T0 at every refresh */
    MICSA_SCHED_LINEAR = 1, /* T0 at the first refresh, T1 at the last one in [0, n_sweeps) */
    MICSA_SCHED_TABLE = 2   /* T = T_table[rho] at refresh rho */
};

/* refresh_period value selecting the logarithmic refresh schedule of the
   procedure in Sec. 2.8.1: refresh before sweep k iff k + 1 is a power of two. */
#define MICSA_REFRESH_LOG2 0

typedef struct micsa_params {
    int32_t Lx, Ly, Lz;    /* lattice sides: even, Lx % 8 == 0, Lx >= 8, Ly, Lz >= 2 */
    int32_t n_samples;     /* coupling realisations, 1 .. 2^24 - 1 */
    int32_t n_replicas;    /* replicas per sample sharing the couplings (Sec. 3), >= 1 */
    int32_t layout;        /* enum micsa_layout */
    int32_t gamma;         /* daemons (or walkers) per site, 1..6 (0 means 1); > 1 needs the byte
                              layout.  A timestep is gamma sweeps; sweep k is sweep a = k mod gamma of
                              timestep k / gamma and uses family a (Sec. 2.8).  Refresh points and
                              refresh temperatures are counted in timesteps; a refresh redraws
                              every family, daemon a of site i as number a*N + i of the daemon
                              stream.  n_sweeps of the schedule still counts sweeps. */
    int32_t lane_mode;     /* enum micsa_lane_mode: what the 64 bits of a bit-plane word hold
                              (BYTE layout: LANES_SAMPLES only) */
    uint64_t seed;         /* Philox key */
} micsa_params;

typedef struct micsa_schedule {
    int32_t kind;           /* enum micsa_sched_kind */
    int32_t refresh_period; /* >= 1: refresh before sweep k iff k % period == 0; or MICSA_REFRESH_LOG2 */
    double T0, T1;          /* temperatures (> 0, finite) */
    int64_t n_sweeps;       /* schedule length; sweeps at k >= n_sweeps fail with ERANGE */
    const double* T_table;  /* TABLE only: temperature of refresh rho, copied by the call */
    int64_t T_len;          /* TABLE only: entries in T_table */
} micsa_schedule;

typedef struct micsa_ctx micsa_ctx;

/* Static description of a status code. */
const char* micsa_status_string(int status);

/* Text of the last failure on this context ("" if none).  Valid until the
   next call on the context. */
const char* micsa_last_error(const micsa_ctx* ctx);

/* Create S x R lattices from the seed (Sec. 3: couplings +-1 with
   probability 1/2, spins drawn at infinite temperature; daemons start at
   m = 0 and are drawn at the first refresh point).  hip_stream is a
   hipStream_t (NULL = the null stream) on which every later call enqueues
   its work.  On success *out owns all device memory; on failure *out is
   NULL and nothing is leaked.  The working buffers of the sweep path the
   lattice takes by default (the multispin planes, the slab sweep's drawn
   levels) are allocated here when they fit, else by the first sweep call
   that needs them.
   Errors: EINVAL (bad sides/counts/layout/gamma), ENOMEM, EHIP. */
int micsa_create(const micsa_params* p, void* hip_stream, micsa_ctx** out);

/* Synchronise the stream and free everything.  NULL is accepted. */
int micsa_destroy(micsa_ctx* ctx);

/* Install the temperature/refresh schedule (Sec. 2.7-2.8; the annealing
   temperature applies to the daemon refresh and, for the heat bath, to the
   sweeps after that refresh point).  The table is copied.  Resets nothing
   else: the sweep counter k is kept.
   Errors: EINVAL (T <= 0 or not finite, period < 0, bad table). */
int micsa_set_schedule(micsa_ctx* ctx, const micsa_schedule* s);

/* Enqueue n sweeps of algo at sweep indices k .. k+n-1 and advance k.  For
   MICSA the daemons are refreshed before every refresh-point sweep at the
   temperature of that refresh; a sweep is the even half then the odd half.
   Asynchronous: returns once the work is enqueued.
   Errors: ESTATE (no schedule), ERANGE (k+n > n_sweeps), EINVAL. */
int micsa_sweep(micsa_ctx* ctx, int32_t algo, int64_t n);

/* As micsa_sweep, and after every `stride` sweeps records the from-scratch
   H^EA (eq. Hamiltonian) and H^aux = sum_x sum_a n_{x,a} (eq. H-total) of each
   lattice.  E_log and D_log are host arrays [n/stride][S*R] (either may be
   NULL), filled when the call returns (the call synchronises). */
int micsa_sweep_logged(micsa_ctx* ctx, int32_t algo, int64_t n, int64_t stride, int64_t* E_log,
                       int64_t* D_log);

/* As micsa_sweep_logged with the logs in device memory: E_log and D_log are
   device arrays of int64 [n/stride][S*R] (either may be NULL), written in
   stream order; the call only enqueues (it does not synchronise), so the
   logs are complete once the stream has reached this call's last sweep, as
   for a kernel the caller launched on the same stream.  The arrays stay the
   caller's and must stay allocated until then.  The library keeps one
   device row of reduction slots per context, allocated on the first call;
   on lattices swept by the resident kernel it keeps a buffer of the whole
   log that grows (after synchronising the stream) when a call logs more
   rows than any call before it.  Errors as micsa_sweep_logged. */
int micsa_sweep_logged_d(micsa_ctx* ctx, int32_t algo, int64_t n, int64_t stride, int64_t* E_log,
                         int64_t* D_log);

/* Wait for all enqueued work. */
int micsa_sync(micsa_ctx* ctx);

/* Reads (synchronous; outputs are host arrays in the natural layout above,
   independent of the device layout). */
int micsa_read_energy(micsa_ctx* ctx, int64_t* E);       /* [S*R] H^EA from scratch */
int micsa_read_energy_tally(micsa_ctx* ctx, int64_t* E); /* [S*R] H^EA from the dH of every accepted move;
                                                            bit-plane layout: kept per lane by the one-launch
                                                            sweep, ESTATE after a per-half sweep until the
                                                            spins are written */
int micsa_read_demon_energy(micsa_ctx* ctx, int64_t* D); /* [S*R] H^aux = 4 sum m */
/* Q[s] = sum_x s^a_x s^b_x, the overlap of replicas a and b (App. C); EINVAL
   unless 0 <= a, b < R and a != b. */
int micsa_read_overlap(micsa_ctx* ctx, int32_t a, int32_t b, int64_t* Q);
/* Four-point correlation of the overlap field q_x = s^a_x s^b_x (Sec. 3):
   G[s][mu][r] = sum over replica pairs a < b and sites x of q_x q_{x + r e_mu}
   (periodic), mu = x, y, z, for r = 0 .. rmax with rmax = max(Lx, Ly, Lz)/2;
   entries with r > L_mu / 2 are 0.  C4(r) is the mean of G over the three
   axes divided by N R (R - 1) / 2 (so C4(0) = 1).  Host array
   [S][3][rmax + 1]; EINVAL unless R >= 2.  Allocates and frees a device
   buffer of at most 256 MiB for the packed overlap fields. */
int micsa_read_c4(micsa_ctx* ctx, int64_t* G);
/* micsa_read_c4 without allocation, for callers that cannot allocate
   device memory (code under HIP graph capture, tight serving loops,
   harnesses that forbid hipMalloc).  Same output as micsa_read_c4.  The
   packed overlap rows and the count slots live in one static device array
   of 32 MiB per device, held until the process ends; the call allocates no
   device memory.  Limit: S*3*(rmax+1)*520 bytes (rounded up to 256 twice)
   plus one replica pair's rows, 8*Ly*Lz*floor((Lx/2 + 63)/32) bytes, must
   fit the 32 MiB (e.g. up to 512^3 with two replicas); ERANGE otherwise.
   Every call on a device shares that device's array and leaves its
   contents behind: calls that overlap in time on one device (two host
   threads, or two streams) race and may return wrong sums.  Synchronous. */
int micsa_read_c4_static(micsa_ctx* ctx, int64_t* G);

/* Coherence lengths per sample (eq. xi-def): I_n = sum_{r=0}^{rmin} r^n C4(r),
   rmin = min(Lx, Ly, Lz)/2 (the integral read as the sum over lattice
   distances up to half the side), xi12 = I2/I1, xi23 = I3/I2 (NaN if I1 or
   I2 is not positive).  Host arrays [S]; EINVAL unless R >= 2. */
int micsa_read_xi(micsa_ctx* ctx, double* xi12, double* xi23);
int micsa_read_spins(micsa_ctx* ctx, uint8_t* sigma);    /* [S][R][N] */
int micsa_read_demons(micsa_ctx* ctx, uint8_t* m);       /* [S][R][gamma][N] */
int micsa_read_couplings(micsa_ctx* ctx, uint8_t* j);    /* [S][N] forward-bond bits 0..2 */
int micsa_get_counters(micsa_ctx* ctx, int64_t* k, int64_t* rho); /* next sweep, its refresh index */

/* Thresholds the device uses for refresh rho of the installed schedule:
   t[k] = floor(2^32 P(m <= k)) from eq. prob-daemons-walkers, and the heat
   bath's tau[v] = floor(2^32 / (1 + exp(-2 beta (6 - 2v)))).  ESTATE
   without a schedule, ERANGE if rho is outside it. */
int micsa_get_thresholds(micsa_ctx* ctx, int64_t rho, uint64_t t[3]);
int micsa_get_heatbath_thresholds(micsa_ctx* ctx, int64_t rho, uint64_t tau[7]);
/* Metropolis acceptance table of refresh rho: a flip with energy change
   dH = 4q - 12 is taken iff the 32-bit uniform is below theta[q];
   theta[q] = floor(2^32 e^{-beta dH}) for dH > 0 and 2^32 for dH <= 0.  The
   uniform is Philox(h>>2, 2k+p, r, 5<<24 | s)[h & 3] for the parity-split
   index h = i >> 1 of the site, as the heat bath's with stream tag 5. */
int micsa_get_metropolis_thresholds(micsa_ctx* ctx, int64_t rho, uint64_t theta[7]);

/* Writes (synchronous).  Spins reset the energy tally to the from-scratch
   energy.  Daemon levels above 3 are rejected with EINVAL. */
int micsa_write_spins(micsa_ctx* ctx, const uint8_t* sigma); /* [S][R][N] */
int micsa_write_demons(micsa_ctx* ctx, const uint8_t* m);    /* [S][R][gamma][N] */

/* Checkpoint and resume.  micsa_save writes into the caller-owned buffer buf
   a self-contained image of everything a run depends on: the parameters,
   the sweep counter k, the installed schedule (with its table), the energy
   tally, the spins [S][R][N], the daemons [S][R][gamma][N] and the
   couplings [S][N] of every lattice, and a checksum.  Because every random
   number is a function of (seed, sample, replica, site, sweep or refresh
   index) (Sec. 2.7 refreshes at fixed points of k), a context that loads the
   image continues bit for bit as the saved one would have.  A walker
   wandering the daemons still owe is applied first.  With buf == NULL only
   *len is set (the image size, which depends on the shape and the schedule
   table); a *len below the size gives ERANGE with *len set to the size.
   Synchronous.
   micsa_load restores an image into a context created with the same
   micsa_params (the couplings, drawn from the seed, must match the
   image's).  Errors: EINVAL for another shape, seed, layout, gamma or lane
   mode, a wrong magic, version, size or checksum, or out-of-range values;
   nothing is changed then.  The image is host-endian and tied to this
   library version. */
int micsa_save(micsa_ctx* ctx, void* buf, size_t* len);
int micsa_load(micsa_ctx* ctx, const void* buf, size_t len);

/* Per-kernel timing with HIP events on the context's stream.  While
   enabled every kernel launch is bracketed by an event pair; the sums are
   read (synchronously) by micsa_get_timing.  kind: 0 = sweep kernels,
   1 = refresh, 2 = heat bath, 3 = reductions, 4 = Metropolis.  Disabled by
   default. */
int micsa_set_timing(micsa_ctx* ctx, int32_t enable);
int micsa_get_timing(micsa_ctx* ctx, int32_t kind, double* total_ms, int64_t* launches);

/* Name of the sweep kernel variant the context uses (static string). */
const char* micsa_kernel_name(const micsa_ctx* ctx, int32_t algo);

/* Launch-shape options (results never depend on them; they exist for the
   tuner and for tests that compare variants).
   MICSA_OPT_SWEEP_KERNEL: MICSA_KERNEL_AUTO (default), MICSA_KERNEL_SIMPLE
     (one launch per half sweep), MICSA_KERNEL_FUSED (one launch per sweep,
     refresh fused in; byte layout: needs Lx % 32 == 0; bit-plane layout:
     the one-launch sweep with its per-lane tally, which AUTO takes where a
     plane has at most 1024 words and which on larger planes runs in row
     tiles only on this request, the per-half kernels being faster there),
     MICSA_KERNEL_RESIDENT (whole
     lattice in LDS for many sweeps per launch; byte layout, N <= 102400),
     MICSA_KERNEL_MULTISPIN (MicSA with daemons, gamma = 1, Lx % 128 == 0:
     multispin coding, Sec. 2.5 -- a sweep call packs the state into bit
     planes of 64 sites per word, sweeps there with one launch per sweep
     (or per half sweep, MICSA_OPT_MSC_FUSED) and the refresh fused in; the
     planes stay the working state after the call and are unpacked only
     when an entry point next reads or writes the state or sweeps it on
     another path, so consecutive multispin calls pack once; walkers
     (gamma = 1) run on the one-launch form too; the heat bath and
     Metropolis keep the fused path).
   MICSA_OPT_TILE_Y / MICSA_OPT_TILE_Z: rows / planes per work-group of the
     fused and one-launch multispin sweeps (0 = automatic); TILE_Z is also
     the planes per work-group of the one-launch bit-plane sweep.  TILE_Z must
     divide Lz.  TILE_Y is at most Ly; the fused byte sweep uses it where it
     divides Ly (else the automatic choice), the multispin sweep as given,
     its last tile along y holding the rows left over (a tile wider than 256
     lanes, (tile_y + 4) * Lx / 128 > 256, runs the per-half multispin
     kernels instead).
   MICSA_OPT_XCD_MAP: tile order over the 8 XCDs, for shared L2 among
     neighbouring tiles' halo reads.  1 gives each XCD a contiguous range of
     tiles (fused and one-launch multispin sweeps; needs the tile count
     divisible by 8).  2 (default) gives each XCD a band of z tiles across
     every y tile on the multispin sweep (needs the z-tile count divisible
     by 8, else it falls back to 1), and acts as 1 on the fused byte sweeps.
     0 is the plain order.
   MICSA_OPT_GRAPHS: 1 replays the per-half paths (bit-plane layout; byte
     lattices using neither the resident nor the fused sweep) as captured
     HIP graphs of 16 sweeps; 0 (default) launches every kernel, which is
     faster for these kernels on MI355X (the graph form adds a refresh-check
     and a counter kernel to every sweep).  Per-launch timing
     (micsa_set_timing) always launches every kernel.
   MICSA_OPT_TEMPORAL: MicSA sweeps per pass over memory on the fused byte
     sweep and the slab sweep: 2 (default) runs sweeps k and k + 1 in one
     launch wherever a call
     sweeps at least two (the state is read and written once per pair); 1
     runs one sweep per launch.  Results are identical.
   MICSA_OPT_MSC_PASS: MicSA sweeps per pass on the one-launch multispin
     sweep: 2 (default: sweeps k and k + 1 in one launch, rings of 8 rows
     and planes, the state read and written once per pair; a pass whose
     sweeps include a refresh takes the levels drawn ahead, and a pair with
     two refreshes, a refresh with DRAW_AHEAD 0, the last odd sweep of a
     call, walkers, or a tile whose work-group does not fit runs one sweep
     per launch) or 1 (one sweep per launch).  Results are identical; at
     512^3 on MI355X the pair takes 36 us against 2 x 27 us.
   MICSA_OPT_MSC_FUSED: the multispin sweep in one launch per sweep marching
     along z (1, default) or one launch per half sweep (0).
   MICSA_OPT_PREFETCH: steps of global loads in flight in the fused MicSA
     sweep, 1 (default) or 2 (used for work-groups of at most 640 lanes,
     i.e. (tile_y + 4) * Lx / 32 <= 640; larger tiles run with 1).
   MICSA_OPT_DRAW_AHEAD: one-launch multispin, slab and bit-plane sweeps.  On
     two-sweep slab launches, 1 (default) has a launch without a refresh of
     its own draw the levels of the schedule's next refresh for its planes,
     kept across calls until the schedule changes, and 0 draws them inside
     the refresh launch.  Elsewhere, 1 (default for the multispin sweep;
     the bit-plane layout defaults to 0) draws
     the daemon levels of each refresh (Sec. 2.3; they depend on the refresh
     index and temperature, not on the state) in a kernel of their own on a
     second stream of the library, while the sweeps before the refresh run;
     the refresh sweep then reads them (multispin: the first refresh after
     a call is drawn during it and kept for the call that starts there,
     until the schedule changes; a refresh at a call's first sweep with no
     such levels is drawn by a full grid, beside the call's pack of the
     planes when there is one).  0 draws them in place: inside the
     refresh sweep (multispin), or in a draw kernel just before it on the
     library's stream (bit-plane).  Every draw is joined into the context's
     stream before the call that launched it returns.  Results are
     identical.
   Errors: EINVAL for an unknown option or a value the lattice cannot use. */
enum micsa_option {
    MICSA_OPT_SWEEP_KERNEL = 1,
    MICSA_OPT_TILE_Y = 2,
    MICSA_OPT_TILE_Z = 3,
    MICSA_OPT_XCD_MAP = 4,
    MICSA_OPT_GRAPHS = 5,
    MICSA_OPT_PREFETCH = 6,
    MICSA_OPT_TEMPORAL = 7,
    MICSA_OPT_MSC_FUSED = 8,
    MICSA_OPT_DRAW_AHEAD = 9,
    MICSA_OPT_MSC_PASS = 10
};
enum micsa_kernel_choice {
    MICSA_KERNEL_AUTO = 0,    /* resident if the lattice fits; else, for MicSA calls of >= 8 sweeps, multispin
                                 if Lx % 128 == 0; else fused if Lx >= 128, else simple */
    MICSA_KERNEL_SIMPLE = 1,  /* one launch per half sweep (bit-plane layout: instead of its one-launch sweep) */
    MICSA_KERNEL_FUSED = 2,   /* one launch per sweep, refresh fused in (Lx % 32 == 0) */
    MICSA_KERNEL_RESIDENT = 3, /* one work-group per lattice keeps it in LDS for many sweeps (<= 102400 sites) */
    MICSA_KERNEL_MULTISPIN = 4, /* MicSA daemon sweeps on bit planes, 64 sites of a row per word (Lx % 128 == 0) */
    MICSA_KERNEL_SLAB = 5       /* MicSA, a z plane per work-group with its neighbour planes recomputed (byte
                                   layout, gamma = 1, Ly * Lx / 8 <= 1024): two sweeps per launch while the
                                   lattices have fewer planes than the device has compute units (and two per
                                   pass are set, the default), else one; AUTO takes it for lattices too large
                                   for the resident sweep with Lx < 128 (e.g. L = 64) */
};
int micsa_set_option(micsa_ctx* ctx, int32_t option, int64_t value);

/* ------------------------------------------------------------------------
   Serving pool: continuous batching of annealing jobs.

   A job is one micsa_params (lattices from a seed) plus one schedule, run
   with MicSA to the end of its schedule.  Jobs are queued on submission and
   admitted in arrival order while their device footprint fits the pool's
   HBM budget (and fewer than max_running jobs run); an admitted job keeps
   its lattices and daemons resident until it is released.  micsa_pool_step
   enqueues the next chunk of sweeps of every running job ("batching by
   sweep") and returns without waiting for the device: the jobs whose
   lattices fit one work-group's LDS advance together in one batched launch
   on the pool's stream, each lattice at its own sweep index and
   temperature; every larger job runs its own kernels on a stream of its own
   (default priority), so jobs overlap on the device.  At most two chunks
   of a job (and two batched launches) are in flight: a call skips a job
   whose two previous chunks have not finished, so calling micsa_pool_step
   in a loop keeps the device busy while new jobs are submitted and
   admitted.  A job whose every sweep has been enqueued and has finished on
   the device is DONE; its state stays readable through
   micsa_pool_job_context until micsa_pool_release frees it.
   Results never depend on the other jobs in the pool: every random number
   is keyed by the job's own seed, sample, replica, site and time.
   ------------------------------------------------------------------------ */
typedef struct micsa_pool micsa_pool;

enum micsa_job_state { MICSA_JOB_QUEUED = 0, MICSA_JOB_RUNNING = 1, MICSA_JOB_DONE = 2, MICSA_JOB_RELEASED = 3 };

/* Device bytes a job with these parameters occupies while admitted. */
int micsa_pool_footprint(const micsa_params* p, size_t* bytes);

/* hbm_budget: bytes the pool may hold for admitted jobs; max_running >= 1.
   hip_stream as in micsa_create.  Errors: EINVAL, ENOMEM. */
int micsa_pool_create(size_t hbm_budget, int32_t max_running, void* hip_stream, micsa_pool** out);
int micsa_pool_destroy(micsa_pool* pool); /* frees every job; NULL accepted */

/* Queue a job (parameters and schedule are copied).  *job receives its id.
   EINVAL for invalid parameters or schedule, or a footprint above the whole
   budget (it could never be admitted). */
int micsa_pool_submit(micsa_pool* pool, const micsa_params* p, const micsa_schedule* s, int64_t* job);

/* Retire the jobs whose work has finished, admit what fits, enqueue up to
   `sweeps` more sweeps of every running job with a free chunk slot
   (asynchronous).  Outputs (may be NULL): number of running and queued jobs
   after the step. */
int micsa_pool_step(micsa_pool* pool, int64_t sweeps, int32_t* running, int32_t* queued);

/* Wait until every enqueued chunk of every job has finished. */
int micsa_pool_sync(micsa_pool* pool);

/* State of a job and its sweep counter (sweeps enqueued so far). */
int micsa_pool_job_state(micsa_pool* pool, int64_t job, int32_t* state, int64_t* k);

/* The context of a RUNNING or DONE job (owned by the pool; valid until
   release); read results through the micsa_read_* calls. */
int micsa_pool_job_context(micsa_pool* pool, int64_t job, micsa_ctx** ctx);

/* Free a DONE job's device memory (EINVAL for an unknown or unfinished job). */
int micsa_pool_release(micsa_pool* pool, int64_t job);

/* ------------------------------------------------------------------------
 * Equilibrium workload (App. C): parallel tempering of one sample with
 * Gaussian couplings, continuous walkers and Houdayer cluster moves.
 *
 * Energy mesh: the paper allows continuous walkers or walkers on a fine
 * energy mesh (Sec. 2.3).  Every energy here is an integer multiple of
 * 2^-17: a coupling J becomes Jq = nearest integer to J * 2^17 (ties to
 * even), and H, dH, walkers and the energies returned are in those units.
 * An exponential of rate lambda on the mesh, P(n) = (1 - q) q^n with
 * q = exp(-lambda 2^-17), is drawn as four independent base-256 digits,
 * digit d by inverse CDF on word d of one Philox output against a table
 * t_d[v] = floor(2^32 P(c_d <= v)), v = 0..254 (micsa_pt_get_tables).
 *
 * One EMCS (App. C), for every run: (1) every (temperature t, replica)
 * draws its walkers at beta_t and does `sweeps` times a full sweep (even,
 * then odd sites; uncapped Creutz move: flip iff n - dH >= 0, n -= dH)
 * followed by a forward-X wandering of the sites of parity s & 1 (Sec.
 * 2.6); with MICSA_PT_METROPOLIS each visit draws a fresh walker instead,
 * which is the Metropolis rule (Sec. 2.3); (2) a Houdayer move at every
 * temperature: the connected cluster of sites where the two replicas
 * differ that holds the k-th such site, k = floor(u * count / 2^32), is
 * flipped in both; (3) per replica group, tempering exchanges of pairs
 * (t, t+1), t even then t odd, accepted iff n >= E_{t+1} - E_t with n drawn
 * at rate beta_t - beta_{t+1}, i.e. with probability
 * min(1, exp((beta_t - beta_{t+1}) (E_t - E_{t+1}))).
 *
 * Random numbers: Philox4x32-10 keyed by the seed; per run u the counters
 *   spins (i>>2, t, replica, 10<<24|u)   walkers (i, e, 2t+replica, 6<<24|u)
 *   Metropolis (i, e*sweeps+s, 2t+replica, 7<<24|u)
 *   Houdayer (t, e, 0, 8<<24|u)          swaps (t, e, replica, 9<<24|u)
 * with e the EMCS index and s the sweep within it.
 * Arrays "by temperature" are [runs][2][M][...] with index t the
 * temperature; site i = x + Lx*(y + Ly*z).
 * ------------------------------------------------------------------------ */
typedef struct micsa_pt micsa_pt;

enum micsa_pt_algo { MICSA_PT_WALKERS = 0, MICSA_PT_METROPOLIS = 1 };

typedef struct {
    int32_t Lx, Ly, Lz; /* even, >= 2; Lx <= 64; Lx*Ly*Lz <= MICSA_PT_MAX_SITES */
    int32_t n_runs;     /* independent runs of the sample, 1 .. 2^24 - 1 */
    int32_t n_temps;    /* temperatures M per replica group, 2 .. 64 */
    int32_t sweeps;     /* sweeps per EMCS, 1 .. 64 */
    int32_t algo;       /* enum micsa_pt_algo */
    int32_t houdayer;   /* 1: a Houdayer move every EMCS; 0: none */
    uint64_t seed;
} micsa_pt_params;

#define MICSA_PT_MAX_SITES 16384

/* Create the runs of one sample.  J: host array [3][N], row mu the coupling
   of bond (i, i + e_mu), finite with |J| <= 8.  T: host array [n_temps],
   strictly increasing, positive; the walker tables need beta_t large
   enough that a walker stays below 2^30 mesh units (T up to about 350) and
   every table's top digit stays below 255.  Both arrays are copied.  The
   start is random (infinite temperature), energies are computed.  Errors:
   EINVAL (parameters, J or T), ENOMEM, EHIP; *out = NULL on error. */
int micsa_pt_create(const micsa_pt_params* p, const double* J, const double* T, void* hip_stream,
                    micsa_pt** out);
int micsa_pt_destroy(micsa_pt* pt); /* syncs, then frees; NULL accepted */
const char* micsa_pt_last_error(const micsa_pt* pt);

/* Enqueue n_emcs EMCS (asynchronous).  ERANGE once the EMCS index or
   e * sweeps would pass 2^32. */
int micsa_pt_step(micsa_pt* pt, int64_t n_emcs);
int micsa_pt_sync(micsa_pt* pt);
int micsa_pt_get_emcs(const micsa_pt* pt, int64_t* e); /* EMCS done so far */

/* Synchronous reads, by temperature.  E: [runs][2][M] energies (mesh
   units); Q: [runs][M] overlap sum_x s^a_x s^b_x of the two replicas; either
   may be NULL. */
int micsa_pt_read(micsa_pt* pt, int64_t* E, int64_t* Q);
int micsa_pt_read_spins(micsa_pt* pt, uint8_t* sigma);       /* [runs][2][M][N] spin bits */
int micsa_pt_write_spins(micsa_pt* pt, const uint8_t* sigma); /* same layout, bits 0/1; energies recomputed */
int micsa_pt_read_swaps(micsa_pt* pt, int64_t* swaps);        /* [runs][2][M-1] accepted exchanges per pair */

/* The digit thresholds in use: kind 0 = walker table of temperature index,
   kind 1 = exchange table of pair (index, index + 1); t receives [4][255]. */
int micsa_pt_get_tables(micsa_pt* pt, int32_t kind, int32_t index, uint64_t* t);
int micsa_pt_get_couplings(micsa_pt* pt, int32_t* Jq); /* [3][N] mesh units */

/* Kernel of the fixed-temperature moves.  ROWS: a work-group per (run,
   temperature), threads looping over rows, any shape.  REGISTER: several
   temperatures per work-group, one row per thread with its walkers in
   registers; needs Lx in {4, 6, 8, 10, 12, 16} and 2*Ly*Lz <= 1024 (EINVAL
   otherwise).  AUTO (default) takes REGISTER where it applies.  Results are
   identical. */
enum micsa_pt_kernel { MICSA_PT_KERNEL_AUTO = 0, MICSA_PT_KERNEL_ROWS = 1, MICSA_PT_KERNEL_REGISTER = 2 };
int micsa_pt_set_kernel(micsa_pt* pt, int32_t kernel);
const char* micsa_pt_kernel_name(const micsa_pt* pt); /* kernel the next step launches */

/* Per-kernel timing with HIP events on the stream: kind 0 = EMCS kernel,
   1 = exchange kernel. */
int micsa_pt_set_timing(micsa_pt* pt, int32_t enable);
int micsa_pt_get_timing(micsa_pt* pt, int32_t kind, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* MICSA_H */
