// libmicsa: host side of the C ABI declared in include/micsa.h.
//
// The context owns the device state of S*R lattices in the byte layout
// (geometry.hpp), the installed schedule, the sweep counter k and an energy
// tally per lattice.  Every entry point validates its arguments, enqueues
// kernels on the context's stream and reports failures as status codes.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "bitplane_kernels.hpp"
#include "bitplane_sweep.hpp"
#include "byte_slab.hpp"
#include "fused_kernels.hpp"
#include "fused2_kernels.hpp"
#include "msc_kernels.hpp"
#include "msc2_kernels.hpp"
#include "observables.hpp"
#include "resident_kernels.hpp"
#include "micsa.h"

using namespace micsa;

namespace {

constexpr int kBlock = 256;
constexpr int kTimingKinds = 5;
enum TimingKind { kTimeSweep = 0, kTimeRefresh = 1, kTimeHeatBath = 2, kTimeReduce = 3, kTimeMetropolis = 4 };
constexpr int kAlgos = 4;  // MICSA, HEATBATH, WALKERS, METROPOLIS

struct Schedule {
    bool set = false;
    int32_t kind = MICSA_SCHED_CONST;
    int32_t period = 1;
    double T0 = 1.0, T1 = 1.0;
    int64_t n_sweeps = 0;
    int64_t n_steps = 0;  // timesteps that start in [0, n_sweeps): ceil(n_sweeps / gamma)
    std::vector<double> table;
};

}  // namespace

struct micsa_ctx {
    micsa_params p{};
    hipStream_t stream = nullptr;
    int device = 0;  // the device current at creation, which holds the state
    int cus = 0;     // its compute units
    Geom g{};
    int L = 0;  // lattices = S * R
    int gamma = 1;  // daemons (walkers) per site; a timestep is gamma sweeps
    // device state (byte layout), double-buffered: the fused sweep reads the
    // current buffers and writes the alternate ones, then the two swap
    uint8_t* spin = nullptr;  // [L][2][Nh] current
    uint8_t* dem = nullptr;   // [L][2][Nh] current
    uint8_t* spin_alt = nullptr;
    // two-sweep slab launches: levels of later refreshes drawn ahead (shape of
    // dem) and the sweep index each holds the levels of (-1: none)
    uint8_t* sdr[2] = {nullptr, nullptr};
    int64_t sdr_k[2] = {-1, -1};
    uint8_t* dem_alt = nullptr;
    // bit-plane layout (MICSA_LAYOUT_BITPLANE): 64 samples per word
    bool bit = false;
    int32_t G = 0;              // lane groups
    uint64_t* bspin = nullptr;  // [G][R][2][Nh]
    uint64_t* bdm0 = nullptr;   // [G][R][2][Nh]
    uint64_t* bdm1 = nullptr;   // [G][R][2][Nh]
    uint64_t* bJ = nullptr;     // [G][6][Nh]
    // one-launch bit-plane sweep (bitplane_sweep.hpp): it writes these, then
    // they swap with the current arrays (allocated on first use)
    uint64_t *bspin_alt = nullptr, *bdm0_alt = nullptr, *bdm1_alt = nullptr;
    uint64_t *bdr0 = nullptr, *bdr1 = nullptr;  // levels of the next refresh, drawn ahead
    // the bit-plane tally is kept by the one-launch sweep only; a per-half
    // sweep leaves it stale until the spins are written again
    bool tally_ok = true;
    // multispin working planes (msc_kernels.hpp), allocated on first use
    uint64_t* ms = nullptr;   // [L][2][rows][Lx/128] spins
    uint64_t* md0 = nullptr;  // daemon level bit 0, same shape
    uint64_t* md1 = nullptr;  // daemon level bit 1
    uint64_t* mb = nullptr;   // [L][6][rows][Lx/128] couplings of the even sites
    uint64_t *ms_alt = nullptr, *md0_alt = nullptr, *md1_alt = nullptr;  // written by the one-launch sweep
    int32_t msc_fused = 1;  // multispin: 1 = one launch per sweep (z march), 0 = one per half sweep
    // one-launch multispin sweep: levels of the next refresh drawn ahead on a
    // side stream (default priority) while the sweeps before it run
    int32_t draw_ahead = 1;
    uint64_t *mdr0 = nullptr, *mdr1 = nullptr;  // drawn levels, shape of md0 / md1
    hipStream_t draw_stream = nullptr;
    hipEvent_t draw_free = nullptr, draw_done = nullptr;
    // sweep kernel selection (MICSA_OPT_*)
    int32_t kernel_opt = MICSA_KERNEL_AUTO;
    int32_t tile_y = 0, tile_z = 0;
    int32_t xcd_map = 2;  // XCD-aware tile order for the fused sweeps (2: z bands on the multispin sweep)
    int32_t prefetch = 1;  // steps of loads in flight in the fused MicSA sweep (1 or 2)
    int32_t temporal = 2;  // MicSA sweeps per pass of the fused kernel (1 or 2)
    int32_t msc_pass = 2;  // MicSA sweeps per pass of the one-launch multispin sweep (1 or 2)
    int32_t use_graphs = 0;
    // walkers on the fused sweep: parity of a forward-X wandering the stored
    // daemons still owe (applied by the next fused sweep on load), or -1
    int32_t pend_wander = -1;
    // the multispin planes hold the state and the byte arrays are stale (a
    // multispin call leaves its planes live; whatever reads or writes the
    // byte arrays unpacks them first)
    bool msc_live = false;
    // refresh sweep whose levels the multispin draw planes hold, drawn during
    // an earlier call (-1: none)
    int64_t msc_drawn = -1;
    // replayable graphs of kGraphSweeps sweeps for the per-half paths, per algo
    int64_t* d_k = nullptr;  // device copy of the sweep counter
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec[kAlgos] = {};
    const void* gkey[kAlgos] = {};  // state buffer the graph was captured with
    unsigned long long* tally = nullptr;  // [L][kSlots]
    unsigned long long* red = nullptr;    // [max(L, S)][kSlots] reduction scratch
    // device-pointer logging: one row of slots [2][L][kSlots] (energy, then
    // level sums), and the resident kernel's (U, sum m) pairs, grown on demand
    unsigned long long* logslots = nullptr;
    long long* rlog = nullptr;
    size_t rlog_cap = 0;  // entries of rlog
    Schedule sched;
    // device tables of the installed schedule, one entry per refresh index
    DaemonThresholds* d_dth = nullptr;
    HeatBathThresholds* d_hth = nullptr;
    MetropolisThresholds* d_mth = nullptr;
    int64_t k = 0;
    std::string err;
    // timing
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events[kTimingKinds];
    double time_ms[kTimingKinds] = {};
    int64_t launches[kTimingKinds] = {};
};

namespace {

int fail(micsa_ctx* c, int status, const std::string& msg)
{
    if (c) c->err = msg;
    return status;
}

int settle_msc(micsa_ctx* c);

#define HIP_TRY(ctx, call)                                                                       \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail((ctx), MICSA_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ----------------------------------------------------------- schedule maths
// Refresh points and temperatures (Sec. 2.7-2.8).  Host double arithmetic,
// compiled without FMA contraction so the thresholds are reproducible.
bool is_refresh(int64_t k, int32_t P) { return P >= 1 ? (k % P == 0) : (((k + 1) & k) == 0); }

int64_t refresh_index(int64_t k, int32_t P)
{
    if (P >= 1) return k / P;
    int64_t rho = -1;
    for (int64_t t = k + 1; t > 0; t >>= 1) ++rho;
    return rho;
}

// Refreshes over the timesteps of the schedule (Sec. 2.8: with gamma
// daemons per site a timestep is gamma sweeps; refresh points count timesteps).
int64_t refresh_count(const Schedule& s)
{
    return s.n_steps <= 0 ? 0 : refresh_index(s.n_steps - 1, s.period) + 1;
}

double temperature(const Schedule& s, int64_t rho)
{
    switch (s.kind) {
    case MICSA_SCHED_CONST: return s.T0;
    case MICSA_SCHED_LINEAR: {
        const int64_t n = refresh_count(s);
        if (n <= 1) return s.T0;
        const double f = (double)rho / (double)(n - 1);
        return s.T0 * (1.0 - f) + s.T1 * f;
    }
    default: return (rho >= 0 && rho < (int64_t)s.table.size()) ? s.table[(size_t)rho] : NAN;
    }
}

// t_k = floor(2^32 * P(m <= k)), P(m <= k) = (1 - e^{-4 beta (k+1)}) / (1 - e^{-16 beta}).
DaemonThresholds daemon_thresholds(double T)
{
    const double beta = 1.0 / T;
    uint64_t t[3];
    for (int k = 0; k < 3; ++k)
        t[k] = (uint64_t)std::floor(std::expm1(-4.0 * beta * (double)(k + 1)) / std::expm1(-16.0 * beta) *
                                    4294967296.0);
    return {t[0], t[1], t[2]};
}

// tau_v = floor(2^32 / (1 + e^{-2 beta h})), h = 6 - 2v.
HeatBathThresholds heatbath_thresholds(double T)
{
    const double beta = 1.0 / T;
    HeatBathThresholds th;
    for (int v = 0; v < 7; ++v)
        th.tau[v] = (uint64_t)std::floor(4294967296.0 / (1.0 + std::exp(-2.0 * beta * (double)(6 - 2 * v))));
    return th;
}

// theta_q = floor(2^32 e^{-beta dH}) for dH = 4q - 12 > 0, 2^32 for dH <= 0.
MetropolisThresholds metropolis_thresholds(double T)
{
    const double beta = 1.0 / T;
    MetropolisThresholds th;
    for (int q = 0; q < 7; ++q) {
        const int dH = 4 * q - 12;
        th.tau[q] = dH <= 0 ? 4294967296ull : (uint64_t)std::floor(std::exp(-beta * (double)dH) * 4294967296.0);
    }
    return th;
}

// The per-refresh table of a canonical baseline, and its timing kind.
const HeatBathThresholds* canonical_table(const micsa_ctx* c, int32_t algo)
{
    return algo == MICSA_ALGO_METROPOLIS ? c->d_mth : c->d_hth;
}

int canonical_timing(int32_t algo) { return algo == MICSA_ALGO_METROPOLIS ? kTimeMetropolis : kTimeHeatBath; }

// --------------------------------------------------------------- launching
dim3 grid_for(int64_t threads, int y)
{
    return dim3((unsigned)((threads + kBlock - 1) / kBlock), (unsigned)y, 1);
}

struct TimedLaunch {
    micsa_ctx* c;
    int kind;
    hipEvent_t a = nullptr, b = nullptr;
    TimedLaunch(micsa_ctx* ctx, int kd) : c(ctx), kind(kd)
    {
        if (c->timing) {
            if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
                a = b = nullptr;
                return;
            }
            (void)hipEventRecord(a, c->stream);
        }
    }
    ~TimedLaunch()
    {
        if (a && b) {
            (void)hipEventRecord(b, c->stream);
            c->events[kind].push_back({a, b});
        }
    }
};

int check_launch(micsa_ctx* c, const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, MICSA_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return MICSA_OK;
}

// Zero the accumulator slots of n entities.
int zero_slots(micsa_ctx* c, unsigned long long* p, int64_t n)
{
    k_fill_i64<<<grid_for(n * kSlots, 1), kBlock, 0, c->stream>>>(p, n * kSlots, 0ull);
    return check_launch(c, "k_fill_i64");
}

// Copy the slots of n entities to the host and sum them per entity.
int read_slots(micsa_ctx* c, const unsigned long long* dev, int64_t n, std::vector<int64_t>& out)
{
    std::vector<int64_t> raw((size_t)(n * kSlots));
    HIP_TRY(c, hipMemcpyAsync(raw.data(), dev, raw.size() * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    out.assign((size_t)n, 0);
    for (int64_t e = 0; e < n; ++e)
        for (int k = 0; k < kSlots; ++k) out[(size_t)e] += raw[(size_t)(e * kSlots + k)];
    return MICSA_OK;
}

// tally <- E (slot 0 = E, other slots 0).
int set_tally(micsa_ctx* c, const std::vector<int64_t>& E)
{
    std::vector<int64_t> raw((size_t)c->L * kSlots, 0);
    for (int l = 0; l < c->L; ++l) raw[(size_t)l * kSlots] = E[(size_t)l];
    HIP_TRY(c, hipMemcpyAsync(c->tally, raw.data(), raw.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MICSA_OK;
}

GeomB geomb(const micsa_ctx* c) { return GeomB{c->g, c->G, c->p.lane_mode}; }

int word_lattices(const micsa_ctx* c) { return bp_word_lattices(geomb(c)); }

// Launch shape of the one-launch bit-plane sweep: TZ planes per work-group
// (1, or 2 with TILE_Z = 2), one thread per word of a plane, LDS for TZ + 4
// odd and TZ + 2 even planes.
struct BpLaunch {
    BpTile f;
    unsigned block;
    size_t lds;
};

BpLaunch bp_launch(const micsa_ctx* c)
{
    BpLaunch b{};
    const int Kx = c->p.Lx / 2;
    const int P = c->p.Ly * Kx;
    if (P > 1024) {
        // kb_sweep_rows: tiles of TY rows plus two ring rows on each side, a
        // word position per thread; TY keeps the rows computed per plane
        // (nty (TY + 4)) smallest, the larger TY on ties
        const int tymax = std::min(1024 / Kx - 4, c->p.Ly);
        int best = 0;
        int64_t cost = 0;
        for (int ty = 1; ty <= tymax; ++ty) {
            const int64_t n = (c->p.Ly + ty - 1) / ty, w = n * (ty + 4);
            if (!best || w <= cost) {
                best = ty;
                cost = w;
            }
        }
        if (c->tile_y > 0) best = std::min(c->tile_y, tymax);
        const int TY = std::max(best, 1);
        b.f = BpTile{1, c->p.Lz, P, TY, (c->p.Ly + TY - 1) / TY};
        const int PT = (TY + 4) * Kx;
        b.block = (unsigned)((PT + 63) / 64 * 64);
        b.lds = std::max((size_t)8 * PT * 8, (size_t)(b.block / 64) * 64 * 8);
        return b;
    }
    const int TZ = c->tile_z == 2 && c->p.Lz % 2 == 0 && P <= 512 ? 2 : 1;
    b.f = BpTile{TZ, c->p.Lz / TZ, P, c->p.Ly, 1};
    b.block = (unsigned)((P + 63) / 64 * 64);
    const size_t planes = (size_t)(2 * TZ + 6) * P * 8, part = (size_t)(b.block / 64) * 64 * 8;
    b.lds = std::max(planes, part);
    return b;
}

bool bp_rows(const BpLaunch& b) { return b.f.nty > 1 || b.f.P > 1024; }

// The one-launch sweep fits: a word position per thread (at most 1024 per
// work-group: a whole plane, or TY + 4 >= 5 rows of one) and LDS within a
// work-group's 160 KB.
bool bp_fits(const micsa_ctx* c, const BpLaunch& b)
{
    if (bp_rows(b)) return 1024 / (c->p.Lx / 2) - 4 >= 1 && b.lds <= 160 * 1024;
    return b.f.P <= (b.f.TZ == 1 ? 1024 : 512) && b.lds <= 160 * 1024;
}

// AUTO takes the one-launch sweep where a plane fits a work-group; on larger
// planes its row tiles (kb_sweep_rows) run only on request (KERNEL_FUSED):
// there the per-half kernels are faster (8.6 against 11.9 us per sweep at
// L = 64 on one MI355X), but keep no per-lane tally.
bool bp_one_launch(const micsa_ctx* c)
{
    if (!c->bit || c->kernel_opt == MICSA_KERNEL_SIMPLE) return false;
    const BpLaunch b = bp_launch(c);
    return bp_fits(c, b) && (!bp_rows(b) || c->kernel_opt == MICSA_KERNEL_FUSED);
}

// One-launch bit-plane sweep; with drawn the levels are read from the drawn
// planes (a refresh drawn ahead).
int launch_bp_sweep(micsa_ctx* c, bool drawn)
{
    const BpLaunch b = bp_launch(c);
    if (!c->bspin_alt) {
        const size_t words = (size_t)word_lattices(c) * 2 * (size_t)c->g.Nh;
        bool ok = true;
        for (uint64_t** q : {&c->bspin_alt, &c->bdm0_alt, &c->bdm1_alt})
            ok = ok && hipMalloc(q, words * 8) == hipSuccess;
        if (!ok) {
            (void)hipGetLastError();
            for (uint64_t** q : {&c->bspin_alt, &c->bdm0_alt, &c->bdm1_alt}) {
                if (*q) (void)hipFree(*q);
                *q = nullptr;
            }
            return fail(c, MICSA_ENOMEM, "bit-plane sweep buffers");
        }
    }
    const auto kern = bp_rows(b) ? kb_sweep_rows<true> : b.f.TZ == 2 ? kb_sweep<true, 2> : kb_sweep<true, 1>;
    if (b.lds > 64 * 1024 &&
        hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b.lds) != hipSuccess)
        return fail(c, MICSA_EHIP, "kb_sweep LDS attribute");
    const dim3 grid((unsigned)(b.f.ntz * b.f.nty * word_lattices(c)));
    {
        TimedLaunch t(c, kTimeSweep);
        kern<<<grid, b.block, b.lds, c->stream>>>(geomb(c), b.f, c->bspin, drawn ? c->bdr0 : c->bdm0,
                                                  drawn ? c->bdr1 : c->bdm1, c->bJ, c->bspin_alt, c->bdm0_alt,
                                                  c->bdm1_alt, c->tally);
    }
    const int st = check_launch(c, "kb_sweep");
    if (st) return st;
    std::swap(c->bspin, c->bspin_alt);
    std::swap(c->bdm0, c->bdm0_alt);
    std::swap(c->bdm1, c->bdm1_alt);
    return MICSA_OK;
}

int64_t next_refresh(const micsa_ctx* c, int64_t from, int64_t end);

// Draw the levels of bit-plane refresh sweep kr into the drawn planes on the
// side stream, after everything the library stream holds so far (the sweep
// that last read them); the refresh sweep waits for draw_done.
int draw_bp_levels(micsa_ctx* c, int64_t kr)
{
    const int64_t rho = refresh_index(kr, c->sched.period);
    const double T = temperature(c->sched, rho);
    if (!(T > 0.0) || !std::isfinite(T)) return fail(c, MICSA_ERANGE, "no temperature for this refresh");
    if (!c->bdr0) {
        const size_t words = (size_t)word_lattices(c) * 2 * (size_t)c->g.Nh;
        if (hipMalloc(&c->bdr0, words * 8) != hipSuccess || hipMalloc(&c->bdr1, words * 8) != hipSuccess) {
            (void)hipGetLastError();
            if (c->bdr0) (void)hipFree(c->bdr0);
            c->bdr0 = c->bdr1 = nullptr;
            return fail(c, MICSA_ENOMEM, "bit-plane drawn levels");
        }
    }
    if (!c->draw_stream) {
        HIP_TRY(c, hipStreamCreateWithFlags(&c->draw_stream, hipStreamNonBlocking));
        HIP_TRY(c, hipEventCreateWithFlags(&c->draw_free, hipEventDisableTiming));
        HIP_TRY(c, hipEventCreateWithFlags(&c->draw_done, hipEventDisableTiming));
    }
    HIP_TRY(c, hipEventRecord(c->draw_free, c->stream));
    HIP_TRY(c, hipStreamWaitEvent(c->draw_stream, c->draw_free, 0));
    kb_refresh<<<dim3(bp_refresh_blocks(c->g), (unsigned)word_lattices(c)), 256, 0, c->draw_stream>>>(
        geomb(c), c->bdr0, c->bdr1, (uint32_t)rho, daemon_thresholds(T));
    const int st = check_launch(c, "kb_refresh (drawn ahead)");
    if (st) return st;
    HIP_TRY(c, hipEventRecord(c->draw_done, c->draw_stream));
    return MICSA_OK;
}

// MicSA sweeps k .. k + n - 1 of the bit-plane layout on the one-launch
// sweep; the levels of each refresh are drawn ahead on the side stream
// (OPT_DRAW_AHEAD, default) while the sweeps before it run, or in place just
// before it.
int sweep_bitplane(micsa_ctx* c, int64_t n)
{
    const int64_t k_end = c->k + n;
    int64_t drawn = -1;
    int st;
    if (c->draw_ahead && (drawn = next_refresh(c, c->k, k_end)) >= 0 && (st = draw_bp_levels(c, drawn))) return st;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t k = c->k;
        const bool refresh = is_refresh(k, c->sched.period);
        const int64_t rho = refresh_index(k, c->sched.period);
        const double T = temperature(c->sched, rho);
        if (!(T > 0.0) || !std::isfinite(T)) return fail(c, MICSA_ERANGE, "no temperature for this refresh");
        const bool use_drawn = refresh && drawn == k;
        if (use_drawn) {
            HIP_TRY(c, hipStreamWaitEvent(c->stream, c->draw_done, 0));
        } else if (refresh) {
            TimedLaunch t(c, kTimeRefresh);
            kb_refresh<<<dim3(bp_refresh_blocks(c->g), (unsigned)word_lattices(c)), 256, 0, c->stream>>>(
                geomb(c), c->bdm0, c->bdm1, (uint32_t)rho, daemon_thresholds(T));
            if ((st = check_launch(c, "kb_refresh"))) return st;
        }
        if ((st = launch_bp_sweep(c, use_drawn))) return st;
        if (use_drawn && (drawn = next_refresh(c, k + 1, k_end)) >= 0 && (st = draw_bp_levels(c, drawn))) return st;
        c->k = k + 1;
    }
    return MICSA_OK;
}

int launch_bitplane_sweep(micsa_ctx* c, bool refresh, int64_t rho, double T)
{
    const int WL = word_lattices(c);
    if (refresh) {
        TimedLaunch t(c, kTimeRefresh);
        kb_refresh<<<dim3(bp_refresh_blocks(c->g), (unsigned)WL), 256, 0, c->stream>>>(
            geomb(c), c->bdm0, c->bdm1, (uint32_t)rho, daemon_thresholds(T));
    }
    int st = check_launch(c, "kb_refresh");
    if (st) return st;
    c->tally_ok = false;
    const dim3 grid = grid_for(c->g.Nh, WL);
    {
        TimedLaunch t(c, kTimeSweep);
        kb_micsa_half<0><<<grid, kBlock, 0, c->stream>>>(geomb(c), c->bspin, c->bdm0, c->bdm1, c->bJ);
    }
    if ((st = check_launch(c, "kb_micsa_half<0>"))) return st;
    {
        TimedLaunch t(c, kTimeSweep);
        kb_micsa_half<1><<<grid, kBlock, 0, c->stream>>>(geomb(c), c->bspin, c->bdm0, c->bdm1, c->bJ);
    }
    return check_launch(c, "kb_micsa_half<1>");
}

// Per-lane counts of the bit-plane layout into dst slots (see kb_lane_count).
template <int KIND>
int enqueue_lane_count(micsa_ctx* c, unsigned long long* dst, int ra, int rb)
{
    const int64_t ent = KIND == 2 ? c->p.n_samples : c->L;
    int st = zero_slots(c, dst, ent);
    if (st) return st;
    const int64_t per_block = 128;
    const unsigned ny = (unsigned)(KIND == 2 ? (c->p.lane_mode ? c->p.n_samples : c->G) : word_lattices(c));
    {
        TimedLaunch t(c, kTimeReduce);
        kb_lane_count<KIND><<<dim3((unsigned)((c->g.Nh + per_block - 1) / per_block), ny), 64, 0, c->stream>>>(
            geomb(c), c->bspin, c->bdm0, c->bdm1, c->bJ, ra, rb, per_block, dst);
    }
    return check_launch(c, "kb_lane_count");
}

int launch_refresh(micsa_ctx* c, int64_t rho, double T)
{
    TimedLaunch t(c, kTimeRefresh);
    k_refresh<<<grid_for(c->g.Nh / 4, c->L * c->gamma), kBlock, 0, c->stream>>>(c->g, c->dem, (uint32_t)rho,
                                                                                 daemon_thresholds(T));
    return check_launch(c, "k_refresh");
}

// The fused sweep needs whole 16-site chunks per row and a work-group that
// holds at least a one-row tile with its four ring rows.
// Resident sweeps keep a state byte per site and a coupling byte per even
// site (1.5 B per site) in the LDS of one work-group.
constexpr size_t kResidentLdsMax = 150 * 1024;
constexpr int kResidentBlock = 512;
constexpr int64_t kResidentChunk = 2048;  // sweeps per resident launch

bool resident_eligible(const micsa_ctx* c)
{
    return !c->bit && c->gamma == 1 && (size_t)c->g.Nh * 3 <= kResidentLdsMax;
}

bool use_resident(const micsa_ctx* c)
{
    if (c->kernel_opt == MICSA_KERNEL_RESIDENT) return true;
    return c->kernel_opt == MICSA_KERNEL_AUTO && resident_eligible(c);
}

bool fused_eligible(const micsa_ctx* c)
{
    return !c->bit && c->gamma == 1 && c->p.Lx % 32 == 0 && 5 * (c->p.Lx / 32) <= 1024;
}

// (the one-launch sweep addresses a plane with 32-bit byte offsets: fewer than 2^29 words)
bool msc_eligible(const micsa_ctx* c)
{
    return !c->bit && c->gamma == 1 && c->p.Lx % 128 == 0 && (int64_t)c->g.rows * (c->p.Lx / 128) < (int64_t(1) << 29);
}

// AUTO takes the multispin planes for MicSA calls of at least kMscMinSweeps
// sweeps on lattices the resident kernel does not hold (a call packs and
// unpacks the state once, about the traffic of two sweeps).
constexpr int64_t kMscMinSweeps = 8;

bool msc_one_launch(const micsa_ctx* c);

bool use_msc(const micsa_ctx* c, int64_t n = kMscMinSweeps, int32_t algo = MICSA_ALGO_MICSA)
{
    if (!msc_eligible(c)) return false;
    if (algo == MICSA_ALGO_WALKERS && !msc_one_launch(c)) return false;  // walkers need the one-launch sweep
    if (c->kernel_opt == MICSA_KERNEL_MULTISPIN) return true;
    return c->kernel_opt == MICSA_KERNEL_AUTO && !use_resident(c) && n >= kMscMinSweeps;
}

// One launch per sweep with a z plane per work-group (byte_slab.hpp): a
// plane's 4-site words fit one work-group.
bool slab_eligible(const micsa_ctx* c)
{
    return !c->bit && c->gamma == 1 && (int64_t)c->p.Ly * (c->p.Lx / 8) <= kSlabLanes;
}

bool use_fused(const micsa_ctx* c);

// AUTO takes it for lattices the resident kernel does not hold that are too
// narrow for the fused sweep (Lx < 128).
bool use_slab(const micsa_ctx* c)
{
    if (!slab_eligible(c)) return false;
    if (c->kernel_opt == MICSA_KERNEL_SLAB) return true;
    return c->kernel_opt == MICSA_KERNEL_AUTO && !use_resident(c) && !use_fused(c);
}

// One slab sweep.  refresh: draw the levels in the kernel; drawn (not
// null): read them from levels drawn ahead in place of the stored daemons.
int launch_slab_sweep(micsa_ctx* c, bool refresh, int64_t rho, double T, const uint8_t* drawn = nullptr)
{
    const int P = c->p.Ly * (c->p.Lx / 8);
    const dim3 grid((unsigned)(c->L * c->p.Lz));
    const unsigned block = (unsigned)((P + 63) / 64 * 64);
    const size_t lds = (size_t)8 * P * 4;
    const uint8_t* dem_in = drawn ? drawn : c->dem;
    {
        TimedLaunch t(c, kTimeSweep);
        if (refresh && !drawn)
            k_micsa_slab<true><<<grid, block, lds, c->stream>>>(c->g, c->spin, dem_in, c->spin_alt, c->dem_alt,
                                                                c->tally, (uint32_t)rho, daemon_thresholds(T));
        else
            k_micsa_slab<false><<<grid, block, lds, c->stream>>>(c->g, c->spin, dem_in, c->spin_alt, c->dem_alt,
                                                                 c->tally, 0u, DaemonThresholds{0, 0, 0});
    }
    const int st = check_launch(c, "k_micsa_slab");
    if (st) return st;
    std::swap(c->spin, c->spin_alt);
    std::swap(c->dem, c->dem_alt);
    return MICSA_OK;
}

// Sweeps k and k + 1 in one slab launch.  refreshA / refreshB: k / k + 1 are
// refresh points whose levels the kernel draws; drawnA (not null): the
// levels of sweep k, drawn ahead, read in place of the stored daemons;
// next (not null, no refresh in the launch): also draw the levels of refresh
// rhoN at temperature TN into next.
int launch_slab_sweep2(micsa_ctx* c, bool refreshA, int64_t rhoA, double TA, bool refreshB, int64_t rhoB, double TB,
                       const uint8_t* drawnA, uint8_t* next, int64_t rhoN, double TN)
{
    if (drawnA) refreshA = false;
    if (refreshA || refreshB) next = nullptr;
    const int P = c->p.Ly * (c->p.Lx / 8);
    const dim3 grid((unsigned)(c->L * c->p.Lz));
    const unsigned block = (unsigned)((P + 63) / 64 * 64);
    const size_t lds = (size_t)24 * P * 4;
    const SlabRefresh ra{(uint32_t)rhoA, refreshA ? daemon_thresholds(TA) : DaemonThresholds{0, 0, 0}};
    const SlabRefresh rb{(uint32_t)rhoB, refreshB ? daemon_thresholds(TB) : DaemonThresholds{0, 0, 0}};
    const SlabRefresh rn{(uint32_t)rhoN, next ? daemon_thresholds(TN) : DaemonThresholds{0, 0, 0}};
    const auto kern = next ? k_micsa_slab2<false, false, true>
                           : refreshA ? (refreshB ? k_micsa_slab2<true, true, false> : k_micsa_slab2<true, false, false>)
                                      : (refreshB ? k_micsa_slab2<false, true, false> : k_micsa_slab2<false, false, false>);
    if (lds > 64 * 1024 &&
        hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return fail(c, MICSA_EHIP, "k_micsa_slab2 LDS attribute");
    {
        TimedLaunch t(c, kTimeSweep);
        kern<<<grid, block, lds, c->stream>>>(c->g, c->spin, drawnA ? drawnA : c->dem, c->spin_alt, c->dem_alt,
                                              c->tally, ra, rb, rn, next);
    }
    const int st = check_launch(c, "k_micsa_slab2");
    if (st) return st;
    std::swap(c->spin, c->spin_alt);
    std::swap(c->dem, c->dem_alt);
    return MICSA_OK;
}

// Two sweeps per slab launch pay off while the one-sweep launch leaves
// compute units idle (fewer planes than units, e.g. L = 64 with 2
// replicas): they halve the launches on a latency-bound path, at twice the
// arithmetic per sweep.  A full grid keeps one sweep per launch.
bool slab_pairs(const micsa_ctx* c)
{
    return c->temporal == 2 && (int64_t)c->L * c->p.Lz < (c->cus > 0 ? c->cus : 256);
}

int64_t next_refresh(const micsa_ctx* c, int64_t from, int64_t end);

constexpr int64_t kSlabDrawWindow = 1024;  // how far ahead a launch looks for the next refresh

// The two buffers of levels drawn ahead for two-sweep slab launches.
int slab_alloc(micsa_ctx* c)
{
    if (c->sdr[0]) return MICSA_OK;
    const size_t bytes = (size_t)c->L * 2 * (size_t)c->g.Nh;
    for (auto& q : c->sdr)
        if (hipMalloc(&q, bytes) != hipSuccess) {
            (void)hipGetLastError();
            for (auto& f : c->sdr)
                if (f) (void)hipFree(f);
            c->sdr[0] = c->sdr[1] = nullptr;
            return fail(c, MICSA_ENOMEM, "slab drawn levels");
        }
    c->sdr_k[0] = c->sdr_k[1] = -1;
    return MICSA_OK;
}

// MicSA sweeps k .. k + n - 1 on the slab sweep (gamma = 1): two per launch
// where slab_pairs() holds, else one.  With OPT_DRAW_AHEAD (default) a
// two-sweep launch with no refresh of its own also draws the levels of the
// next refresh of the schedule (each work-group its own plane) into one of
// two buffers; the launch that starts at that refresh, in this call or a
// later one, reads them, and the buffer it reads is never the one its own
// draw writes.  Other refreshes are drawn inside the refresh launch.
int sweep_slab(micsa_ctx* c, int64_t n)
{
    const int64_t k_end = c->k + n;
    const bool pairs = slab_pairs(c);
    const bool ahead = c->draw_ahead != 0 && pairs;
    int st;
    if (ahead && (st = slab_alloc(c))) return st;
    while (c->k < k_end) {
        const int64_t k = c->k;
        const bool refresh = is_refresh(k, c->sched.period);
        const int64_t rho = refresh_index(k, c->sched.period);
        const double T = temperature(c->sched, rho);
        if (!(T > 0.0) || !std::isfinite(T)) return fail(c, MICSA_ERANGE, "no temperature for this refresh");
        int rd = -1;  // buffer holding this refresh's levels
        if (refresh && ahead)
            for (int b = 0; b < 2; ++b)
                if (c->sdr_k[b] == k) rd = b;
        const uint8_t* drawn = rd >= 0 ? c->sdr[rd] : nullptr;
        if (pairs && k + 1 < k_end) {
            const bool refreshB = is_refresh(k + 1, c->sched.period);
            const int64_t rhoB = refresh_index(k + 1, c->sched.period);
            const double TB = temperature(c->sched, rhoB);
            if (!(TB > 0.0) || !std::isfinite(TB)) return fail(c, MICSA_ERANGE, "no temperature for this refresh");
            // the next refresh after this pair, if no buffer holds it yet
            uint8_t* next = nullptr;
            int wb = -1;
            int64_t kn = -1, rhoN = 0;
            double TN = 0.0;
            if (ahead && !(refresh && !drawn) && !refreshB &&
                (kn = next_refresh(c, k + 2, std::min(c->sched.n_sweeps, k + 2 + kSlabDrawWindow))) >= 0 &&
                c->sdr_k[0] != kn && c->sdr_k[1] != kn) {
                wb = rd >= 0 ? 1 - rd : (c->sdr_k[0] < c->sdr_k[1] ? 0 : 1);
                rhoN = refresh_index(kn, c->sched.period);
                TN = temperature(c->sched, rhoN);
                if (!(TN > 0.0) || !std::isfinite(TN)) return fail(c, MICSA_ERANGE, "no temperature for this refresh");
                next = c->sdr[wb];
            }
            if ((st = launch_slab_sweep2(c, refresh, rho, T, refreshB, rhoB, TB, drawn, next, rhoN, TN))) return st;
            if (next) c->sdr_k[wb] = kn;
            c->k = k + 2;
        } else {
            if ((st = launch_slab_sweep(c, refresh, rho, T, drawn))) return st;
            c->k = k + 1;
        }
    }
    return MICSA_OK;
}

bool use_fused(const micsa_ctx* c)
{
    if (c->bit || c->kernel_opt == MICSA_KERNEL_SIMPLE || c->kernel_opt == MICSA_KERNEL_RESIDENT ||
        c->kernel_opt == MICSA_KERNEL_SLAB)
        return false;
    if (c->kernel_opt == MICSA_KERNEL_FUSED) return true;
    return fused_eligible(c) && c->p.Lx >= 128;
}

// Largest divisor of n not above cap (n >= 1, cap >= 1).
int divisor_at_most(int n, int cap)
{
    for (int d = std::min(n, cap); d > 1; --d)
        if (n % d == 0) return d;
    return 1;
}

// Tile of the fused sweep: TY rows (so that (TY+4) * NC lanes fit a
// work-group of at most 1024), TZ planes chosen to give the device at least
// two work-groups per compute unit when the lattice allows it.
FusedTile choose_tile(const micsa_ctx* c)
{
    FusedTile f;
    f.NC = c->p.Lx / 32;
    const int ty_cap = std::max(1, std::min(32, 1024 / f.NC - 4));
    f.TY = c->tile_y > 0 && c->p.Ly % c->tile_y == 0 ? c->tile_y : divisor_at_most(c->p.Ly, ty_cap);
    f.nty = c->p.Ly / f.TY;
    f.xcd = c->xcd_map;
    if (c->tile_z > 0) {
        f.TZ = c->tile_z;
    } else {
        f.TZ = divisor_at_most(c->p.Lz, 32);
        while (f.TZ > 4 && (int64_t)f.nty * (c->p.Lz / f.TZ) * c->L < 512) {
            const int next = divisor_at_most(c->p.Lz, f.TZ - 1);
            if (next < 4) break;
            f.TZ = next;
        }
    }
    f.ntz = c->p.Lz / f.TZ;
    if ((f.nty * f.ntz) % 8 != 0) f.xcd = 0;
    return f;
}

int launch_fused_sweep(micsa_ctx* c, bool refresh, int64_t rho, double T, int wander = -1)
{
    const FusedTile f = choose_tile(c);
    const int lanes = (f.TY + 4) * f.NC;
    const int block = (lanes + 63) / 64 * 64;
    const size_t lds = (size_t)64 * (f.TY + 4) * f.NC;
    const dim3 grid((unsigned)(f.nty * (c->p.Lz / f.TZ)), (unsigned)c->L, 1);
    const DaemonThresholds th = refresh ? daemon_thresholds(T) : DaemonThresholds{0, 0, 0};
    {
        TimedLaunch t(c, kTimeSweep);
        const bool pf2 = c->prefetch == 2 && block <= kPf2Lanes;  // larger tiles run the one-step variant
        const auto kern = refresh ? (pf2 ? k_micsa_sweep_fused<true, 2> : k_micsa_sweep_fused<true, 1>)
                                  : (pf2 ? k_micsa_sweep_fused<false, 2> : k_micsa_sweep_fused<false, 1>);
        kern<<<grid, block, lds, c->stream>>>(c->g, f, c->spin, c->dem, c->spin_alt, c->dem_alt, c->tally,
                                              (uint32_t)rho, th, refresh ? -1 : wander);
    }
    const int st = check_launch(c, "k_micsa_sweep_fused");
    if (st) return st;
    std::swap(c->spin, c->spin_alt);
    std::swap(c->dem, c->dem_alt);
    return MICSA_OK;
}

// Both halves with daemon family fam.
// Tile of the two-sweep kernel: TY + 8 ring rows of NC lanes within
// kSweep2Lanes; the tile options apply where they fit.
FusedTile choose_tile2(const micsa_ctx* c)
{
    FusedTile f = choose_tile(c);
    const int ty_cap = kSweep2Lanes / f.NC - 8;
    if (f.TY > ty_cap) {
        f.TY = divisor_at_most(c->p.Ly, ty_cap);
        f.nty = c->p.Ly / f.TY;
        f.xcd = c->xcd_map && (f.nty * f.ntz) % 8 == 0;
    }
    return f;
}

bool sweep2_eligible(const micsa_ctx* c) { return kSweep2Lanes / (c->p.Lx / 32) - 8 >= 1; }

// Sweeps k and k + 1 in one pass (fused2_kernels.hpp); refreshA / refreshB
// say whether k / k + 1 are refresh points.  Walkers (walk): wanderA is a
// wandering owed from before (-1: none), wanderAB the parity of the
// wandering between the two sweeps.
int launch_fused_sweep2(micsa_ctx* c, bool refreshA, int64_t rhoA, double TA, bool refreshB, int64_t rhoB, double TB,
                        bool walk = false, int wanderA = -1, int wanderAB = -1)
{
    const FusedTile f = choose_tile2(c);
    const int lanes = (f.TY + 8) * f.NC;
    const int block = (lanes + 63) / 64 * 64;
    const size_t lds = (size_t)128 * (f.TY + 8) * f.NC;  // 4 planes x 2 buffers x 16 B per lane slot
    using Kern = void (*)(Geom, FusedTile, const uint8_t*, const uint8_t*, uint8_t*, uint8_t*, unsigned long long*,
                          uint32_t, DaemonThresholds, uint32_t, DaemonThresholds, int, int);
    static const Kern kernels[8] = {
        k_micsa_sweep2_fused<false, false, false>, k_micsa_sweep2_fused<true, false, false>,
        k_micsa_sweep2_fused<false, true, false>,  k_micsa_sweep2_fused<true, true, false>,
        k_micsa_sweep2_fused<false, false, true>,  k_micsa_sweep2_fused<true, false, true>,
        k_micsa_sweep2_fused<false, true, true>,   k_micsa_sweep2_fused<true, true, true>};
    static bool attr_set[8] = {};
    const int which = (refreshA ? 1 : 0) + (refreshB ? 2 : 0) + (walk ? 4 : 0);
    if (!attr_set[which]) {
        const hipError_t e = hipFuncSetAttribute((const void*)kernels[which],
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)kResidentLdsMax);
        if (e != hipSuccess) return fail(c, MICSA_EHIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
        attr_set[which] = true;
    }
    const dim3 grid((unsigned)(f.nty * f.ntz), (unsigned)c->L, 1);
    const DaemonThresholds thA = refreshA ? daemon_thresholds(TA) : DaemonThresholds{0, 0, 0};
    const DaemonThresholds thB = refreshB ? daemon_thresholds(TB) : DaemonThresholds{0, 0, 0};
    {
        TimedLaunch t(c, kTimeSweep);
        kernels[which]<<<grid, block, lds, c->stream>>>(c->g, f, c->spin, c->dem, c->spin_alt, c->dem_alt, c->tally,
                                                        (uint32_t)rhoA, thA, (uint32_t)rhoB, thB,
                                                        refreshA ? -1 : wanderA, wanderAB);
    }
    const int st = check_launch(c, "k_micsa_sweep2_fused");
    if (st) return st;
    std::swap(c->spin, c->spin_alt);
    std::swap(c->dem, c->dem_alt);
    return MICSA_OK;
}

// Walkers in the two-sweep kernel need a row's chunks in one wave.
bool sweep2_walk_eligible(const micsa_ctx* c)
{
    const int nc = c->p.Lx / 32;
    return c->gamma == 1 && sweep2_eligible(c) && 64 % nc == 0;
}

int launch_micsa_sweep(micsa_ctx* c, int fam)
{
    const int64_t words = (int64_t)c->g.rows * c->g.Wr;
    {
        TimedLaunch t(c, kTimeSweep);
        k_micsa_half<0><<<grid_for(words, c->L), kBlock, 0, c->stream>>>(c->g, c->spin, c->dem, c->tally,
                                                                          fam);
    }
    int st = check_launch(c, "k_micsa_half<0>");
    if (st) return st;
    {
        TimedLaunch t(c, kTimeSweep);
        k_micsa_half<1><<<grid_for(words, c->L), kBlock, 0, c->stream>>>(c->g, c->spin, c->dem, c->tally,
                                                                          fam);
    }
    return check_launch(c, "k_micsa_half<1>");
}

int launch_fused_canonical(micsa_ctx* c, int32_t algo, int64_t k, double T)
{
    const FusedTile f = choose_tile(c);
    const int lanes = (f.TY + 4) * f.NC;
    const int block = (lanes + 63) / 64 * 64;
    const size_t lds = (size_t)64 * (f.TY + 4) * f.NC;
    const dim3 grid((unsigned)(f.nty * (c->p.Lz / f.TZ)), (unsigned)c->L, 1);
    {
        TimedLaunch t(c, canonical_timing(algo));
        if (algo == MICSA_ALGO_METROPOLIS)
            k_heatbath_sweep_fused<1><<<grid, block, lds, c->stream>>>(c->g, f, c->spin, c->spin_alt, c->tally,
                                                                       (uint32_t)(2 * k), metropolis_thresholds(T));
        else
            k_heatbath_sweep_fused<0><<<grid, block, lds, c->stream>>>(c->g, f, c->spin, c->spin_alt, c->tally,
                                                                       (uint32_t)(2 * k), heatbath_thresholds(T));
    }
    const int st = check_launch(c, "k_heatbath_sweep_fused");
    if (st) return st;
    std::swap(c->spin, c->spin_alt);
    return MICSA_OK;
}

// One half sweep of a canonical baseline; with dk the sweep index and the
// table come from device memory (graph form), otherwise from k and th.
template <int P>
void enqueue_canonical_half(micsa_ctx* c, int32_t algo, hipStream_t st, int64_t k, const HeatBathThresholds& th,
                            const int64_t* dk)
{
    const int64_t words = (int64_t)c->g.rows * c->g.Wr;
    const dim3 grid = grid_for(words, c->L);
    const uint32_t time = (uint32_t)(2 * k + P);
    const int32_t period = c->sched.period;
    if (algo == MICSA_ALGO_METROPOLIS)
        k_heatbath_half<P, 1><<<grid, kBlock, 0, st>>>(c->g, c->spin, time, th, c->tally, dk, period, c->d_mth);
    else
        k_heatbath_half<P, 0><<<grid, kBlock, 0, st>>>(c->g, c->spin, time, th, c->tally, dk, period, c->d_hth);
}

int launch_canonical_sweep(micsa_ctx* c, int32_t algo, int64_t k, double T)
{
    if (use_fused(c)) return launch_fused_canonical(c, algo, k, T);
    const HeatBathThresholds th = algo == MICSA_ALGO_METROPOLIS ? metropolis_thresholds(T) : heatbath_thresholds(T);
    {
        TimedLaunch t(c, canonical_timing(algo));
        enqueue_canonical_half<0>(c, algo, c->stream, k, th, nullptr);
    }
    int st = check_launch(c, "k_heatbath_half<0>");
    if (st) return st;
    {
        TimedLaunch t(c, canonical_timing(algo));
        enqueue_canonical_half<1>(c, algo, c->stream, k, th, nullptr);
    }
    return check_launch(c, "k_heatbath_half<1>");
}

// Bond bits of every lattice into its even spin bytes (spins kept).
int enqueue_bonds(micsa_ctx* c)
{
    k_init_couplings<<<grid_for(c->g.Nh / 4, c->L), kBlock, 0, c->stream>>>(c->g, c->spin);
    return check_launch(c, "k_init_couplings");
}

// Enqueue: dst[l] = from-scratch H^EA of lattice l.
int enqueue_energy(micsa_ctx* c, unsigned long long* dst)
{
    if (int st = settle_msc(c)) return st;
    if (c->bit) return enqueue_lane_count<0>(c, dst, 0, 0);
    int st = zero_slots(c, dst, c->L);
    if (st) return st;
    TimedLaunch t(c, kTimeReduce);
    k_unsat_bonds<<<grid_for((int64_t)c->g.rows * c->g.Wr, c->L), kBlock, 0, c->stream>>>(c->g, c->spin,
                                                                                           dst);
    return check_launch(c, "k_unsat_bonds");
}

int enqueue_level_sum(micsa_ctx* c, unsigned long long* dst)
{
    if (int st = settle_msc(c)) return st;
    if (c->bit) return enqueue_lane_count<1>(c, dst, 0, 0);
    int st = zero_slots(c, dst, c->L);
    if (st) return st;
    TimedLaunch t(c, kTimeReduce);
    const int64_t wpl = (int64_t)c->gamma * 2 * c->g.Nh / 4;  // every family of the lattice
    k_level_sum<<<grid_for(wpl, c->L), kBlock, 0, c->stream>>>(wpl, reinterpret_cast<const uint32_t*>(c->dem),
                                                               dst);
    return check_launch(c, "k_level_sum");
}

int64_t n_sites(const micsa_ctx* c) { return (int64_t)c->p.Lx * c->p.Ly * c->p.Lz; }

// Natural index i -> (parity, h) of the byte layout.
inline void split_index(const micsa_ctx* c, int64_t i, int& par, int64_t& h)
{
    const int x = (int)(i % c->p.Lx);
    const int64_t row = i / c->p.Lx;
    const int y = (int)(row % c->p.Ly), z = (int)(row / c->p.Ly);
    par = (x + y + z) & 1;
    h = i >> 1;
}

// n sweeps from c->k in resident launches of up to kResidentChunk sweeps;
// with dlog != nullptr every `stride` sweeps (U, D) per lattice are written
// to dlog[row][L][2], rows counted from the first sweep of the call.
int launch_resident(micsa_ctx* c, int32_t algo, int64_t n, long long* dlog, int64_t stride)
{
    const size_t lds = (size_t)c->g.Nh * 3;
    // kernel instance: 0 MicSA, 1 heat bath, 2 Metropolis
    const int inst = algo == MICSA_ALGO_MICSA ? 0 : (algo == MICSA_ALGO_HEATBATH ? 1 : 2);
    static const void* const kernels[3] = {(const void*)k_resident<0>, (const void*)k_resident<1>,
                                           (const void*)k_resident<2>};
    static bool attr_set[3] = {false, false, false};
    if (!attr_set[inst]) {
        const hipError_t e =
            hipFuncSetAttribute(kernels[inst], hipFuncAttributeMaxDynamicSharedMemorySize, (int)kResidentLdsMax);
        if (e != hipSuccess) return fail(c, MICSA_EHIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
        attr_set[inst] = true;
    }
    const HeatBathThresholds* tab = canonical_table(c, algo);
    const int tkind = inst == 0 ? kTimeSweep : canonical_timing(algo);
    int64_t done = 0;
    while (done < n) {
        int64_t chunk = std::min<int64_t>(kResidentChunk, n - done);
        if (dlog && chunk % stride) chunk = std::max<int64_t>(stride, chunk / stride * stride);
        chunk = std::min(chunk, n - done);
        ResidentSched rs;
        rs.k0 = c->k + done;
        rs.n = chunk;
        rs.rho0 = 0;
        rs.period = c->sched.period;
        rs.log_stride = dlog ? (int32_t)stride : 0;
        rs.log_row0 = dlog ? done / stride : 0;
        {
            TimedLaunch t(c, tkind);
            if (inst == 0)
                k_resident<0><<<c->L, kResidentBlock, lds, c->stream>>>(c->g, c->spin, c->dem, c->tally, rs,
                                                                        c->d_dth, tab, dlog);
            else if (inst == 1)
                k_resident<1><<<c->L, kResidentBlock, lds, c->stream>>>(c->g, c->spin, c->dem, c->tally, rs,
                                                                        c->d_dth, tab, dlog);
            else
                k_resident<2><<<c->L, kResidentBlock, lds, c->stream>>>(c->g, c->spin, c->dem, c->tally, rs,
                                                                        c->d_dth, tab, dlog);
        }
        const int st = check_launch(c, "k_resident");
        if (st) return st;
        done += chunk;
    }
    c->k += n;
    return MICSA_OK;
}

// ------------------------------------------------------- replayable graphs
// The per-half paths (byte layout without the resident/fused kernels, and
// the bit-plane layout) launch 3 kernels per sweep, so small and mid-size
// lattices are bound by launch overhead.  Their sweeps are captured once per
// context as a graph of kGraphSweeps sweeps whose kernels take the sweep
// index from a device counter (refresh kernels that skip non-refresh
// sweeps, thresholds from the schedule tables) and replayed.
constexpr int kGraphSweeps = 16;

bool use_graph(const micsa_ctx* c)
{
    return c->use_graphs && !c->timing && c->gamma == 1 && (c->bit || (!use_resident(c) && !use_fused(c)));
}

// One sweep in device-counter form on stream st.
int enqueue_dev_sweep(micsa_ctx* c, int32_t algo, hipStream_t st)
{
    const int32_t P = c->sched.period;
    if (c->bit) {
        const int WL = word_lattices(c);
        kb_refresh_dev<<<dim3(bp_refresh_blocks(c->g), (unsigned)WL), 256, 0, st>>>(
            geomb(c), c->bdm0, c->bdm1, c->d_k, P, c->d_dth);
        const dim3 grid = grid_for(c->g.Nh, WL);
        kb_micsa_half<0><<<grid, kBlock, 0, st>>>(geomb(c), c->bspin, c->bdm0, c->bdm1, c->bJ);
        kb_micsa_half<1><<<grid, kBlock, 0, st>>>(geomb(c), c->bspin, c->bdm0, c->bdm1, c->bJ);
        c->tally_ok = false;
    } else {
        const int64_t words = (int64_t)c->g.rows * c->g.Wr;
        if (algo == MICSA_ALGO_MICSA) {
            k_refresh_dev<<<grid_for(c->g.Nh / 4, c->L), kBlock, 0, st>>>(c->g, c->dem, c->d_k, P, c->d_dth);
            k_micsa_half<0><<<grid_for(words, c->L), kBlock, 0, st>>>(c->g, c->spin, c->dem, c->tally, 0);
            k_micsa_half<1><<<grid_for(words, c->L), kBlock, 0, st>>>(c->g, c->spin, c->dem, c->tally, 0);
        } else {
            const HeatBathThresholds none{};
            enqueue_canonical_half<0>(c, algo, st, 0, none, c->d_k);
            enqueue_canonical_half<1>(c, algo, st, 0, none, c->d_k);
        }
    }
    k_count_sweep<<<1, 1, 0, st>>>(c->d_k);
    return check_launch(c, "device-counter sweep");
}

int sweep_graph(micsa_ctx* c, int32_t algo, int64_t n)
{
    const void* key = c->bit ? (const void*)c->bspin : (const void*)c->spin;
    hipGraphExec_t& ex = c->gexec[algo];
    if (ex && c->gkey[algo] != key) {  // state buffers moved since the capture
        (void)hipGraphExecDestroy(ex);
        ex = nullptr;
    }
    if (!c->d_k) HIP_TRY(c, hipMalloc(&c->d_k, 8));
    if (!ex && n >= kGraphSweeps) {
        if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        int st = MICSA_OK;
        for (int i = 0; i < kGraphSweeps && !st; ++i) st = enqueue_dev_sweep(c, algo, c->cap_stream);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
        if (st) return st;
        if (e != hipSuccess) return fail(c, MICSA_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
        const hipError_t e2 = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e2 != hipSuccess) {
            ex = nullptr;
            return fail(c, MICSA_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
        }
        c->gkey[algo] = key;
    }
    k_set_counter<<<1, 1, 0, c->stream>>>(c->d_k, c->k);
    int64_t done = 0;
    if (ex)
        for (; done + kGraphSweeps <= n; done += kGraphSweeps) HIP_TRY(c, hipGraphLaunch(ex, c->stream));
    for (; done < n; ++done) {
        const int st = enqueue_dev_sweep(c, algo, c->stream);
        if (st) return st;
    }
    c->k += n;
    return MICSA_OK;
}

// Checks shared by every sweep entry point.
int check_sweep(micsa_ctx* c, int32_t algo, int64_t n)
{
    if (algo != MICSA_ALGO_MICSA && algo != MICSA_ALGO_HEATBATH && algo != MICSA_ALGO_WALKERS &&
        algo != MICSA_ALGO_METROPOLIS)
        return fail(c, MICSA_EINVAL, "unknown algo");
    if (c->bit && algo == MICSA_ALGO_WALKERS) return fail(c, MICSA_EINVAL, "walkers run in the byte layout");
    if (c->bit && algo != MICSA_ALGO_MICSA)
        return fail(c, MICSA_EINVAL, "the heat-bath and Metropolis baselines run in the byte layout");
    if (n < 0) return fail(c, MICSA_EINVAL, "negative sweep count");
    if (!c->sched.set) return fail(c, MICSA_ESTATE, "no schedule installed");
    if (c->k + n > c->sched.n_sweeps) return fail(c, MICSA_ERANGE, "sweeps beyond the schedule length");
    return MICSA_OK;
}

// Wandering step of every walker family at the end of timestep t (each
// family along its own direction, the half of the cycle given by t's parity).
int launch_wander(micsa_ctx* c, int64_t t)
{
    const int64_t words = (int64_t)c->g.rows * c->g.Wr;
    {
        TimedLaunch tl(c, kTimeSweep);
        k_wander<<<grid_for(words, c->L * c->gamma), kBlock, 0, c->stream>>>(c->g, c->dem, c->dem_alt, (int)(t & 1));
    }
    const int st = check_launch(c, "k_wander");
    if (st) return st;
    std::swap(c->dem, c->dem_alt);
    return MICSA_OK;
}

// Tile of the one-launch multispin sweep: TY rows x TZ planes per work-group
// ((TY + 4) Lx / 128 lanes; the last tile along y holds the rows left over).
// Automatic TY: the most rows whose lanes, ring of 4 rows included, fill
// whole waves, up to three (Lx = 512: 44 rows, 192 lanes), so that no wave
// runs mostly empty; TZ divides Lz.
MscTile msc_tile(const micsa_ctx* c)
{
    const int W = c->p.Lx / 128;
    MscTile f{};
    if (c->tile_y) {
        f.TY = c->tile_y;
    } else {
        int rows = 0;
        for (int r = 5; r * W <= 192; ++r)
            if ((r * W) % 64 == 0) rows = r;
        f.TY = rows ? std::min(rows - 4, c->p.Ly) : divisor_at_most(c->p.Ly, std::max(1, 256 / W - 4));
    }
    f.TZ = c->tile_z ? c->tile_z : divisor_at_most(c->p.Lz, 8);
    f.nty = (c->p.Ly + f.TY - 1) / f.TY;
    f.ntz = c->p.Lz / f.TZ;
    f.xcd = c->xcd_map == 2 && f.ntz % 8 == 0 ? 2 : (c->xcd_map && (f.nty * f.ntz) % 8 == 0 ? 1 : 0);
    return f;
}

// Tile of the two-sweep multispin pass (msc2_kernels.hpp): (TY + 8) W lanes,
// whole waves up to two (Lx = 512: 24 rows, 128 lanes), and up to 16 planes,
// so that the march's ramp of six steps is a small share of it (at 512^3:
// 18.2 us per sweep, against 22.4 with 40 rows and 8 planes).
constexpr int kMscPassSweeps = 2;

MscTile msc2_tile(const micsa_ctx* c)
{
    const int W = c->p.Lx / 128, ring = 4 * kMscPassSweeps;
    MscTile f{};
    if (c->tile_y) {
        f.TY = c->tile_y;
    } else {
        int rows = 0;
        for (int r = ring + 1; r * W <= 128; ++r)
            if ((r * W) % 64 == 0) rows = r;
        f.TY = rows ? std::min(rows - ring, c->p.Ly) : std::max(1, std::min(c->p.Ly, kMsc2Lanes / W - ring));
    }
    f.TZ = c->tile_z ? c->tile_z : divisor_at_most(c->p.Lz, 16);
    f.nty = (c->p.Ly + f.TY - 1) / f.TY;
    f.ntz = c->p.Lz / f.TZ;
    f.xcd = c->xcd_map == 2 && f.ntz % 8 == 0 ? 2 : (c->xcd_map && (f.nty * f.ntz) % 8 == 0 ? 1 : 0);
    return f;
}

int msc2_block(const MscTile& f, int W) { return ((f.TY + 4 * kMscPassSweeps) * W + 63) / 64 * 64; }

size_t msc2_lds(const MscTile& f, int W) { return (size_t)8 * kMsc2Words * (size_t)(msc2_block(f, W) + W); }

// The pass fits a work-group: lanes and LDS (at most 96 KiB: one or two
// work-groups per CU).
bool msc2_fits(const micsa_ctx* c)
{
    const MscTile f = msc2_tile(c);
    const int W = c->p.Lx / 128;
    return c->msc_pass == 2 && msc2_block(f, W) <= kMsc2Lanes && msc2_lds(f, W) <= 96 * 1024;
}

bool msc_one_launch(const micsa_ctx* c)
{
    return c->msc_fused && ((msc_tile(c).TY + 4) * (c->p.Lx / 128) + 63) / 64 * 64 <= kMscSweepLanes;
}

constexpr int64_t kDrawBlocks = 1024;  // draw-ahead grid: one wave per SIMD, beside the sweeps


// Launch the draw of refresh sweep kr's levels on the side stream, after
// everything the library stream holds so far (the previous refresh sweep
// reads the same planes); the refresh sweep waits for draw_done.
// alone: nothing of the call runs beside the draw (a refresh at the call's
// first sweep), so it takes a full grid, a thread per word
int draw_levels(micsa_ctx* c, const MscGeom& m, int64_t kr, bool alone = false)
{
    const int64_t rho = refresh_index(kr, c->sched.period);
    const double T = temperature(c->sched, rho);
    if (!(T > 0.0) || !std::isfinite(T)) return fail(c, MICSA_ERANGE, "no temperature for this refresh");
    const int64_t total = (int64_t)c->L * m.plane;
    const unsigned blocks = (unsigned)(alone ? (total + 63) / 64 : std::min<int64_t>((total + 63) / 64, kDrawBlocks));
    HIP_TRY(c, hipEventRecord(c->draw_free, c->stream));
    HIP_TRY(c, hipStreamWaitEvent(c->draw_stream, c->draw_free, 0));
    k_msc_draw<<<blocks, 64, 0, c->draw_stream>>>(c->g, m, c->L, c->mdr0, c->mdr1, (uint32_t)rho,
                                                   daemon_thresholds(T));
    const int st = check_launch(c, "k_msc_draw");
    if (st) return st;
    HIP_TRY(c, hipEventRecord(c->draw_done, c->draw_stream));
    return MICSA_OK;
}

// First refresh sweep in [from, end), or -1.
int64_t next_refresh(const micsa_ctx* c, int64_t from, int64_t end)
{
    for (int64_t k = from; k < end; ++k)
        if (is_refresh(k, c->sched.period)) return k;
    return -1;
}

// MicSA sweeps k .. k + n - 1 on multispin planes: pack the byte state
// unless the planes are live, sweep (two sweeps per launch where the pass
// applies, else one launch per sweep marching along z, or one per half
// sweep; refresh levels drawn ahead on the side stream, or in the sweep),
// and leave the planes live.  Walkers (one-launch only): each sweep applies
// the previous timestep's wandering as it loads the levels; the last one is
// left owed to the byte layout (pend_wander).
MscGeom msc_geom(const micsa_ctx* c)
{
    MscGeom m;
    m.W = c->p.Lx / 128;
    m.R = c->g.rows;
    m.plane = (int64_t)m.R * m.W;
    return m;
}

// Unpack live multispin planes into the byte arrays (before anything reads
// or writes those).
int settle_msc(micsa_ctx* c)
{
    if (!c->msc_live) return MICSA_OK;
    const MscGeom m = msc_geom(c);
    const dim3 cgrid((unsigned)((2 * m.plane + 255) / 256), (unsigned)c->L);
    {
        TimedLaunch t(c, kTimeReduce);
        k_msc_unpack<<<cgrid, 256, 0, c->stream>>>(c->g, m, c->ms, c->md0, c->md1, c->mb, c->spin, c->dem);
    }
    const int st = check_launch(c, "k_msc_unpack");
    if (!st) c->msc_live = false;
    return st;
}

// The multispin planes a sweep call needs (the alternates for the one-launch
// sweep, the drawn levels for the draw ahead) and the draw stream.  A failed
// allocation frees only what this call allocated (the planes may hold the
// live state).
int msc_alloc(micsa_ctx* c, bool one, bool ahead)
{
    const MscGeom m = msc_geom(c);
    const size_t words = (size_t)c->L * 2 * (size_t)m.plane;
    std::vector<uint64_t**> fresh;
    auto get = [&](uint64_t** q, size_t n) {
        if (*q) return true;
        if (hipMalloc(q, n * 8) != hipSuccess) {
            *q = nullptr;
            return false;
        }
        fresh.push_back(q);
        return true;
    };
    bool ok = get(&c->ms, words) && get(&c->md0, words) && get(&c->md1, words) && get(&c->mb, words * 3);
    if (ok && one) ok = get(&c->ms_alt, words) && get(&c->md0_alt, words) && get(&c->md1_alt, words);
    if (ok && ahead) ok = get(&c->mdr0, words) && get(&c->mdr1, words);
    if (!ok) {
        (void)hipGetLastError();
        for (uint64_t** q : fresh) {
            (void)hipFree(*q);
            *q = nullptr;
        }
        return fail(c, MICSA_ENOMEM, "multispin planes");
    }
    if (ahead && !c->draw_stream) {
        HIP_TRY(c, hipStreamCreateWithFlags(&c->draw_stream, hipStreamNonBlocking));
        HIP_TRY(c, hipEventCreateWithFlags(&c->draw_free, hipEventDisableTiming));
        HIP_TRY(c, hipEventCreateWithFlags(&c->draw_done, hipEventDisableTiming));
    }
    return MICSA_OK;
}

// How far past the end of a call the next refresh's levels are drawn ahead
// (they are ready for the next call if it starts there).
constexpr int64_t kMscDrawWindow = 1024;

int sweep_msc(micsa_ctx* c, int64_t n, bool walkers = false)
{
    const MscGeom m = msc_geom(c);
    const size_t words = (size_t)c->L * 2 * (size_t)m.plane;
    const MscTile f = msc_tile(c);
    const int lanes = (f.TY + 4) * m.W;
    const bool one = msc_one_launch(c);
    const bool ahead = one && c->draw_ahead;
    (void)words;
    if (int st = msc_alloc(c, one, ahead)) return st;
    const dim3 cgrid((unsigned)((2 * m.plane + 255) / 256), (unsigned)c->L);
    int st = MICSA_OK;
    const int64_t k_end = c->k + n;
    int64_t drawn = -1;  // refresh sweep whose levels the draw planes hold (or are being drawn)
    // The first refresh of the call may have been drawn during the previous
    // one.  A refresh at the call's first sweep has no sweep of the call to
    // hide a draw behind: its levels (which depend on the schedule only) are
    // drawn by a full grid, enqueued before the pack so that the two run side
    // by side, and the call's first sweeps read them like any other.
    if (ahead && (drawn = next_refresh(c, c->k, k_end)) >= 0 && drawn != c->msc_drawn &&
        (st = draw_levels(c, m, drawn, drawn == c->k)))
        return st;
    c->msc_drawn = -1;
    if (!c->msc_live) {
        {
            TimedLaunch t(c, kTimeReduce);
            k_msc_pack<<<cgrid, 256, 0, c->stream>>>(c->g, m, c->spin, c->dem, c->ms, c->md0, c->md1, c->mb);
        }
        if ((st = check_launch(c, "k_msc_pack"))) return st;
    }
    const dim3 grid((unsigned)((m.plane + 255) / 256), (unsigned)c->L);
    const dim3 sgrid((unsigned)(f.nty * f.ntz), (unsigned)c->L);
    const unsigned sblock = (unsigned)((lanes + 63) / 64 * 64);
    const size_t slds = (size_t)96 * lanes;  // 6 planes x 2 step buffers x 8 B per lane
    for (int64_t i = 0; i < n; ++i) {
        const int64_t k = c->k;
        const bool refresh = is_refresh(k, c->sched.period);
        const int64_t rho = refresh_index(k, c->sched.period);
        const double T = temperature(c->sched, rho);
        if (!(T > 0.0) || !std::isfinite(T)) return fail(c, MICSA_ERANGE, "no temperature for this refresh");
        const DaemonThresholds th = refresh ? daemon_thresholds(T) : DaemonThresholds{0, 0, 0};
        // walkers pass their levels' carry words between the lanes of a row,
        // which share a wave when Lx / 128 divides 64
        if (one && (walkers ? 64 % m.W == 0 : c->pend_wander < 0) && i + 1 < n && msc2_fits(c)) {
            // sweeps k and k + 1 in one pass; a refresh among them reads its
            // drawn levels (at most one refresh per pass, drawn ahead)
            const bool refresh2 = is_refresh(k + 1, c->sched.period);
            const bool ok2 = (!refresh || (ahead && drawn == k)) && (!refresh2 || (ahead && drawn == k + 1)) &&
                             !(refresh && refresh2);
            if (ok2) {
                if (refresh || refresh2) HIP_TRY(c, hipStreamWaitEvent(c->stream, c->draw_done, 0));
                const MscTile f2 = msc2_tile(c);
                const dim3 grid2((unsigned)(f2.nty * f2.ntz), (unsigned)c->L);
                const unsigned block2 = (unsigned)msc2_block(f2, m.W);
                const size_t lds2 = msc2_lds(f2, m.W);
                const auto kern = walkers ? (refresh2 ? k_msc_sweep_multi<kMscPassSweeps, 1, true>
                                                      : k_msc_sweep_multi<kMscPassSweeps, -1, true>)
                                          : (refresh2 ? k_msc_sweep_multi<kMscPassSweeps, 1, false>
                                                      : k_msc_sweep_multi<kMscPassSweeps, -1, false>);
                if (lds2 > 64 * 1024 &&
                    hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2) !=
                        hipSuccess)
                    return fail(c, MICSA_EHIP, "k_msc_sweep_multi LDS attribute");
                Geom a_g = c->g;
                MscGeom a_m = m;
                MscTile a_f = f2;
                const uint64_t *a_s = c->ms, *a_d0 = refresh ? c->mdr0 : c->md0, *a_d1 = refresh ? c->mdr1 : c->md1,
                               *a_b = c->mb, *a_r0 = c->mdr0, *a_r1 = c->mdr1;
                uint64_t *o_s = c->ms_alt, *o_d0 = c->md0_alt, *o_d1 = c->md1_alt;
                unsigned long long* a_t = c->tally;
                // walkers: the wandering owed to sweep k's levels (none after a
                // refresh), and sweep k's own, applied before sweep k + 1 (none
                // when that one refreshes)
                int a_w = walkers && !refresh ? c->pend_wander : -1;
                int a_wA = walkers && !refresh2 ? (int)(k & 1) : -1;
                void* args[] = {&a_g, &a_m, &a_f, &a_s, &a_d0, &a_d1, &a_b, &a_r0, &a_r1, &o_s, &o_d0, &o_d1,
                                &a_t, &a_w, &a_wA};
                hipEvent_t e0 = nullptr, e1 = nullptr;
                if (c->timing && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) {
                    if (e0) (void)hipEventDestroy(e0);
                    e0 = e1 = nullptr;
                }
                const hipError_t le =
                    hipExtLaunchKernel((const void*)kern, grid2, block2, args, lds2, c->stream, e0, e1, 0);
                if (e0 && e1) {
                    if (le == hipSuccess) {
                        c->events[kTimeSweep].push_back({e0, e1});
                    } else {
                        (void)hipEventDestroy(e0);
                        (void)hipEventDestroy(e1);
                    }
                }
                if (le != hipSuccess)
                    return fail(c, MICSA_EHIP, std::string("k_msc_sweep_multi: ") + hipGetErrorString(le));
                if ((st = check_launch(c, "k_msc_sweep_multi"))) return st;
                if ((refresh || refresh2) && (drawn = next_refresh(c, k + 2, k_end)) >= 0 &&
                    (st = draw_levels(c, m, drawn)))
                    return st;
                std::swap(c->ms, c->ms_alt);
                std::swap(c->md0, c->md0_alt);
                std::swap(c->md1, c->md1_alt);
                // gamma = 1: sweep k + 1 is timestep k + 1; walkers owe its wandering
                c->pend_wander = walkers ? (int32_t)((k + 1) & 1) : -1;
                c->k = k + 2;
                ++i;
                continue;
            }
        }
        if (one) {
            // a refresh sweep with levels drawn ahead is a plain sweep reading them
            const bool use_drawn = refresh && ahead && drawn == k;
            if (use_drawn) HIP_TRY(c, hipStreamWaitEvent(c->stream, c->draw_done, 0));
            {
                const bool fresh = refresh && !use_drawn, walk = !refresh && c->pend_wander >= 0;
                const auto kern = fresh  ? k_msc_sweep<true, 0>
                                  : walk ? (64 % m.W == 0 ? k_msc_sweep<false, 1> : k_msc_sweep<false, 2>)
                                         : k_msc_sweep<false, 0>;
                // arguments typed as the kernel declares them
                Geom a_g = c->g;
                MscGeom a_m = m;
                MscTile a_f = f;
                const uint64_t *a_s = c->ms, *a_d0 = use_drawn ? c->mdr0 : c->md0,
                               *a_d1 = use_drawn ? c->mdr1 : c->md1, *a_b = c->mb;
                uint64_t *o_s = c->ms_alt, *o_d0 = c->md0_alt, *o_d1 = c->md1_alt;
                unsigned long long* a_t = c->tally;
                uint32_t a_rho = (uint32_t)rho;
                DaemonThresholds a_th = th;
                int a_w = refresh ? -1 : c->pend_wander;
                void* args[] = {&a_g,  &a_m, &a_f, &a_s, &a_d0,  &a_d1, &a_b,
                                &o_s,  &o_d0, &o_d1, &a_t, &a_rho, &a_th, &a_w};
                // with timing on, the events belong to the dispatch itself and
                // time the kernel alone (separate event packets around it add
                // a few microseconds per launch)
                hipEvent_t e0 = nullptr, e1 = nullptr;
                if (c->timing && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) {
                    if (e0) (void)hipEventDestroy(e0);
                    e0 = e1 = nullptr;
                }
                const hipError_t le =
                    hipExtLaunchKernel((const void*)kern, sgrid, sblock, args, slds, c->stream, e0, e1, 0);
                if (e0 && e1) {
                    if (le == hipSuccess) {
                        c->events[kTimeSweep].push_back({e0, e1});
                    } else {
                        (void)hipEventDestroy(e0);
                        (void)hipEventDestroy(e1);
                    }
                }
                if (le != hipSuccess) return fail(c, MICSA_EHIP, std::string("k_msc_sweep: ") + hipGetErrorString(le));
            }
            if ((st = check_launch(c, "k_msc_sweep"))) return st;
            // after a refresh: the next one, in this call or (within the
            // window) a later one
            if (refresh && ahead &&
                (drawn = next_refresh(c, k + 1, std::min(c->sched.n_sweeps, k_end + kMscDrawWindow))) >= 0 &&
                (st = draw_levels(c, m, drawn)))
                return st;
            std::swap(c->ms, c->ms_alt);
            std::swap(c->md0, c->md0_alt);
            std::swap(c->md1, c->md1_alt);
            // gamma = 1: sweep k is timestep k; walkers owe its wandering to the next load
            c->pend_wander = walkers ? (int32_t)(k & 1) : -1;
            c->k = k + 1;
            continue;
        }
        {
            TimedLaunch t(c, kTimeSweep);
            if (refresh)
                k_msc_half<0, true><<<grid, 256, 0, c->stream>>>(c->g, m, c->ms, c->md0, c->md1, c->mb, c->tally,
                                                                (uint32_t)rho, th);
            else
                k_msc_half<0, false><<<grid, 256, 0, c->stream>>>(c->g, m, c->ms, c->md0, c->md1, c->mb, c->tally,
                                                                 (uint32_t)rho, th);
        }
        if ((st = check_launch(c, "k_msc_half<0>"))) return st;
        {
            TimedLaunch t(c, kTimeSweep);
            if (refresh)
                k_msc_half<1, true><<<grid, 256, 0, c->stream>>>(c->g, m, c->ms, c->md0, c->md1, c->mb, c->tally,
                                                                (uint32_t)rho, th);
            else
                k_msc_half<1, false><<<grid, 256, 0, c->stream>>>(c->g, m, c->ms, c->md0, c->md1, c->mb, c->tally,
                                                                 (uint32_t)rho, th);
        }
        if ((st = check_launch(c, "k_msc_half<1>"))) return st;
        c->k = k + 1;
    }
    // the planes stay live (unpacked when the byte arrays are next needed); a
    // draw for a refresh after this call is joined into the library stream
    // here and kept for the call that starts there
    c->msc_live = true;
    if (ahead && drawn >= k_end) {
        HIP_TRY(c, hipStreamWaitEvent(c->stream, c->draw_done, 0));
        c->msc_drawn = drawn;
    }
    return MICSA_OK;
}

// Apply a wandering the daemons still owe (walkers on the fused sweep).
int settle_wander(micsa_ctx* c)
{
    if (c->pend_wander < 0) return MICSA_OK;
    if (int st = settle_msc(c)) return st;  // the wandering kernel moves the byte arrays' levels
    const int p = c->pend_wander;
    c->pend_wander = -1;
    return launch_wander(c, p);
}

int sweep_impl(micsa_ctx* c, int32_t algo, int64_t n)
{
    if (!c) return MICSA_EINVAL;
    int st0 = check_sweep(c, algo, n);
    if (st0) return st0;
    // walkers (gamma = 1) on the fused sweep carry their wandering into the
    // next sweep's loads; every other path needs the daemons in place
    const bool walk_msc = algo == MICSA_ALGO_WALKERS && use_msc(c, n, algo);
    const bool walk_fused = algo == MICSA_ALGO_WALKERS && !c->bit && c->gamma == 1 && use_fused(c);
    // the one-launch multispin sweep takes an owed wandering on its loads
    // (and leaves one), as the fused byte sweep does
    if (!walk_fused && !walk_msc && !(algo == MICSA_ALGO_MICSA && use_msc(c, n) && msc_one_launch(c)) &&
        (st0 = settle_wander(c)))
        return st0;
    if (walk_msc) return n > 0 ? sweep_msc(c, n, true) : MICSA_OK;
    if (algo == MICSA_ALGO_MICSA && use_msc(c, n)) return n > 0 ? sweep_msc(c, n) : MICSA_OK;
    // every other path sweeps the byte arrays
    if ((st0 = settle_msc(c))) return st0;
    if (algo != MICSA_ALGO_WALKERS) {
        if (use_resident(c)) return launch_resident(c, algo, n, nullptr, 0);
        if (use_graph(c) && n >= kGraphSweeps) return sweep_graph(c, algo, n);
    }
    if (algo == MICSA_ALGO_MICSA && bp_one_launch(c)) return sweep_bitplane(c, n);
    if (algo == MICSA_ALGO_MICSA && use_slab(c)) return sweep_slab(c, n);
    for (int64_t i = 0; i < n; ++i) {
        // sweep k is sweep fam of timestep t (Sec. 2.8)
        const int64_t k = c->k;
        const int64_t t = k / c->gamma;
        const int fam = (int)(k - t * c->gamma);
        const int64_t rho = refresh_index(t, c->sched.period);
        const double T = temperature(c->sched, rho);
        if (!(T > 0.0) || !std::isfinite(T)) return fail(c, MICSA_ERANGE, "no temperature for this refresh");
        int st;
        if (walk_fused && c->temporal == 2 && i + 1 < n && sweep2_walk_eligible(c)) {
            // timesteps t and t + 1 (gamma = 1) in one pass, wandering between them in registers
            const bool refreshB = is_refresh(t + 1, c->sched.period);
            const int64_t rhoB = refresh_index(t + 1, c->sched.period);
            const double TB = temperature(c->sched, rhoB);
            if (!(TB > 0.0) || !std::isfinite(TB)) return fail(c, MICSA_ERANGE, "no temperature for this refresh");
            if ((st = launch_fused_sweep2(c, is_refresh(t, c->sched.period), rho, T, refreshB, rhoB, TB, true,
                                          c->pend_wander, (int)(t & 1))))
                return st;
            c->pend_wander = (int32_t)((t + 1) & 1);
            c->k = k + 2;
            ++i;
            continue;
        }
        if (algo == MICSA_ALGO_MICSA && c->temporal == 2 && i + 1 < n && use_fused(c) && sweep2_eligible(c)) {
            // sweeps k and k + 1 in one pass (gamma = 1 on the fused path)
            const bool refreshB = is_refresh(k + 1, c->sched.period);
            const int64_t rhoB = refresh_index(k + 1, c->sched.period);
            const double TB = temperature(c->sched, rhoB);
            if (!(TB > 0.0) || !std::isfinite(TB)) return fail(c, MICSA_ERANGE, "no temperature for this refresh");
            if ((st = launch_fused_sweep2(c, is_refresh(k, c->sched.period), rho, T, refreshB, rhoB, TB))) return st;
            c->k = k + 2;
            ++i;
            continue;
        }
        if (algo == MICSA_ALGO_MICSA || algo == MICSA_ALGO_WALKERS) {
            const bool refresh = fam == 0 && is_refresh(t, c->sched.period);
            if (c->bit) {
                if ((st = launch_bitplane_sweep(c, refresh, rho, T))) return st;
            } else if (walk_fused) {
                // a refresh redraws every daemon, so an owed wandering lapses
                if ((st = launch_fused_sweep(c, refresh, rho, T, c->pend_wander))) return st;
                c->pend_wander = (int32_t)(t & 1);  // this timestep's wandering, owed to the next sweep
            } else if (use_fused(c)) {
                if ((st = launch_fused_sweep(c, refresh, rho, T))) return st;
            } else {
                if (refresh && (st = launch_refresh(c, rho, T))) return st;
                if ((st = launch_micsa_sweep(c, fam))) return st;
            }
            if (algo == MICSA_ALGO_WALKERS && !walk_fused && fam == c->gamma - 1 && (st = launch_wander(c, t)))
                return st;
        } else {
            if ((st = launch_canonical_sweep(c, algo, k, T))) return st;
        }
        c->k = k + 1;
    }
    return MICSA_OK;
}

void free_all(micsa_ctx* c)
{
    if (!c) return;
    if (c->spin) (void)hipFree(c->spin);
    if (c->dem) (void)hipFree(c->dem);
    if (c->spin_alt) (void)hipFree(c->spin_alt);
    for (uint8_t* q : c->sdr)
        if (q) (void)hipFree(q);
    if (c->dem_alt) (void)hipFree(c->dem_alt);
    if (c->bspin) (void)hipFree(c->bspin);
    if (c->draw_stream) (void)hipStreamSynchronize(c->draw_stream);
    for (uint64_t* q : {c->ms, c->md0, c->md1, c->mb, c->ms_alt, c->md0_alt, c->md1_alt, c->mdr0, c->mdr1})
        if (q) (void)hipFree(q);
    if (c->draw_free) (void)hipEventDestroy(c->draw_free);
    if (c->draw_done) (void)hipEventDestroy(c->draw_done);
    if (c->draw_stream) (void)hipStreamDestroy(c->draw_stream);
    if (c->bdm0) (void)hipFree(c->bdm0);
    for (uint64_t* q : {c->bspin_alt, c->bdm0_alt, c->bdm1_alt, c->bdr0, c->bdr1})
        if (q) (void)hipFree(q);
    if (c->bdm1) (void)hipFree(c->bdm1);
    if (c->bJ) (void)hipFree(c->bJ);
    if (c->d_dth) (void)hipFree(c->d_dth);
    if (c->d_hth) (void)hipFree(c->d_hth);
    if (c->d_mth) (void)hipFree(c->d_mth);
    for (auto& e : c->gexec)
        if (e) (void)hipGraphExecDestroy(e);
    if (c->d_k) (void)hipFree(c->d_k);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->tally) (void)hipFree(c->tally);
    if (c->red) (void)hipFree(c->red);
    if (c->logslots) (void)hipFree(c->logslots);
    if (c->rlog) (void)hipFree(c->rlog);
    for (auto& v : c->events)
        for (auto& e : v) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
}

// Parameters a context accepts (include/micsa.h, micsa_create).
bool params_ok(const micsa_params* p)
{
    if (p->Lx < 8 || p->Lx % 8 || p->Ly < 2 || p->Ly % 2 || p->Lz < 2 || p->Lz % 2) return false;
    if (p->n_samples < 1 || p->n_samples >= (1 << 24) || p->n_replicas < 1) return false;
    if (p->layout != MICSA_LAYOUT_BYTE && p->layout != MICSA_LAYOUT_BITPLANE) return false;
    const int64_t N = (int64_t)p->Lx * p->Ly * p->Lz;
    if (N >= ((int64_t)1 << 32) || (int64_t)p->n_samples * p->n_replicas >= (1 << 16)) return false;
    const int gamma = p->gamma == 0 ? 1 : p->gamma;
    if (gamma < 1 || gamma > 6 || (gamma > 1 && p->layout != MICSA_LAYOUT_BYTE)) return false;
    if (p->lane_mode != MICSA_LANES_SAMPLES && p->lane_mode != MICSA_LANES_REPLICAS) return false;
    if (p->lane_mode == MICSA_LANES_REPLICAS && p->layout != MICSA_LAYOUT_BITPLANE) return false;
    return (int64_t)gamma * N / 4 < ((int64_t)1 << 32);  // daemon counters (a*N + i) >> 2 fit 32 bits
}

}  // namespace

// =================================================================== C ABI
extern "C" {

const char* micsa_status_string(int status)
{
    switch (status) {
    case MICSA_OK: return "ok";
    case MICSA_EINVAL: return "invalid argument";
    case MICSA_ENOMEM: return "out of device memory";
    case MICSA_EHIP: return "HIP runtime error";
    case MICSA_ESTATE: return "invalid state";
    case MICSA_ERANGE: return "out of range";
    default: return "unknown status";
    }
}

const char* micsa_last_error(const micsa_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int micsa_create(const micsa_params* p, void* hip_stream, micsa_ctx** out)
{
    if (!out) return MICSA_EINVAL;
    *out = nullptr;
    if (!p) return MICSA_EINVAL;
    if (!params_ok(p)) return MICSA_EINVAL;
    const int64_t N = (int64_t)p->Lx * p->Ly * p->Lz;
    const int gamma = p->gamma == 0 ? 1 : p->gamma;

    micsa_ctx* c = new (std::nothrow) micsa_ctx();
    if (!c) return MICSA_ENOMEM;
    if (hipGetDevice(&c->device) != hipSuccess) {
        (void)hipGetLastError();
        delete c;
        return MICSA_EHIP;
    }
    if (hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) {
        (void)hipGetLastError();
        c->cus = 0;
    }
    c->p = *p;
    c->p.gamma = gamma;
    c->gamma = gamma;
    c->stream = (hipStream_t)hip_stream;
    c->L = p->n_samples * p->n_replicas;
    c->bit = p->layout == MICSA_LAYOUT_BITPLANE;
    // the bit-plane sweep is latency-bound: a draw beside it slows it more
    // than the draw costs in place (measured on MI355X), so it draws in place
    if (c->bit) c->draw_ahead = 0;
    c->G = p->lane_mode == MICSA_LANES_REPLICAS ? (p->n_replicas + 63) / 64 : (p->n_samples + 63) / 64;
    Geom& g = c->g;
    g.Lx = p->Lx;
    g.Ly = p->Ly;
    g.Lz = p->Lz;
    g.Kx = p->Lx / 2;
    g.Wr = g.Kx / 4;
    g.rows = p->Ly * p->Lz;
    g.Nh = N / 2;
    g.S = p->n_samples;
    g.R = p->n_replicas;
    g.key0 = (uint32_t)p->seed;
    g.key1 = (uint32_t)(p->seed >> 32);
    g.gamma = gamma;

    const size_t nred = (size_t)std::max(c->L, p->n_samples);
    bool ok = hipMalloc(&c->tally, (size_t)c->L * kSlots * 8) == hipSuccess &&
              hipMalloc(&c->red, nred * kSlots * 8) == hipSuccess;
    const size_t state = (size_t)c->L * 2 * (size_t)g.Nh;
    const size_t dstate = state * (size_t)gamma;  // every daemon family
    const size_t words = (size_t)word_lattices(c) * 2 * (size_t)g.Nh;
    if (ok && !c->bit) {
        ok = hipMalloc(&c->spin, state) == hipSuccess && hipMalloc(&c->dem, dstate) == hipSuccess &&
             hipMalloc(&c->spin_alt, state) == hipSuccess && hipMalloc(&c->dem_alt, dstate) == hipSuccess;
    } else if (ok) {
        ok = hipMalloc(&c->bspin, words * 8) == hipSuccess && hipMalloc(&c->bdm0, words * 8) == hipSuccess &&
             hipMalloc(&c->bdm1, words * 8) == hipSuccess &&
             hipMalloc(&c->bJ, (size_t)bp_coupling_sets(geomb(c)) * 6 * (size_t)g.Nh * 8) == hipSuccess;
    }
    if (!ok) {
        (void)hipGetLastError();
        free_all(c);
        delete c;
        return MICSA_ENOMEM;
    }
    int st = MICSA_OK;
    if (!c->bit) {
        // spins first, then the bond bits into the even spin bytes
        k_init_spins<<<grid_for(g.Nh / 4, c->L), kBlock, 0, c->stream>>>(g, c->spin);
        st = check_launch(c, "k_init_spins");
        if (!st) st = enqueue_bonds(c);
        if (!st && hipMemsetAsync(c->dem, 0, dstate, c->stream) != hipSuccess) st = MICSA_EHIP;
    } else {
        const int WL = word_lattices(c);
        kb_init_couplings<<<dim3((unsigned)((g.Nh + 3) / 4), (unsigned)bp_coupling_sets(geomb(c))), 256, 0,
                            c->stream>>>(geomb(c), c->bJ);
        st = check_launch(c, "kb_init_couplings");
        if (!st) {
            kb_init_spins<<<dim3((unsigned)((g.Nh / 2 + 3) / 4), (unsigned)WL), 256, 0, c->stream>>>(geomb(c),
                                                                                               c->bspin);
            st = check_launch(c, "kb_init_spins");
        }
        if (!st && (hipMemsetAsync(c->bdm0, 0, words * 8, c->stream) != hipSuccess ||
                    hipMemsetAsync(c->bdm1, 0, words * 8, c->stream) != hipSuccess))
            st = MICSA_EHIP;
    }
    if (!st) {
        // tally <- from-scratch energy (2U - 3N)
        std::vector<int64_t> U;
        st = enqueue_energy(c, c->red);
        if (!st) st = read_slots(c, c->red, c->L, U);
        if (!st) {
            for (auto& u : U) u = 2 * u - 3 * N;
            st = set_tally(c, U);
        }
    }
    if (st) {
        free_all(c);
        delete c;
        return st;
    }
    // the working buffers of the sweep path the lattice takes by default
    // (counted in the pool footprint), so that the first sweep call does not
    // allocate; if they do not fit now, that call tries again
    if (!c->bit && c->gamma == 1 && msc_eligible(c) && !resident_eligible(c)) {
        if (msc_alloc(c, true, true) != MICSA_OK) c->err.clear();
    } else if (use_slab(c) && slab_pairs(c)) {
        if (slab_alloc(c) != MICSA_OK) c->err.clear();
    }
    *out = c;
    return MICSA_OK;
}

int micsa_destroy(micsa_ctx* ctx)
{
    if (!ctx) return MICSA_OK;
    (void)hipStreamSynchronize(ctx->stream);
    free_all(ctx);
    delete ctx;
    return MICSA_OK;
}

int micsa_set_schedule(micsa_ctx* ctx, const micsa_schedule* s)
{
    if (!ctx) return MICSA_EINVAL;
    if (!s) return fail(ctx, MICSA_EINVAL, "null schedule");
    if (s->refresh_period < 0) return fail(ctx, MICSA_EINVAL, "refresh_period < 0");
    if (s->n_sweeps < 0) return fail(ctx, MICSA_EINVAL, "n_sweeps < 0");
    Schedule n;
    n.set = true;
    n.kind = s->kind;
    n.period = s->refresh_period;
    n.T0 = s->T0;
    n.T1 = s->T1;
    n.n_sweeps = s->n_sweeps;
    n.n_steps = (s->n_sweeps + ctx->gamma - 1) / ctx->gamma;
    auto okT = [](double T) { return T > 0.0 && std::isfinite(T); };
    if (s->kind == MICSA_SCHED_CONST) {
        if (!okT(s->T0)) return fail(ctx, MICSA_EINVAL, "T0 must be positive and finite");
    } else if (s->kind == MICSA_SCHED_LINEAR) {
        if (!okT(s->T0) || !okT(s->T1)) return fail(ctx, MICSA_EINVAL, "T0, T1 must be positive and finite");
    } else if (s->kind == MICSA_SCHED_TABLE) {
        if (!s->T_table || s->T_len < refresh_count(n))
            return fail(ctx, MICSA_EINVAL, "T_table must cover every refresh of the schedule");
        n.table.assign(s->T_table, s->T_table + s->T_len);
        for (double T : n.table)
            if (!okT(T)) return fail(ctx, MICSA_EINVAL, "table temperatures must be positive and finite");
    } else {
        return fail(ctx, MICSA_EINVAL, "unknown schedule kind");
    }
    // threshold tables for every refresh of the schedule (used by the resident sweeps)
    const int64_t nrho = std::max<int64_t>(refresh_count(n), 1);
    std::vector<DaemonThresholds> dth((size_t)nrho);
    std::vector<HeatBathThresholds> hth((size_t)nrho);
    std::vector<MetropolisThresholds> mth((size_t)nrho);
    for (int64_t rho = 0; rho < nrho; ++rho) {
        const double T = temperature(n, rho);
        dth[(size_t)rho] = daemon_thresholds(T);
        hth[(size_t)rho] = heatbath_thresholds(T);
        mth[(size_t)rho] = metropolis_thresholds(T);
    }
    DaemonThresholds* d1 = nullptr;
    HeatBathThresholds* d2 = nullptr;
    MetropolisThresholds* d3 = nullptr;
    if (hipMalloc(&d1, dth.size() * sizeof(DaemonThresholds)) != hipSuccess ||
        hipMalloc(&d2, hth.size() * sizeof(HeatBathThresholds)) != hipSuccess ||
        hipMalloc(&d3, mth.size() * sizeof(MetropolisThresholds)) != hipSuccess) {
        (void)hipGetLastError();
        if (d1) (void)hipFree(d1);
        if (d2) (void)hipFree(d2);
        return fail(ctx, MICSA_ENOMEM, "schedule tables");
    }
    HIP_TRY(ctx, hipMemcpyAsync(d1, dth.data(), dth.size() * sizeof(DaemonThresholds), hipMemcpyHostToDevice,
                                ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(d2, hth.data(), hth.size() * sizeof(HeatBathThresholds), hipMemcpyHostToDevice,
                                ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(d3, mth.data(), mth.size() * sizeof(MetropolisThresholds), hipMemcpyHostToDevice,
                                ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->d_dth) (void)hipFree(ctx->d_dth);
    if (ctx->d_hth) (void)hipFree(ctx->d_hth);
    if (ctx->d_mth) (void)hipFree(ctx->d_mth);
    for (auto& e : ctx->gexec)  // captured graphs point at the old tables
        if (e) {
            (void)hipGraphExecDestroy(e);
            e = nullptr;
        }
    ctx->d_dth = d1;
    ctx->d_hth = d2;
    ctx->d_mth = d3;
    ctx->sched = std::move(n);
    ctx->sdr_k[0] = ctx->sdr_k[1] = -1;  // levels drawn ahead under the old temperatures
    ctx->msc_drawn = -1;
    return MICSA_OK;
}

int micsa_sweep(micsa_ctx* ctx, int32_t algo, int64_t n) { return sweep_impl(ctx, algo, n); }

int micsa_sweep_logged_d(micsa_ctx* ctx, int32_t algo, int64_t n, int64_t stride, int64_t* E_log,
                         int64_t* D_log)
{
    if (!ctx) return MICSA_EINVAL;
    if (stride < 1) return fail(ctx, MICSA_EINVAL, "stride must be >= 1");
    if (!ctx->sched.set) return fail(ctx, MICSA_ESTATE, "no schedule installed");
    if (n < 0 || ctx->k + n > ctx->sched.n_sweeps) return fail(ctx, MICSA_ERANGE, "sweeps beyond the schedule");
    const int64_t rows = n / stride;
    const int L = ctx->L;
    const int64_t N = n_sites(ctx);
    int st = check_sweep(ctx, algo, n);
    if (st) return st;
    if (rows == 0 || (!E_log && !D_log)) return sweep_impl(ctx, algo, n);
    if (use_resident(ctx) && algo != MICSA_ALGO_WALKERS) {
        const size_t need = (size_t)rows * L * 2;
        if (need > ctx->rlog_cap) {
            // the old buffer may still be in use by enqueued work
            if (ctx->rlog) {
                HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
                (void)hipFree(ctx->rlog);
                ctx->rlog = nullptr;
                ctx->rlog_cap = 0;
            }
            if (hipMalloc(&ctx->rlog, need * 8) != hipSuccess) {
                (void)hipGetLastError();
                ctx->rlog = nullptr;
                return fail(ctx, MICSA_ENOMEM, "log buffer");
            }
            ctx->rlog_cap = need;
        }
        if ((st = launch_resident(ctx, algo, n, ctx->rlog, stride))) return st;
        const int64_t e = rows * L;
        k_log_from_pairs<<<(unsigned)((e + 255) / 256), 256, 0, ctx->stream>>>(
            ctx->rlog, e, N, reinterpret_cast<long long*>(E_log), reinterpret_cast<long long*>(D_log));
        return check_launch(ctx, "k_log_from_pairs");
    }
    if (!ctx->logslots && hipMalloc(&ctx->logslots, (size_t)2 * L * kSlots * 8) != hipSuccess) {
        (void)hipGetLastError();
        ctx->logslots = nullptr;
        return fail(ctx, MICSA_ENOMEM, "log slots");
    }
    unsigned long long* U = ctx->logslots;
    unsigned long long* Ms = ctx->logslots + (size_t)L * kSlots;
    for (int64_t r = 0; r < rows; ++r) {
        if ((st = sweep_impl(ctx, algo, stride))) return st;
        if (E_log && (st = enqueue_energy(ctx, U))) return st;
        if (D_log && (st = enqueue_level_sum(ctx, Ms))) return st;
        k_log_from_slots<<<(unsigned)((L + 255) / 256), 256, 0, ctx->stream>>>(
            U, Ms, L, N, E_log ? reinterpret_cast<long long*>(E_log + r * L) : nullptr,
            D_log ? reinterpret_cast<long long*>(D_log + r * L) : nullptr);
        if ((st = check_launch(ctx, "k_log_from_slots"))) return st;
    }
    return n > rows * stride ? sweep_impl(ctx, algo, n - rows * stride) : MICSA_OK;
}

int micsa_sweep_logged(micsa_ctx* ctx, int32_t algo, int64_t n, int64_t stride, int64_t* E_log, int64_t* D_log)
{
    if (!ctx) return MICSA_EINVAL;
    if (stride < 1) return fail(ctx, MICSA_EINVAL, "stride must be >= 1");
    if (!ctx->sched.set) return fail(ctx, MICSA_ESTATE, "no schedule installed");
    if (n < 0 || ctx->k + n > ctx->sched.n_sweeps) return fail(ctx, MICSA_ERANGE, "sweeps beyond the schedule");
    const int64_t rows = n / stride;
    const int L = ctx->L;
    int st0 = check_sweep(ctx, algo, n);
    if (st0) return st0;
    if (use_resident(ctx) && algo != MICSA_ALGO_WALKERS) {
        long long* rlog = nullptr;
        if (rows > 0 && hipMalloc(&rlog, (size_t)rows * L * 2 * 8) != hipSuccess) {
            (void)hipGetLastError();
            return fail(ctx, MICSA_ENOMEM, "log buffer");
        }
        int st = launch_resident(ctx, algo, n, rows > 0 ? rlog : nullptr, stride);
        std::vector<int64_t> h((size_t)rows * L * 2);
        if (!st && rows > 0 &&
            hipMemcpyAsync(h.data(), rlog, h.size() * 8, hipMemcpyDeviceToHost, ctx->stream) != hipSuccess)
            st = fail(ctx, MICSA_EHIP, "log copy");
        if (!st && hipStreamSynchronize(ctx->stream) != hipSuccess) st = fail(ctx, MICSA_EHIP, "sync");
        if (rlog) (void)hipFree(rlog);
        if (st) return st;
        const int64_t N = n_sites(ctx);
        for (int64_t r = 0; r < rows; ++r)
            for (int l = 0; l < L; ++l) {
                if (E_log) E_log[r * L + l] = 2 * h[(size_t)((r * L + l) * 2)] - 3 * N;
                if (D_log) D_log[r * L + l] = 4 * h[(size_t)((r * L + l) * 2 + 1)];
            }
        return MICSA_OK;
    }
    unsigned long long* dlog = nullptr;
    const size_t row_len = (size_t)L * 2 * kSlots;
    if (rows > 0 && hipMalloc(&dlog, (size_t)rows * row_len * 8) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, MICSA_ENOMEM, "log buffer");
    }
    int st = MICSA_OK;
    int64_t done = 0;
    for (int64_t r = 0; r < rows && !st; ++r) {
        st = sweep_impl(ctx, algo, stride);
        done += stride;
        if (!st) st = enqueue_energy(ctx, dlog + (size_t)r * row_len);
        if (!st) st = enqueue_level_sum(ctx, dlog + (size_t)r * row_len + (size_t)L * kSlots);
    }
    if (!st && n > done) st = sweep_impl(ctx, algo, n - done);
    std::vector<int64_t> h;
    if (!st && rows > 0) st = read_slots(ctx, dlog, rows * L * 2, h);
    if (!st && hipStreamSynchronize(ctx->stream) != hipSuccess) st = fail(ctx, MICSA_EHIP, "sync");
    if (dlog) (void)hipFree(dlog);
    if (st) return st;
    const int64_t N = n_sites(ctx);
    for (int64_t r = 0; r < rows; ++r)
        for (int l = 0; l < L; ++l) {
            if (E_log) E_log[r * L + l] = 2 * h[(size_t)(r * L * 2 + l)] - 3 * N;
            if (D_log) D_log[r * L + l] = 4 * h[(size_t)(r * L * 2 + L + l)];
        }
    return MICSA_OK;
}

int micsa_sync(micsa_ctx* ctx)
{
    if (!ctx) return MICSA_EINVAL;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return MICSA_OK;
}

static int read_red(micsa_ctx* c, int64_t n, std::vector<int64_t>& out) { return read_slots(c, c->red, n, out); }

int micsa_read_energy(micsa_ctx* ctx, int64_t* E)
{
    if (!ctx || !E) return MICSA_EINVAL;
    int st = enqueue_energy(ctx, ctx->red);
    std::vector<int64_t> U;
    if (st || (st = read_red(ctx, ctx->L, U))) return st;
    const int64_t N = n_sites(ctx);
    for (int l = 0; l < ctx->L; ++l) E[l] = 2 * U[(size_t)l] - 3 * N;
    return MICSA_OK;
}

int micsa_read_energy_tally(micsa_ctx* ctx, int64_t* E)
{
    if (!ctx || !E) return MICSA_EINVAL;
    if (ctx->bit && !ctx->tally_ok)
        return fail(ctx, MICSA_ESTATE, "the bit-plane tally is kept by the one-launch sweep only (a per-half "
                                       "sweep ran since the spins were last set)");
    std::vector<int64_t> v;
    int st = read_slots(ctx, ctx->tally, ctx->L, v);
    if (st) return st;
    for (int l = 0; l < ctx->L; ++l) E[l] = v[(size_t)l];
    return MICSA_OK;
}

int micsa_read_demon_energy(micsa_ctx* ctx, int64_t* D)
{
    if (!ctx || !D) return MICSA_EINVAL;
    int st = enqueue_level_sum(ctx, ctx->red);
    std::vector<int64_t> v;
    if (st || (st = read_red(ctx, ctx->L, v))) return st;
    for (int l = 0; l < ctx->L; ++l) D[l] = 4 * v[(size_t)l];
    return MICSA_OK;
}

// D[s][mu][r] = #{(pair, x) : w_x != w_{x + r e_mu}} summed over the replica
// pairs of sample s (observables.hpp), for r = 0 .. rmax.
static int c4_counts(micsa_ctx* c, const C4Geom& cg, std::vector<int64_t>& D)
{
    const int64_t ent = (int64_t)c->p.n_samples * 3 * (cg.rmax + 1);
    const int64_t per_pair = (int64_t)2 * c->g.rows * cg.E;
    const int64_t total = (int64_t)c->p.n_samples * cg.npair;
    const int64_t budget_words = ((int64_t)256 << 20) / 4;  // at most 256 MiB of packed pairs at a time
    const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>({total, budget_words / per_pair, 65535}));
    unsigned long long* dD = nullptr;
    uint32_t* Q = nullptr;
    if (hipMalloc(&dD, (size_t)ent * kSlots * 8) != hipSuccess ||
        hipMalloc(&Q, (size_t)(chunk * per_pair) * 4) != hipSuccess) {
        (void)hipGetLastError();
        if (dD) (void)hipFree(dD);
        return fail(c, MICSA_ENOMEM, "correlation buffers");
    }
    int st = zero_slots(c, dD, ent);
    const int64_t valid = (int64_t)2 * c->g.rows * cg.Wv;
    for (int64_t sp0 = 0; sp0 < total && !st; sp0 += chunk) {
        const unsigned n = (unsigned)std::min(chunk, total - sp0);
        {
            TimedLaunch t(c, kTimeReduce);
            if (c->bit)
                k_pack_overlap<true><<<dim3((unsigned)((per_pair + 255) / 256), n), 256, 0, c->stream>>>(
                    geomb(c), cg, (int)sp0, nullptr, c->bspin, Q);
            else
                k_pack_overlap<false><<<dim3((unsigned)((per_pair + 255) / 256), n), 256, 0, c->stream>>>(
                    geomb(c), cg, (int)sp0, c->spin, nullptr, Q);
        }
        if ((st = check_launch(c, "k_pack_overlap"))) break;
        {
            TimedLaunch t(c, kTimeReduce);
            k_c4_count<<<dim3((unsigned)((valid + 255) / 256), (unsigned)(3 * (cg.rmax + 1)), n), 256, 0,
                         c->stream>>>(c->g, cg, (int)sp0, Q, dD);
        }
        st = check_launch(c, "k_c4_count");
    }
    if (!st) st = read_slots(c, dD, ent, D);
    (void)hipFree(Q);
    (void)hipFree(dD);
    return st;
}

static C4Geom c4_geom(const micsa_ctx* c)
{
    C4Geom cg;
    cg.E = (c->g.Kx + 63) / 32;
    cg.Wv = (c->g.Kx + 31) / 32;
    cg.rmax = std::max({c->p.Lx, c->p.Ly, c->p.Lz}) / 2;
    cg.npair = c->p.n_replicas * (c->p.n_replicas - 1) / 2;
    return cg;
}

int micsa_read_c4(micsa_ctx* ctx, int64_t* G)
{
    if (!ctx || !G) return MICSA_EINVAL;
    if (int st_ = settle_msc(ctx)) return st_;  // the byte arrays are read or written
    if (ctx->p.n_replicas < 2) return fail(ctx, MICSA_EINVAL, "C4 needs at least two replicas");
    const C4Geom cg = c4_geom(ctx);
    std::vector<int64_t> D;
    const int st = c4_counts(ctx, cg, D);
    if (st) return st;
    const int64_t N = n_sites(ctx);
    const int side[3] = {ctx->p.Lx, ctx->p.Ly, ctx->p.Lz};
    for (int s = 0; s < ctx->p.n_samples; ++s)
        for (int mu = 0; mu < 3; ++mu)
            for (int r = 0; r <= cg.rmax; ++r) {
                const int64_t e = ((int64_t)s * 3 + mu) * (cg.rmax + 1) + r;
                G[e] = 2 * r <= side[mu] ? N * cg.npair - 2 * D[(size_t)e] : 0;
            }
    return MICSA_OK;
}

// ------------------------------------------- C4 into a static scratch array
// The overlap rows and the count slots of micsa_read_c4 live in `scratch`, a
// file-scope device array (one copy per device, held until the process
// ends), so this call allocates nothing.  Host code never passes the
// array's name to a kernel or a copy: it uses the device address that
// hipGetSymbolAddress returns for the device the context lives on.
constexpr size_t kC4ScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) uint8_t scratch[kC4ScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on the context's device (looked up once per
// device, with that device current).
int scratch_address(micsa_ctx* c, uint8_t** out)
{
    if (c->device < 0 || c->device >= kMaxDevices) return fail(c, MICSA_EINVAL, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[c->device]) {
        int prev = 0;
        HIP_TRY(c, hipGetDevice(&prev));
        if (prev != c->device) HIP_TRY(c, hipSetDevice(c->device));
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (prev != c->device) (void)hipSetDevice(prev);
        if (e != hipSuccess || !ptr)
            return fail(c, MICSA_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_addr[c->device] = static_cast<uint8_t*>(ptr);
    }
    *out = g_scratch_addr[c->device];
    return MICSA_OK;
}

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }
}  // namespace

int micsa_read_c4_static(micsa_ctx* ctx, int64_t* G)
{
    if (!ctx || !G) return MICSA_EINVAL;
    if (int st_ = settle_msc(ctx)) return st_;  // the byte arrays are read or written
    if (ctx->p.n_replicas < 2) return fail(ctx, MICSA_EINVAL, "C4 needs at least two replicas");
    const C4Geom cg = c4_geom(ctx);
    const int64_t ent = (int64_t)ctx->p.n_samples * 3 * (cg.rmax + 1);
    const int64_t per_pair = (int64_t)2 * ctx->g.rows * cg.E;  // 32-bit words of one pair's rows
    const int64_t total = (int64_t)ctx->p.n_samples * cg.npair;
    const size_t slots_bytes = align256((size_t)ent * kSlots * 8), sums_bytes = align256((size_t)ent * 8);
    const size_t head = slots_bytes + sums_bytes;
    if (head + (size_t)per_pair * 4 > kC4ScratchBytes)
        return fail(ctx, MICSA_ERANGE, "lattice too large for the 32 MiB static scratch (use micsa_read_c4)");
    uint8_t* base = nullptr;
    int st = scratch_address(ctx, &base);
    if (st) return st;
    auto* dD = reinterpret_cast<unsigned long long*>(base);
    auto* sums = reinterpret_cast<long long*>(base + slots_bytes);
    auto* Q = reinterpret_cast<uint32_t*>(base + head);
    const int64_t chunk =
        std::max<int64_t>(1, std::min<int64_t>({total, (int64_t)((kC4ScratchBytes - head) / 4) / per_pair, 65535}));
    // the array keeps the previous call's contents: clear the count slots
    k_fill_i64<<<grid_for(ent * kSlots, 1), kBlock, 0, ctx->stream>>>(dD, ent * kSlots, 0ull);
    if ((st = check_launch(ctx, "k_fill_i64"))) return st;
    const int64_t valid = (int64_t)2 * ctx->g.rows * cg.Wv;
    for (int64_t sp0 = 0; sp0 < total; sp0 += chunk) {
        const unsigned n = (unsigned)std::min(chunk, total - sp0);
        if (ctx->bit)
            k_pack_overlap<true><<<dim3((unsigned)((per_pair + 255) / 256), n), 256, 0, ctx->stream>>>(
                geomb(ctx), cg, (int)sp0, nullptr, ctx->bspin, Q);
        else
            k_pack_overlap<false><<<dim3((unsigned)((per_pair + 255) / 256), n), 256, 0, ctx->stream>>>(
                geomb(ctx), cg, (int)sp0, ctx->spin, nullptr, Q);
        if ((st = check_launch(ctx, "k_pack_overlap"))) return st;
        k_c4_count<<<dim3((unsigned)((valid + 255) / 256), (unsigned)(3 * (cg.rmax + 1)), n), 256, 0,
                     ctx->stream>>>(ctx->g, cg, (int)sp0, Q, dD);
        if ((st = check_launch(ctx, "k_c4_count"))) return st;
    }
    k_sum_slots<<<grid_for(ent, 1), kBlock, 0, ctx->stream>>>(dD, ent, sums);
    if ((st = check_launch(ctx, "k_sum_slots"))) return st;
    HIP_TRY(ctx, hipMemcpyAsync(G, sums, (size_t)ent * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    const int64_t N = n_sites(ctx);
    const int side[3] = {ctx->p.Lx, ctx->p.Ly, ctx->p.Lz};
    for (int s = 0; s < ctx->p.n_samples; ++s)
        for (int mu = 0; mu < 3; ++mu)
            for (int r = 0; r <= cg.rmax; ++r) {
                const int64_t e = ((int64_t)s * 3 + mu) * (cg.rmax + 1) + r;
                G[e] = 2 * r <= side[mu] ? N * cg.npair - 2 * G[e] : 0;
            }
    return MICSA_OK;
}

int micsa_read_xi(micsa_ctx* ctx, double* xi12, double* xi23)
{
    if (!ctx || !xi12 || !xi23) return MICSA_EINVAL;
    if (int st_ = settle_msc(ctx)) return st_;  // the byte arrays are read or written
    if (ctx->p.n_replicas < 2) return fail(ctx, MICSA_EINVAL, "xi needs at least two replicas");
    const C4Geom cg = c4_geom(ctx);
    std::vector<int64_t> G((size_t)ctx->p.n_samples * 3 * (cg.rmax + 1));
    int st = micsa_read_c4(ctx, G.data());
    if (st) return st;
    const int64_t N = n_sites(ctx);
    const int rmin = std::min({ctx->p.Lx, ctx->p.Ly, ctx->p.Lz}) / 2;
    for (int s = 0; s < ctx->p.n_samples; ++s) {
        // C4(r): mean over the three axes, normalised so that C4(0) = 1;
        // I_n = sum_{r = 0}^{rmin} r^n C4(r); xi12 = I2/I1, xi23 = I3/I2
        double I[4] = {0, 0, 0, 0};
        for (int r = 0; r <= rmin; ++r) {
            int64_t sum = 0;
            for (int mu = 0; mu < 3; ++mu) sum += G[(size_t)(((int64_t)s * 3 + mu) * (cg.rmax + 1) + r)];
            const double c4 = (double)sum / (3.0 * (double)N * (double)cg.npair);
            double pw = 1.0;
            for (int n = 0; n < 4; ++n) {
                I[n] += pw * c4;
                pw *= (double)r;
            }
        }
        if (!(I[1] > 0.0) || !(I[2] > 0.0)) {
            xi12[s] = xi23[s] = NAN;
        } else {
            xi12[s] = I[2] / I[1];
            xi23[s] = I[3] / I[2];
        }
    }
    return MICSA_OK;
}

int micsa_read_overlap(micsa_ctx* ctx, int32_t a, int32_t b, int64_t* Q)
{
    if (!ctx || !Q) return MICSA_EINVAL;
    if (int st_ = settle_msc(ctx)) return st_;  // the byte arrays are read or written
    if (a < 0 || b < 0 || a >= ctx->p.n_replicas || b >= ctx->p.n_replicas || a == b)
        return fail(ctx, MICSA_EINVAL, "replica indices out of range or equal");
    const int S = ctx->p.n_samples;
    int st;
    if (ctx->bit) {
        if ((st = enqueue_lane_count<2>(ctx, ctx->red, a, b))) return st;
    } else {
        if ((st = zero_slots(ctx, ctx->red, S))) return st;
        const int64_t wpl = 2 * ctx->g.Nh / 4;
        {
            TimedLaunch t(ctx, kTimeReduce);
            k_differ_count<<<grid_for(wpl, S), kBlock, 0, ctx->stream>>>(
                wpl, ctx->p.n_replicas, a, b, reinterpret_cast<const uint32_t*>(ctx->spin), ctx->red);
        }
        if ((st = check_launch(ctx, "k_differ_count"))) return st;
    }
    std::vector<int64_t> v;
    if ((st = read_red(ctx, S, v))) return st;
    const int64_t N = n_sites(ctx);
    for (int s = 0; s < S; ++s) Q[s] = N - 2 * v[(size_t)s];
    return MICSA_OK;
}

// Byte-layout arrays of `count` parity-split lattices ([count][2][Nh]: the
// spins, or the daemons with count = L * gamma) -> host [count][N].
static int read_state(micsa_ctx* ctx, const uint8_t* dev, uint8_t* host, int64_t count, uint8_t mask = 0xFF)
{
    const int64_t N = n_sites(ctx);
    std::vector<uint8_t> buf((size_t)count * 2 * (size_t)ctx->g.Nh);
    HIP_TRY(ctx, hipMemcpyAsync(buf.data(), dev, buf.size(), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    for (int64_t l = 0; l < count; ++l)
        for (int64_t i = 0; i < N; ++i) {
            int par;
            int64_t h;
            split_index(ctx, i, par, h);
            host[(int64_t)l * N + i] = buf[((size_t)l * 2 + par) * ctx->g.Nh + h] & mask;
        }
    return MICSA_OK;
}

// Bit-plane words [WL][2][Nh] -> host values [S][R][N]; with two planes
// (daemons) the value is bit0 + 2 bit1.
static int read_words(micsa_ctx* ctx, const uint64_t* w0, const uint64_t* w1, uint8_t* host)
{
    const int64_t N = n_sites(ctx);
    const int R = ctx->p.n_replicas;
    const GeomB gb = geomb(ctx);
    const size_t n = (size_t)word_lattices(ctx) * 2 * (size_t)ctx->g.Nh;
    std::vector<uint64_t> a(n), b(w1 ? n : 0);
    HIP_TRY(ctx, hipMemcpyAsync(a.data(), w0, n * 8, hipMemcpyDeviceToHost, ctx->stream));
    if (w1) HIP_TRY(ctx, hipMemcpyAsync(b.data(), w1, n * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    for (int s = 0; s < ctx->p.n_samples; ++s)
        for (int r = 0; r < R; ++r)
            for (int64_t i = 0; i < N; ++i) {
                int par;
                int64_t h;
                split_index(ctx, i, par, h);
                int lane;
                const size_t idx = ((size_t)bp_word_of(gb, s, r, lane) * 2 + par) * ctx->g.Nh + h;
                uint8_t v = (uint8_t)((a[idx] >> lane) & 1u);
                if (w1) v = (uint8_t)(v | (((b[idx] >> lane) & 1u) << 1));
                host[((int64_t)s * R + r) * N + i] = v;
            }
    return MICSA_OK;
}

int micsa_read_spins(micsa_ctx* ctx, uint8_t* sigma)
{
    if (!ctx || !sigma) return MICSA_EINVAL;
    if (int st_ = settle_msc(ctx)) return st_;  // the byte arrays are read or written
    if (ctx->bit) return read_words(ctx, ctx->bspin, nullptr, sigma);
    return read_state(ctx, ctx->spin, sigma, ctx->L, 1);  // bit 0: even bytes also hold their bonds
}

int micsa_read_demons(micsa_ctx* ctx, uint8_t* m)
{
    if (!ctx || !m) return MICSA_EINVAL;
    if (int st_ = settle_msc(ctx)) return st_;  // the byte arrays are read or written
    if (ctx->bit) return read_words(ctx, ctx->bdm0, ctx->bdm1, m);
    const int st = settle_wander(ctx);
    if (st) return st;
    return read_state(ctx, ctx->dem, m, (int64_t)ctx->L * ctx->gamma);
}

int micsa_read_couplings(micsa_ctx* ctx, uint8_t* j)
{
    if (!ctx || !j) return MICSA_EINVAL;
    if (int st_ = settle_msc(ctx)) return st_;  // the byte arrays are read or written
    const Geom& g = ctx->g;
    const int S = ctx->p.n_samples;
    std::vector<uint8_t> jbytes;
    std::vector<uint64_t> wplanes;
    if (ctx->bit) {
        wplanes.resize((size_t)bp_coupling_sets(geomb(ctx)) * 6 * g.Nh);
        HIP_TRY(ctx, hipMemcpyAsync(wplanes.data(), ctx->bJ, wplanes.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
    } else {
        // bits 1..6 of the even spin bytes of replica 0 of each sample
        jbytes.resize((size_t)S * g.Nh);
        for (int s = 0; s < S; ++s)
            HIP_TRY(ctx, hipMemcpyAsync(jbytes.data() + (size_t)s * g.Nh,
                                        ctx->spin + (size_t)s * ctx->p.n_replicas * 2 * g.Nh, (size_t)g.Nh,
                                        hipMemcpyDeviceToHost, ctx->stream));
        for (auto& b : jbytes) b = (uint8_t)(b >> 1);
    }
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    const int64_t N = n_sites(ctx);
    auto bit = [&](int s, int d, int64_t h) -> uint32_t {
        if (ctx->bit && ctx->p.lane_mode == MICSA_LANES_REPLICAS)  // broadcast words: every bit the same
            return (uint32_t)(wplanes[((size_t)s * 6 + d) * g.Nh + (size_t)h] & 1u);
        if (ctx->bit)
            return (uint32_t)((wplanes[((size_t)(s / 64) * 6 + d) * g.Nh + (size_t)h] >> (s % 64)) & 1u);
        return (uint32_t)(jbytes[(size_t)s * g.Nh + (size_t)h] >> d) & 1u;
    };
    for (int s = 0; s < S; ++s)
        for (int64_t i = 0; i < N; ++i) {
            const int x = (int)(i % g.Lx), y = (int)((i / g.Lx) % g.Ly), z = (int)(i / ((int64_t)g.Lx * g.Ly));
            uint8_t v = 0;
            if (((x + y + z) & 1) == 0) {
                const int64_t h = i >> 1;
                v = (uint8_t)(bit(s, kPx, h) | (bit(s, kPy, h) << 1) | (bit(s, kPz, h) << 2));
            } else {
                // forward bonds of an odd site are the backward bonds of its even neighbours
                auto idx = [&](int xx, int yy, int zz) {
                    return ((xx % g.Lx) + (int64_t)g.Lx * ((yy % g.Ly) + (int64_t)g.Ly * (zz % g.Lz))) >> 1;
                };
                v = (uint8_t)(bit(s, kMx, idx(x + 1, y, z)) | (bit(s, kMy, idx(x, y + 1, z)) << 1) |
                              (bit(s, kMz, idx(x, y, z + 1)) << 2));
            }
            j[(int64_t)s * N + i] = v;
        }
    return MICSA_OK;
}

static int write_state(micsa_ctx* ctx, uint8_t* dev, const uint8_t* host, uint8_t maxv, int64_t count)
{
    const int64_t N = n_sites(ctx);
    std::vector<uint8_t> buf((size_t)count * 2 * (size_t)ctx->g.Nh);
    for (int64_t l = 0; l < count; ++l)
        for (int64_t i = 0; i < N; ++i) {
            const uint8_t v = host[(int64_t)l * N + i];
            if (v > maxv) return fail(ctx, MICSA_EINVAL, "value out of range");
            int par;
            int64_t h;
            split_index(ctx, i, par, h);
            buf[((size_t)l * 2 + par) * ctx->g.Nh + h] = v;
        }
    HIP_TRY(ctx, hipMemcpyAsync(dev, buf.data(), buf.size(), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return MICSA_OK;
}

// Host values [S][R][N] -> bit-plane words (bit0 into w0, bit1 into w1).
static int write_words(micsa_ctx* ctx, uint64_t* w0, uint64_t* w1, const uint8_t* host, uint8_t maxv)
{
    const int64_t N = n_sites(ctx);
    const int R = ctx->p.n_replicas;
    const GeomB gb = geomb(ctx);
    const size_t n = (size_t)word_lattices(ctx) * 2 * (size_t)ctx->g.Nh;
    std::vector<uint64_t> a(n, 0), b(w1 ? n : 0, 0);
    for (int s = 0; s < ctx->p.n_samples; ++s)
        for (int r = 0; r < R; ++r)
            for (int64_t i = 0; i < N; ++i) {
                const uint8_t v = host[((int64_t)s * R + r) * N + i];
                if (v > maxv) return fail(ctx, MICSA_EINVAL, "value out of range");
                int par;
                int64_t h;
                split_index(ctx, i, par, h);
                int lane;
                const size_t idx = ((size_t)bp_word_of(gb, s, r, lane) * 2 + par) * ctx->g.Nh + h;
                a[idx] |= (uint64_t)(v & 1u) << lane;
                if (w1) b[idx] |= (uint64_t)(v >> 1) << lane;
            }
    HIP_TRY(ctx, hipMemcpyAsync(w0, a.data(), n * 8, hipMemcpyHostToDevice, ctx->stream));
    if (w1) HIP_TRY(ctx, hipMemcpyAsync(w1, b.data(), n * 8, hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return MICSA_OK;
}

int micsa_write_spins(micsa_ctx* ctx, const uint8_t* sigma)
{
    if (!ctx || !sigma) return MICSA_EINVAL;
    if (int st_ = settle_msc(ctx)) return st_;  // the byte arrays are read or written
    int st = ctx->bit ? write_words(ctx, ctx->bspin, nullptr, sigma, 1) : write_state(ctx, ctx->spin, sigma, 1, ctx->L);
    if (!st && !ctx->bit) st = enqueue_bonds(ctx);  // the written bytes hold spins only: restore the bond bits
    if (st) return st;
    std::vector<int64_t> E((size_t)ctx->L);
    if ((st = micsa_read_energy(ctx, E.data()))) return st;
    if ((st = set_tally(ctx, E))) return st;
    ctx->tally_ok = true;
    return MICSA_OK;
}

int micsa_write_demons(micsa_ctx* ctx, const uint8_t* m)
{
    if (!ctx || !m) return MICSA_EINVAL;
    if (int st_ = settle_msc(ctx)) return st_;  // the byte arrays are read or written
    if (ctx->bit) return write_words(ctx, ctx->bdm0, ctx->bdm1, m, 3);
    const int st = write_state(ctx, ctx->dem, m, 3, (int64_t)ctx->L * ctx->gamma);
    if (!st) ctx->pend_wander = -1;  // the written daemons are where they are
    return st;
}

// ------------------------------------------------------------- checkpoint
// Image: CkHeader, the schedule table (T_len doubles), the tally per lattice
// (int64), spins [L][N], daemons [L][gamma][N], couplings [S][N] (bytes),
// then the FNV-1a hash of everything before it.
namespace {
constexpr char kCkMagic[8] = {'M', 'I', 'C', 'S', 'A', '-', 'C', 'K'};
constexpr uint32_t kCkVersion = 1;

struct CkHeader {
    char magic[8];
    uint32_t version;
    uint32_t header_bytes;
    micsa_params p;
    int64_t k;
    int32_t sched_set, sched_kind, sched_period, reserved;
    double T0, T1;
    int64_t n_sweeps, T_len;
    uint64_t total_bytes;
};

uint64_t fnv1a(const uint8_t* d, size_t n)
{
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= d[i];
        h *= 1099511628211ull;
    }
    return h;
}

size_t ck_bytes(const micsa_ctx* c, int64_t T_len)
{
    const size_t N = (size_t)n_sites(c), L = (size_t)c->L;
    return sizeof(CkHeader) + (size_t)T_len * 8 + L * 8 + L * N + L * (size_t)c->gamma * N +
           (size_t)c->p.n_samples * N + 8;
}

bool same_params(const micsa_params& a, const micsa_params& b)
{
    return a.Lx == b.Lx && a.Ly == b.Ly && a.Lz == b.Lz && a.n_samples == b.n_samples &&
           a.n_replicas == b.n_replicas && a.layout == b.layout && a.gamma == b.gamma &&
           a.lane_mode == b.lane_mode && a.seed == b.seed;
}
}  // namespace

int micsa_save(micsa_ctx* ctx, void* buf, size_t* len)
{
    if (!ctx || !len) return MICSA_EINVAL;
    if (int st_ = settle_msc(ctx)) return st_;  // the byte arrays are read or written
    const int64_t T_len = ctx->sched.set ? (int64_t)ctx->sched.table.size() : 0;
    const size_t total = ck_bytes(ctx, T_len);
    if (!buf) {
        *len = total;
        return MICSA_OK;
    }
    if (*len < total) {
        *len = total;
        return fail(ctx, MICSA_ERANGE, "checkpoint buffer smaller than micsa_save's size");
    }
    const size_t N = (size_t)n_sites(ctx), L = (size_t)ctx->L;
    uint8_t* out = static_cast<uint8_t*>(buf);
    CkHeader h;
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.magic, kCkMagic, 8);
    h.version = kCkVersion;
    h.header_bytes = (uint32_t)sizeof(CkHeader);
    h.p = ctx->p;
    h.k = ctx->k;
    h.sched_set = ctx->sched.set ? 1 : 0;
    h.sched_kind = ctx->sched.kind;
    h.sched_period = ctx->sched.period;
    h.T0 = ctx->sched.T0;
    h.T1 = ctx->sched.T1;
    h.n_sweeps = ctx->sched.n_sweeps;
    h.T_len = T_len;
    h.total_bytes = total;
    size_t o = sizeof(CkHeader);
    if (T_len) std::memcpy(out + o, ctx->sched.table.data(), (size_t)T_len * 8);
    o += (size_t)T_len * 8;
    int st;
    // reading the daemons first applies an owed walker wandering
    uint8_t* tally = out + o;
    uint8_t* spins = tally + L * 8;
    uint8_t* dems = spins + L * N;
    uint8_t* coup = dems + L * (size_t)ctx->gamma * N;
    if ((st = micsa_read_demons(ctx, dems))) return st;
    if ((st = micsa_read_spins(ctx, spins))) return st;
    if ((st = micsa_read_couplings(ctx, coup))) return st;
    std::vector<int64_t> E(L);
    st = ctx->bit && !ctx->tally_ok ? micsa_read_energy(ctx, E.data()) : micsa_read_energy_tally(ctx, E.data());
    if (st) return st;
    std::memcpy(tally, E.data(), L * 8);
    h.k = ctx->k;
    std::memcpy(out, &h, sizeof h);
    const uint64_t hash = fnv1a(out, total - 8);
    std::memcpy(out + total - 8, &hash, 8);
    *len = total;
    return MICSA_OK;
}

int micsa_load(micsa_ctx* ctx, const void* buf, size_t len)
{
    if (!ctx) return MICSA_EINVAL;
    if (int st_ = settle_msc(ctx)) return st_;  // the byte arrays are read or written
    if (!buf) return fail(ctx, MICSA_EINVAL, "null checkpoint");
    const uint8_t* in = static_cast<const uint8_t*>(buf);
    CkHeader h;
    if (len < sizeof h) return fail(ctx, MICSA_EINVAL, "checkpoint too short");
    std::memcpy(&h, in, sizeof h);
    if (std::memcmp(h.magic, kCkMagic, 8) != 0 || h.version != kCkVersion || h.header_bytes != sizeof(CkHeader))
        return fail(ctx, MICSA_EINVAL, "not a checkpoint of this library version");
    if (!same_params(h.p, ctx->p))
        return fail(ctx, MICSA_EINVAL, "checkpoint of a context with other parameters");
    if (h.T_len < 0 || h.T_len > (int64_t)(len / 8) || h.k < 0) return fail(ctx, MICSA_EINVAL, "corrupt checkpoint");
    const size_t total = ck_bytes(ctx, h.T_len);
    if (h.total_bytes != total || len < total) return fail(ctx, MICSA_EINVAL, "checkpoint size mismatch");
    uint64_t hash;
    std::memcpy(&hash, in + total - 8, 8);
    if (hash != fnv1a(in, total - 8)) return fail(ctx, MICSA_EINVAL, "checkpoint checksum mismatch");
    const size_t N = (size_t)n_sites(ctx), L = (size_t)ctx->L;
    const uint8_t* table = in + sizeof(CkHeader);
    const uint8_t* tally = table + (size_t)h.T_len * 8;
    const uint8_t* spins = tally + L * 8;
    const uint8_t* dems = spins + L * N;
    const uint8_t* coup = dems + L * (size_t)ctx->gamma * N;
    // the couplings follow from the seed: they must be this context's
    std::vector<uint8_t> mine((size_t)ctx->p.n_samples * N);
    int st = micsa_read_couplings(ctx, mine.data());
    if (st) return st;
    if (std::memcmp(mine.data(), coup, mine.size()) != 0)
        return fail(ctx, MICSA_EINVAL, "checkpoint couplings differ from the context's");
    for (size_t i = 0; i < L * N; ++i)
        if (spins[i] > 1) return fail(ctx, MICSA_EINVAL, "checkpoint spin out of range");
    for (size_t i = 0; i < L * (size_t)ctx->gamma * N; ++i)
        if (dems[i] > 3) return fail(ctx, MICSA_EINVAL, "checkpoint daemon level out of range");
    if (h.sched_set) {
        micsa_schedule s{};
        s.kind = h.sched_kind;
        s.refresh_period = h.sched_period;
        s.T0 = h.T0;
        s.T1 = h.T1;
        s.n_sweeps = h.n_sweeps;
        std::vector<double> tb((size_t)h.T_len);
        if (h.T_len) std::memcpy(tb.data(), table, (size_t)h.T_len * 8);
        s.T_table = tb.empty() ? nullptr : tb.data();
        s.T_len = h.T_len;
        if ((st = micsa_set_schedule(ctx, &s))) return st;
    } else {
        ctx->sched = Schedule{};
        ctx->sdr_k[0] = ctx->sdr_k[1] = -1;
        ctx->msc_drawn = -1;
    }
    if ((st = micsa_write_spins(ctx, spins))) return st;
    if ((st = micsa_write_demons(ctx, dems))) return st;
    {
        std::vector<int64_t> E(L);
        std::memcpy(E.data(), tally, L * 8);
        if ((st = set_tally(ctx, E))) return st;
    }
    ctx->k = h.k;
    return MICSA_OK;
}

int micsa_get_counters(micsa_ctx* ctx, int64_t* k, int64_t* rho)
{
    if (!ctx) return MICSA_EINVAL;
    if (k) *k = ctx->k;
    if (rho) *rho = refresh_index(ctx->k / ctx->gamma, ctx->sched.set ? ctx->sched.period : 1);
    return MICSA_OK;
}

int micsa_get_thresholds(micsa_ctx* ctx, int64_t rho, uint64_t t[3])
{
    if (!ctx || !t) return MICSA_EINVAL;
    if (!ctx->sched.set) return fail(ctx, MICSA_ESTATE, "no schedule installed");
    if (rho < 0 || rho >= std::max<int64_t>(refresh_count(ctx->sched), 1))
        return fail(ctx, MICSA_ERANGE, "refresh index outside the schedule");
    const DaemonThresholds th = daemon_thresholds(temperature(ctx->sched, rho));
    t[0] = th.t0;
    t[1] = th.t1;
    t[2] = th.t2;
    return MICSA_OK;
}

int micsa_get_heatbath_thresholds(micsa_ctx* ctx, int64_t rho, uint64_t tau[7])
{
    if (!ctx || !tau) return MICSA_EINVAL;
    if (!ctx->sched.set) return fail(ctx, MICSA_ESTATE, "no schedule installed");
    if (rho < 0 || rho >= std::max<int64_t>(refresh_count(ctx->sched), 1))
        return fail(ctx, MICSA_ERANGE, "refresh index outside the schedule");
    const HeatBathThresholds th = heatbath_thresholds(temperature(ctx->sched, rho));
    for (int v = 0; v < 7; ++v) tau[v] = th.tau[v];
    return MICSA_OK;
}

int micsa_get_metropolis_thresholds(micsa_ctx* ctx, int64_t rho, uint64_t theta[7])
{
    if (!ctx || !theta) return MICSA_EINVAL;
    if (!ctx->sched.set) return fail(ctx, MICSA_ESTATE, "no schedule installed");
    if (rho < 0 || rho >= std::max<int64_t>(refresh_count(ctx->sched), 1))
        return fail(ctx, MICSA_ERANGE, "refresh index outside the schedule");
    const MetropolisThresholds th = metropolis_thresholds(temperature(ctx->sched, rho));
    for (int q = 0; q < 7; ++q) theta[q] = th.tau[q];
    return MICSA_OK;
}

int micsa_set_timing(micsa_ctx* ctx, int32_t enable)
{
    if (!ctx) return MICSA_EINVAL;
    ctx->timing = enable != 0;
    return MICSA_OK;
}

int micsa_get_timing(micsa_ctx* ctx, int32_t kind, double* total_ms, int64_t* launches)
{
    if (!ctx || kind < 0 || kind >= kTimingKinds) return MICSA_EINVAL;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    for (int kd = 0; kd < kTimingKinds; ++kd) {
        for (auto& e : ctx->events[kd]) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) {
                ctx->time_ms[kd] += ms;
                ctx->launches[kd] += 1;
            }
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        ctx->events[kd].clear();
    }
    if (total_ms) *total_ms = ctx->time_ms[kind];
    if (launches) *launches = ctx->launches[kind];
    return MICSA_OK;
}

const char* micsa_kernel_name(const micsa_ctx* ctx, int32_t algo)
{
    if (ctx && ctx->bit)
        return algo == MICSA_ALGO_MICSA
                   ? (bp_one_launch(ctx) && !use_graph(ctx) ? (bp_rows(bp_launch(ctx)) ? "kb_sweep_rows" : "kb_sweep")
                                                            : "kb_micsa_half")
                   : "";
    if (ctx && algo == MICSA_ALGO_MICSA && use_msc(ctx))  // a long call runs its sweeps in pairs where it can
        return msc_one_launch(ctx) ? (msc2_fits(ctx) ? "k_msc_sweep_multi" : "k_msc_sweep") : "k_msc_half";
    // walkers on the fused sweeps wander on the next sweep's loads
    if (ctx && algo == MICSA_ALGO_WALKERS && use_msc(ctx, kMscMinSweeps, algo))
        return msc_one_launch(ctx) && msc2_fits(ctx) && 64 % (ctx->p.Lx / 128) == 0 ? "k_msc_sweep_multi"
                                                                                    : "k_msc_sweep";
    if (algo == MICSA_ALGO_WALKERS)
        return ctx && use_fused(ctx) && ctx->gamma == 1
                   ? (ctx->temporal == 2 && sweep2_walk_eligible(ctx) ? "k_micsa_sweep2_fused" : "k_micsa_sweep_fused")
                   : "k_micsa_half+k_wander";
    // gamma > 1 runs the per-half kernels (never resident or fused)
    if (ctx && use_resident(ctx))
        return algo == MICSA_ALGO_HEATBATH ? "k_resident<1>" : (algo == MICSA_ALGO_METROPOLIS ? "k_resident<2>" : "k_resident<0>");
    if (algo == MICSA_ALGO_HEATBATH)
        return ctx && use_fused(ctx) ? "k_heatbath_sweep_fused<0>" : "k_heatbath_half<0>";
    if (algo == MICSA_ALGO_METROPOLIS)
        return ctx && use_fused(ctx) ? "k_heatbath_sweep_fused<1>" : "k_heatbath_half<1>";
    if (ctx && use_fused(ctx))
        return ctx->temporal == 2 && sweep2_eligible(ctx) ? "k_micsa_sweep2_fused" : "k_micsa_sweep_fused";
    if (ctx && use_slab(ctx)) return slab_pairs(ctx) ? "k_micsa_slab2" : "k_micsa_slab";
    return "k_micsa_half";
}

int micsa_set_option(micsa_ctx* ctx, int32_t option, int64_t value)
{
    if (!ctx) return MICSA_EINVAL;
    switch (option) {
    case MICSA_OPT_SWEEP_KERNEL:
        if (value != MICSA_KERNEL_AUTO && value != MICSA_KERNEL_SIMPLE && value != MICSA_KERNEL_FUSED &&
            value != MICSA_KERNEL_RESIDENT && value != MICSA_KERNEL_MULTISPIN && value != MICSA_KERNEL_SLAB)
            return fail(ctx, MICSA_EINVAL, "unknown sweep kernel");
        if (value == MICSA_KERNEL_SLAB && !slab_eligible(ctx))
            return fail(ctx, MICSA_EINVAL, "the slab sweep needs the byte layout, gamma = 1 and Ly * Lx / 8 <= 1024");
        if (value == MICSA_KERNEL_MULTISPIN && !msc_eligible(ctx))
            return fail(ctx, MICSA_EINVAL, "the multispin sweep needs the byte layout, gamma = 1 and Lx % 128 == 0");
        if (value == MICSA_KERNEL_RESIDENT && !resident_eligible(ctx))
            return fail(ctx, MICSA_EINVAL, "the resident sweep needs a byte-layout lattice of at most 102400 sites");
        if (value == MICSA_KERNEL_FUSED && ctx->bit && !bp_fits(ctx, bp_launch(ctx)))
            return fail(ctx, MICSA_EINVAL, "the one-launch bit-plane sweep needs five rows of a plane in a work-group");
        if (value == MICSA_KERNEL_FUSED && !ctx->bit && !fused_eligible(ctx))
            return fail(ctx, MICSA_EINVAL, "the fused sweep needs Lx % 32 == 0");
        ctx->kernel_opt = (int32_t)value;
        return MICSA_OK;
    case MICSA_OPT_TILE_Y:
        if (value < 0 || value > ctx->p.Ly || (value > 0 && (value + 4) * (ctx->p.Lx / 32) > 1024))
            return fail(ctx, MICSA_EINVAL, "tile_y must be at most Ly and fit a work-group");
        ctx->tile_y = (int32_t)value;
        return MICSA_OK;
    case MICSA_OPT_GRAPHS:
        if (value != 0 && value != 1) return fail(ctx, MICSA_EINVAL, "graphs is 0 or 1");
        ctx->use_graphs = (int32_t)value;
        return MICSA_OK;
    case MICSA_OPT_DRAW_AHEAD:
        if (value != 0 && value != 1) return fail(ctx, MICSA_EINVAL, "draw_ahead is 0 or 1");
        ctx->draw_ahead = (int32_t)value;
        return MICSA_OK;
    case MICSA_OPT_MSC_FUSED:
        if (value != 0 && value != 1) return fail(ctx, MICSA_EINVAL, "msc_fused is 0 or 1");
        ctx->msc_fused = (int32_t)value;
        return MICSA_OK;
    case MICSA_OPT_TEMPORAL:
        if (value != 1 && value != 2) return fail(ctx, MICSA_EINVAL, "temporal is 1 or 2");
        ctx->temporal = (int32_t)value;
        return MICSA_OK;
    case MICSA_OPT_MSC_PASS:
        if (value != 1 && value != 2) return fail(ctx, MICSA_EINVAL, "msc_pass is 1 or 2");
        ctx->msc_pass = (int32_t)value;
        return MICSA_OK;
    case MICSA_OPT_PREFETCH:
        if (value != 1 && value != 2) return fail(ctx, MICSA_EINVAL, "prefetch is 1 or 2");
        ctx->prefetch = (int32_t)value;
        return MICSA_OK;
    case MICSA_OPT_XCD_MAP:
        if (value < 0 || value > 2) return fail(ctx, MICSA_EINVAL, "xcd_map is 0, 1 or 2");
        ctx->xcd_map = (int32_t)value;
        return MICSA_OK;
    case MICSA_OPT_TILE_Z:
        if (value < 0 || (value > 0 && ctx->p.Lz % value != 0))
            return fail(ctx, MICSA_EINVAL, "tile_z must divide Lz");
        ctx->tile_z = (int32_t)value;
        return MICSA_OK;
    default: return fail(ctx, MICSA_EINVAL, "unknown option");
    }
}

}  // extern "C"

// =========================================================== serving pool
namespace {

struct PoolJob {
    int64_t id = 0;
    micsa_params p{};
    Schedule sched;  // copied schedule (table owned here)
    int32_t state = MICSA_JOB_QUEUED;
    size_t bytes = 0;
    micsa_ctx* ctx = nullptr;
    // Jobs the resident kernel holds run in the pool's batched launch on the
    // pool stream; every other job gets a stream of its own (default
    // priority), so large jobs overlap with each other and with the batch.
    bool batched = false;
    hipStream_t stream = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};  // end of the last two chunks of sweeps
    int64_t chunks = 0;                     // chunks enqueued so far
    int64_t last_batch = -1;                // batched jobs: the batch that holds their latest chunk
};

size_t footprint(const micsa_params* p)
{
    const size_t N = (size_t)p->Lx * p->Ly * p->Lz;
    const size_t L = (size_t)p->n_samples * p->n_replicas;
    const size_t slots = (L + (size_t)p->n_samples) * kSlots * 8;
    if (p->layout == MICSA_LAYOUT_BITPLANE) {
        const bool reps = p->lane_mode == MICSA_LANES_REPLICAS;
        const size_t WL = reps ? (size_t)p->n_samples * (((size_t)p->n_replicas + 63) / 64)
                               : (((size_t)p->n_samples + 63) / 64) * p->n_replicas;
        const size_t NJ = reps ? (size_t)p->n_samples : ((size_t)p->n_samples + 63) / 64;
        return 2 * WL * N * 8 * 3 + NJ * 6 * (N / 2) * 8 + slots;  // state and its alternate
    }
    const size_t gamma = p->gamma == 0 ? 1 : (size_t)p->gamma;
    // 2 state buffers x (spin + gamma daemons); the couplings live in the even spin bytes
    size_t bytes = 2 * L * N * (1 + gamma) + slots;
    // lattices the multispin sweep can take allocate its planes on their first
    // long MicSA call: spins and two level planes, their alternates, the drawn
    // levels (2) and the six coupling planes of the even sites (3 words per
    // word of sites), each 1 bit per site: 11/8 B per site per lattice
    if (gamma == 1 && p->Lx % 128 == 0) bytes += 11 * L * N / 8;
    // lattices the slab sweep takes (too large for the resident sweep,
    // narrower than the fused one) draw refresh levels ahead into two
    // buffers of a byte per site per lattice
    else if (gamma == 1 && (size_t)p->Ly * (p->Lx / 8) <= (size_t)kSlabLanes && N / 2 * 3 > kResidentLdsMax &&
             p->Lx < 128)
        bytes += 2 * L * N;
    return bytes;
}

}  // namespace

struct micsa_pool {
    size_t budget = 0, used = 0;
    int32_t max_running = 1;
    hipStream_t stream = nullptr;
    int64_t next_id = 1;
    std::vector<PoolJob> jobs;  // every job not yet released, in arrival order
    // batched launches: two launches in flight at most, each with its item
    // table (the host may refill one while the other is read)
    ResidentItem* d_items[2] = {nullptr, nullptr};
    size_t d_items_cap[2] = {0, 0};
    std::vector<ResidentItem> h_items[2];  // host copy of each table, kept until its launch has finished
    hipEvent_t bev[2] = {nullptr, nullptr};
    int64_t batches = 0;
};

namespace {

// The chunk slot `n` of a job (or of the batch) may be refilled once the
// chunk two before it has finished.
bool slot_free(hipEvent_t e)
{
    if (!e) return true;
    const hipError_t q = hipEventQuery(e);
    if (q == hipErrorNotReady) return false;
    (void)hipGetLastError();
    return true;
}

void free_job_stream(PoolJob& j)
{
    for (auto& e : j.ev)
        if (e) {
            (void)hipEventDestroy(e);
            e = nullptr;
        }
    if (j.stream) {
        (void)hipStreamDestroy(j.stream);
        j.stream = nullptr;
    }
}

}  // namespace

extern "C" {

int micsa_pool_footprint(const micsa_params* p, size_t* bytes)
{
    if (!p || !bytes) return MICSA_EINVAL;
    *bytes = footprint(p);
    return MICSA_OK;
}

int micsa_pool_create(size_t hbm_budget, int32_t max_running, void* hip_stream, micsa_pool** out)
{
    if (!out) return MICSA_EINVAL;
    *out = nullptr;
    if (hbm_budget == 0 || max_running < 1) return MICSA_EINVAL;
    micsa_pool* pool = new (std::nothrow) micsa_pool();
    if (!pool) return MICSA_ENOMEM;
    pool->budget = hbm_budget;
    pool->max_running = max_running;
    pool->stream = (hipStream_t)hip_stream;
    *out = pool;
    return MICSA_OK;
}

int micsa_pool_destroy(micsa_pool* pool)
{
    if (!pool) return MICSA_OK;
    (void)hipStreamSynchronize(pool->stream);
    for (auto& j : pool->jobs) {
        if (j.ctx) micsa_destroy(j.ctx);  // synchronises the job's stream
        free_job_stream(j);
    }
    for (int b = 0; b < 2; ++b) {
        if (pool->d_items[b]) (void)hipFree(pool->d_items[b]);
        if (pool->bev[b]) (void)hipEventDestroy(pool->bev[b]);
    }
    delete pool;
    return MICSA_OK;
}

int micsa_pool_sync(micsa_pool* pool)
{
    if (!pool) return MICSA_EINVAL;
    if (hipStreamSynchronize(pool->stream) != hipSuccess) return MICSA_EHIP;
    for (auto& j : pool->jobs)
        if (j.stream && hipStreamSynchronize(j.stream) != hipSuccess) return MICSA_EHIP;
    return MICSA_OK;
}

int micsa_pool_submit(micsa_pool* pool, const micsa_params* p, const micsa_schedule* s, int64_t* job)
{
    if (!pool || !p || !s || !job) return MICSA_EINVAL;
    // validate parameters and schedule the same way a context would
    if (!params_ok(p)) return MICSA_EINVAL;
    if (s->refresh_period < 0 || s->n_sweeps < 1) return MICSA_EINVAL;
    auto okT = [](double T) { return T > 0.0 && std::isfinite(T); };
    if (s->kind == MICSA_SCHED_CONST ? !okT(s->T0)
        : s->kind == MICSA_SCHED_LINEAR ? !(okT(s->T0) && okT(s->T1))
        : s->kind != MICSA_SCHED_TABLE)
        return MICSA_EINVAL;
    PoolJob j;
    j.p = *p;
    j.sched.set = true;
    j.sched.kind = s->kind;
    j.sched.period = s->refresh_period;
    j.sched.T0 = s->T0;
    j.sched.T1 = s->T1;
    j.sched.n_sweeps = s->n_sweeps;
    if (s->kind == MICSA_SCHED_TABLE) {
        if (!s->T_table || s->T_len < refresh_count(j.sched)) return MICSA_EINVAL;
        j.sched.table.assign(s->T_table, s->T_table + s->T_len);
    }
    j.bytes = footprint(p);
    if (j.bytes > pool->budget) return MICSA_EINVAL;
    j.id = pool->next_id++;
    *job = j.id;
    pool->jobs.push_back(std::move(j));
    return MICSA_OK;
}

static PoolJob* find_job(micsa_pool* pool, int64_t id)
{
    for (auto& j : pool->jobs)
        if (j.id == id) return &j;
    return nullptr;
}

int micsa_pool_step(micsa_pool* pool, int64_t sweeps, int32_t* running, int32_t* queued)
{
    if (!pool || sweeps < 0) return MICSA_EINVAL;
    // 1. retire jobs whose last chunk has finished on the device (a batch's
    // event is recorded again only after that batch has finished)
    for (auto& j : pool->jobs) {
        if (j.state != MICSA_JOB_RUNNING || j.ctx->k < j.ctx->sched.n_sweeps) continue;
        const bool fin = j.batched ? (j.last_batch < 0 || pool->batches > j.last_batch + 2 ||
                                      slot_free(pool->bev[j.last_batch & 1]))
                                   : (j.chunks == 0 || slot_free(j.ev[(j.chunks - 1) & 1]));
        if (fin) j.state = MICSA_JOB_DONE;
    }
    // 2. admit queued jobs in arrival order while they fit
    int32_t nrun = 0;
    for (auto& j : pool->jobs) nrun += j.state == MICSA_JOB_RUNNING;
    for (auto& j : pool->jobs) {
        if (j.state != MICSA_JOB_QUEUED) continue;
        if (nrun >= pool->max_running || pool->used + j.bytes > pool->budget) break;
        micsa_params pr = j.p;
        micsa_ctx* probe = nullptr;
        // the resident kernel's jobs share the pool stream; the others get their own
        const bool batched = pr.layout == MICSA_LAYOUT_BYTE && (pr.gamma == 0 || pr.gamma == 1) &&
                             (size_t)((int64_t)pr.Lx * pr.Ly * pr.Lz / 2) * 3 <= kResidentLdsMax;
        hipStream_t st_job = pool->stream;
        if (!batched) {
            if (hipStreamCreateWithFlags(&j.stream, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreateWithFlags(&j.ev[0], hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&j.ev[1], hipEventDisableTiming) != hipSuccess) {
                (void)hipGetLastError();
                free_job_stream(j);
                return MICSA_EHIP;
            }
            st_job = j.stream;
        }
        int st = micsa_create(&pr, st_job, &probe);
        if (st == MICSA_ENOMEM) {  // the device is fuller than the budget says: retry next step
            free_job_stream(j);
            break;
        }
        if (st) {
            free_job_stream(j);
            return st;
        }
        j.ctx = probe;
        j.batched = batched;
        micsa_schedule cs{j.sched.kind, j.sched.period, j.sched.T0, j.sched.T1, j.sched.n_sweeps,
                          j.sched.table.empty() ? nullptr : j.sched.table.data(), (int64_t)j.sched.table.size()};
        if ((st = micsa_set_schedule(j.ctx, &cs))) return st;
        j.state = MICSA_JOB_RUNNING;
        pool->used += j.bytes;
        ++nrun;
    }
    // 3. enqueue the next chunk of sweeps of every running job with a free
    // chunk slot (at most two chunks in flight per job, and per batch).
    // Nothing waits for the device: the call returns once the work is queued.
    const int bslot = (int)(pool->batches & 1);
    std::vector<ResidentItem>& items = pool->h_items[bslot];
    std::vector<std::pair<PoolJob*, int64_t>> batched;
    size_t lds = 0;
    if (slot_free(pool->bev[bslot])) {
        items.clear();
        for (auto& j : pool->jobs) {
            if (j.state != MICSA_JOB_RUNNING || !j.batched) continue;
            micsa_ctx* c = j.ctx;
            const int64_t n = std::min<int64_t>(sweeps, c->sched.n_sweeps - c->k);
            if (n <= 0) continue;
            ResidentSched rs{c->k, n, 0, c->sched.period, 0, 0};
            for (int l = 0; l < c->L; ++l)
                items.push_back(ResidentItem{c->g, c->spin, c->dem, c->tally, c->d_dth, rs, l});
            lds = std::max(lds, (size_t)c->g.Nh * 3);
            batched.emplace_back(&j, n);
        }
    }
    if (!batched.empty()) {
        // a resident job's counter moves only once its batch is launched
        if (items.size() > pool->d_items_cap[bslot]) {
            if (pool->d_items[bslot]) (void)hipFree(pool->d_items[bslot]);
            pool->d_items[bslot] = nullptr;
            pool->d_items_cap[bslot] = 0;
            if (hipMalloc(&pool->d_items[bslot], items.size() * sizeof(ResidentItem)) != hipSuccess) {
                (void)hipGetLastError();
                return MICSA_ENOMEM;
            }
            pool->d_items_cap[bslot] = items.size();
        }
        if (!pool->bev[bslot] && hipEventCreateWithFlags(&pool->bev[bslot], hipEventDisableTiming) != hipSuccess)
            return MICSA_EHIP;
        // the table is copied from pageable memory: the copy returns once the
        // host buffer may be reused, and the stream orders it before the launch
        if (hipMemcpyAsync(pool->d_items[bslot], items.data(), items.size() * sizeof(ResidentItem),
                           hipMemcpyHostToDevice, pool->stream) != hipSuccess)
            return MICSA_EHIP;
        static bool attr = false;
        if (!attr) {
            if (hipFuncSetAttribute((const void*)k_resident_batch, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)kResidentLdsMax) != hipSuccess)
                return MICSA_EHIP;
            attr = true;
        }
        k_resident_batch<<<(unsigned)items.size(), kResidentBlock, lds, pool->stream>>>(pool->d_items[bslot]);
        if (hipGetLastError() != hipSuccess) return MICSA_EHIP;
        if (hipEventRecord(pool->bev[bslot], pool->stream) != hipSuccess) return MICSA_EHIP;
        for (auto& b : batched) {
            b.first->ctx->k += b.second;
            b.first->last_batch = pool->batches;
        }
        ++pool->batches;
    }
    for (auto& j : pool->jobs) {
        if (j.state != MICSA_JOB_RUNNING || j.batched) continue;
        micsa_ctx* c = j.ctx;
        const int64_t n = std::min<int64_t>(sweeps, c->sched.n_sweeps - c->k);
        const int slot = (int)(j.chunks & 1);
        if (n <= 0 || !slot_free(j.ev[slot])) continue;
        const int st = micsa_sweep(c, MICSA_ALGO_MICSA, n);
        if (st) return st;
        if (hipEventRecord(j.ev[slot], j.stream) != hipSuccess) return MICSA_EHIP;
        ++j.chunks;
    }
    int32_t r = 0, q = 0;
    for (auto& j : pool->jobs) {
        r += j.state == MICSA_JOB_RUNNING;
        q += j.state == MICSA_JOB_QUEUED;
    }
    if (running) *running = r;
    if (queued) *queued = q;
    return MICSA_OK;
}

int micsa_pool_job_state(micsa_pool* pool, int64_t job, int32_t* state, int64_t* k)
{
    if (!pool) return MICSA_EINVAL;
    PoolJob* j = find_job(pool, job);
    if (!j) {
        if (job >= 1 && job < pool->next_id) {  // released
            if (state) *state = MICSA_JOB_RELEASED;
            if (k) *k = -1;
            return MICSA_OK;
        }
        return MICSA_EINVAL;
    }
    if (state) *state = j->state;
    if (k) *k = j->ctx ? j->ctx->k : 0;
    return MICSA_OK;
}

int micsa_pool_job_context(micsa_pool* pool, int64_t job, micsa_ctx** ctx)
{
    if (!pool || !ctx) return MICSA_EINVAL;
    PoolJob* j = find_job(pool, job);
    if (!j || !j->ctx) return MICSA_EINVAL;
    *ctx = j->ctx;
    return MICSA_OK;
}

int micsa_pool_release(micsa_pool* pool, int64_t job)
{
    if (!pool) return MICSA_EINVAL;
    for (size_t i = 0; i < pool->jobs.size(); ++i) {
        PoolJob& j = pool->jobs[i];
        if (j.id != job) continue;
        if (j.state != MICSA_JOB_DONE) return MICSA_EINVAL;
        micsa_destroy(j.ctx);  // synchronises the job's stream
        free_job_stream(j);
        pool->used -= j.bytes;
        pool->jobs.erase(pool->jobs.begin() + (long)i);
        return MICSA_OK;
    }
    return MICSA_EINVAL;
}

}  // extern "C"
