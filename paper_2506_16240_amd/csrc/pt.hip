// libmicsa: host side of the tempering entry points (micsa_pt_*, include/
// micsa.h) -- the equilibrium workload of App. C.  The context owns the
// spin rows of runs x 2 replicas x M slots, the slot permutation of every
// replica group, the slot energies, the exchange counters, the coupling
// records and the exponential tables of the temperature ladder.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "micsa.h"
#include "pt_kernels.hpp"

using namespace micsa;

struct micsa_pt {
    micsa_pt_params p{};
    PtGeom g{};
    hipStream_t stream = nullptr;
    int64_t e = 0;  // EMCS done
    bool jl = false;  // coupling records staged in LDS
    uint32_t lds = 0;
    int32_t kernel = MICSA_PT_KERNEL_AUTO;
    int32_t G = 0;        // temperatures per work-group of the register kernel (0: not eligible)
    uint32_t reg_lds = 0;
    int4* rec = nullptr;         // [N][2] records, x-major
    uint64_t* spins = nullptr;   // [runs][2][M][R0]
    int32_t* perm = nullptr;     // [runs][2][M]
    int64_t* E = nullptr;        // [runs][2][M] by slot
    int64_t* swaps = nullptr;    // [runs][2][M-1]
    uint32_t* wtab = nullptr;    // [M][kPtTable] device form (thresholds - 1, guides)
    uint32_t* ptab = nullptr;    // [M-1][kPtTable]
    std::vector<int32_t> Jq;     // [3][N]
    std::vector<uint64_t> hw, hp;  // thresholds [M][4][256], [M-1][4][256] (entry 255 unused)
    std::string err;
    bool timing = false;
    // per timed EMCS: events before the EMCS kernel, between the two kernels, after the exchange kernel
    std::vector<std::array<hipEvent_t, 3>> events;
    double time_ms[2] = {};
    int64_t launches[2] = {};
};

namespace {

constexpr uint32_t kPtLdsMax = 150u * 1024u;

int pt_fail(micsa_pt* c, int st, const std::string& m)
{
    if (c) c->err = m;
    return st;
}

#define PT_TRY(c, call)                                                                           \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return pt_fail((c), MICSA_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));  \
    } while (0)

// Digit thresholds of the mesh exponential of rate lam (per unit energy):
// digit d has ratio r_d = exp(-lam 2^(8d-17)); t_d[v] = floor(2^32 F_d(v)),
// F_d(v) = (1 - r_d^(v+1)) / (1 - r_d^256) for d < 3 and 1 - r_3^(v+1) for
// the untruncated top digit.  t has [4][256] entries, entry 255 unused.
void exp_table(double lam, uint64_t* t)
{
    for (int d = 0; d < 4; ++d) {
        const double a = -lam * std::ldexp(1.0, 8 * d - 17);
        const double den = std::expm1(a * 256.0);
        for (int v = 0; v < 255; ++v) {
            const double F = d < 3 ? std::expm1(a * (double)(v + 1)) / den : -std::expm1(a * (double)(v + 1));
            t[d * 256 + v] = (uint64_t)std::floor(F * 4294967296.0);
        }
        t[d * 256 + 255] = ~0ull;
    }
}

constexpr uint64_t kTwo32 = 4294967296ull;

// Device form of a table: t_d[v] - 1 as u32 (every t_d[v] >= 2^24 since the
// most likely digit value has probability >= 1/256) and, per top byte b of
// the word, the counts at the two ends of its bucket [b 2^24, (b+1) 2^24).
void device_table(const uint64_t* t, uint32_t* out)
{
    uint16_t* guide = (uint16_t*)(out + 1024);
    for (int d = 0; d < 4; ++d) {
        const uint64_t* td = t + d * 256;
        for (int v = 0; v < 255; ++v) out[d * 256 + v] = (uint32_t)(td[v] - 1u);
        out[d * 256 + 255] = 0xFFFFFFFFu;
        auto count = [&](uint64_t w) {
            int c = 0;
            while (c < 255 && td[c] <= w) ++c;
            return c;
        };
        for (int b = 0; b < 256; ++b) {
            const int lo = count((uint64_t)b << 24), hi = count(((uint64_t)(b + 1) << 24) - 1u);
            guide[d * 256 + b] = (uint16_t)(lo | (hi << 8));
        }
    }
}

bool table_in_range(const uint64_t* t)
{
    for (int d = 0; d < 4; ++d)
        if (t[d * 256] < ((uint64_t)1 << 24)) return false;
    return true;
}

void free_pt(micsa_pt* c)
{
    if (!c) return;
    for (void* ptr : {(void*)c->rec, (void*)c->spins, (void*)c->perm, (void*)c->E, (void*)c->swaps, (void*)c->wtab,
                      (void*)c->ptab})
        if (ptr) (void)hipFree(ptr);
    for (auto& ev : c->events)
        for (hipEvent_t x : ev) (void)hipEventDestroy(x);
}

using EmcsKernel = void (*)(PtGeom, const int4*, uint64_t*, const int32_t*, int64_t*, const uint32_t*, uint32_t);

EmcsKernel emcs_kernel(int algo, bool houd, bool jl)
{
    if (algo == MICSA_PT_WALKERS)
        return houd ? (jl ? k_pt_emcs<0, true, true> : k_pt_emcs<0, true, false>)
                    : (jl ? k_pt_emcs<0, false, true> : k_pt_emcs<0, false, false>);
    return houd ? (jl ? k_pt_emcs<1, true, true> : k_pt_emcs<1, true, false>)
                : (jl ? k_pt_emcs<1, false, true> : k_pt_emcs<1, false, false>);
}

using RegKernel = void (*)(PtGeom, int, const int4*, uint64_t*, const int32_t*, int64_t*, const uint32_t*,
                          uint32_t);

template <int LX>
RegKernel reg_kernel_lx(int algo, bool houd)
{
    if (algo == MICSA_PT_WALKERS) return houd ? k_pt_emcs_reg<LX, 0, true> : k_pt_emcs_reg<LX, 0, false>;
    return houd ? k_pt_emcs_reg<LX, 1, true> : k_pt_emcs_reg<LX, 1, false>;
}

// Row lengths with a register-resident instance.
RegKernel reg_kernel(int Lx, int algo, bool houd)
{
    switch (Lx) {
    case 4: return reg_kernel_lx<4>(algo, houd);
    case 6: return reg_kernel_lx<6>(algo, houd);
    case 8: return reg_kernel_lx<8>(algo, houd);
    case 10: return reg_kernel_lx<10>(algo, houd);
    case 12: return reg_kernel_lx<12>(algo, houd);
    case 16: return reg_kernel_lx<16>(algo, houd);
    default: return nullptr;
    }
}

bool use_reg(const micsa_pt* c)
{
    return c->G > 0 && c->kernel != MICSA_PT_KERNEL_ROWS;
}

int launch_energy(micsa_pt* c)
{
    k_pt_energy<<<dim3((unsigned)c->g.M, (unsigned)(2 * c->g.runs)), 128, 0, c->stream>>>(c->g, c->rec, c->spins,
                                                                                          c->E);
    PT_TRY(c, hipGetLastError());
    return MICSA_OK;
}

int identity_perm(micsa_pt* c)
{
    std::vector<int32_t> perm((size_t)c->g.runs * 2 * c->g.M);
    for (size_t k = 0; k < perm.size(); ++k) perm[k] = (int32_t)(k % (size_t)c->g.M);
    PT_TRY(c, hipMemcpyAsync(c->perm, perm.data(), perm.size() * 4, hipMemcpyHostToDevice, c->stream));
    PT_TRY(c, hipStreamSynchronize(c->stream));
    return MICSA_OK;
}

bool pt_params_ok(const micsa_pt_params* p)
{
    auto even = [](int32_t L) { return L >= 2 && L % 2 == 0; };
    if (!even(p->Lx) || !even(p->Ly) || !even(p->Lz) || p->Lx > 64) return false;
    if ((int64_t)p->Lx * p->Ly * p->Lz > MICSA_PT_MAX_SITES) return false;
    if (p->n_runs < 1 || p->n_runs >= (1 << 24) || p->n_temps < 2 || p->n_temps > 64) return false;
    if (p->sweeps < 1 || p->sweeps > 64) return false;
    if (p->algo != MICSA_PT_WALKERS && p->algo != MICSA_PT_METROPOLIS) return false;
    return p->houdayer == 0 || p->houdayer == 1;
}

}  // namespace

extern "C" {

const char* micsa_pt_last_error(const micsa_pt* pt) { return pt ? pt->err.c_str() : "null context"; }

int micsa_pt_create(const micsa_pt_params* p, const double* J, const double* T, void* hip_stream, micsa_pt** out)
{
    if (!out) return MICSA_EINVAL;
    *out = nullptr;
    if (!p || !J || !T || !pt_params_ok(p)) return MICSA_EINVAL;
    const int N = p->Lx * p->Ly * p->Lz, M = p->n_temps;
    // couplings on the mesh
    std::vector<int32_t> Jq((size_t)3 * N);
    for (size_t k = 0; k < Jq.size(); ++k) {
        if (!(std::fabs(J[k]) <= 8.0)) return MICSA_EINVAL;
        Jq[k] = (int32_t)std::nearbyint(J[k] * 131072.0);
    }
    // temperature ladder and its tables
    for (int t = 0; t < M; ++t)
        if (!(T[t] > 0.0) || !std::isfinite(T[t]) || (t > 0 && !(T[t] > T[t - 1]))) return MICSA_EINVAL;
    std::vector<uint64_t> hw((size_t)M * 1024), hp((size_t)(M - 1) * 1024);
    std::vector<uint32_t> dw((size_t)M * kPtTable), dp((size_t)(M - 1) * kPtTable);
    for (int t = 0; t < M; ++t) {
        uint64_t* tw = hw.data() + (size_t)t * 1024;
        exp_table(1.0 / T[t], tw);
        // top digit below 255 always; walkers also below 64 (n < 2^30 in 32 bits)
        if (tw[3 * 256 + 254] != kTwo32 || !table_in_range(tw)) return MICSA_EINVAL;
        if (p->algo == MICSA_PT_WALKERS && tw[3 * 256 + 63] != kTwo32) return MICSA_EINVAL;
        device_table(tw, dw.data() + (size_t)t * kPtTable);
    }
    for (int t = 0; t + 1 < M; ++t) {
        uint64_t* tp = hp.data() + (size_t)t * 1024;
        exp_table(1.0 / T[t] - 1.0 / T[t + 1], tp);
        if (tp[3 * 256 + 254] != kTwo32 || !table_in_range(tp)) return MICSA_EINVAL;
        device_table(tp, dp.data() + (size_t)t * kPtTable);
    }

    micsa_pt* c = new (std::nothrow) micsa_pt();
    if (!c) return MICSA_ENOMEM;
    c->p = *p;
    c->stream = (hipStream_t)hip_stream;
    c->Jq = std::move(Jq);
    c->hw = std::move(hw);
    c->hp = std::move(hp);
    PtGeom& g = c->g;
    g.Lx = p->Lx;
    g.Ly = p->Ly;
    g.Lz = p->Lz;
    g.R0 = p->Ly * p->Lz;
    g.N = N;
    g.M = M;
    g.runs = p->n_runs;
    g.S = p->sweeps;
    g.key0 = (uint32_t)p->seed;
    g.key1 = (uint32_t)(p->seed >> 32);
    g.xmask = p->Lx == 64 ? ~0ull : ((1ull << p->Lx) - 1ull);
    const bool walkers = p->algo == MICSA_PT_WALKERS;
    c->jl = pt_lds_layout(g, true, walkers).total <= kPtLdsMax;
    c->lds = pt_lds_layout(g, c->jl, walkers).total;
    if (c->lds > kPtLdsMax) {  // spin rows and walkers alone exceed the LDS (short x rows, large N)
        delete c;
        return MICSA_EINVAL;
    }

    // coupling records, x-major: J+x, J+y, J+z, J-x, J-y, J-z, sum, 0
    std::vector<int32_t> rec((size_t)N * 8);
    for (int r = 0; r < g.R0; ++r) {
        const int y = r % g.Ly, z = r / g.Ly;
        for (int x = 0; x < g.Lx; ++x) {
            const int i = x + g.Lx * r;
            const int bx = (x + g.Lx - 1) % g.Lx + g.Lx * r;
            const int by = x + g.Lx * ((y + g.Ly - 1) % g.Ly + g.Ly * z);
            const int bz = x + g.Lx * (y + g.Ly * ((z + g.Lz - 1) % g.Lz));
            int32_t* o = rec.data() + ((size_t)x * g.R0 + r) * 8;
            o[0] = c->Jq[(size_t)0 * N + i];
            o[1] = c->Jq[(size_t)1 * N + i];
            o[2] = c->Jq[(size_t)2 * N + i];
            o[3] = c->Jq[(size_t)0 * N + bx];
            o[4] = c->Jq[(size_t)1 * N + by];
            o[5] = c->Jq[(size_t)2 * N + bz];
            o[6] = o[0] + o[1] + o[2] + o[3] + o[4] + o[5];
            o[7] = 0;
        }
    }
    const size_t nslot = (size_t)g.runs * 2 * M;
    bool ok = hipMalloc(&c->rec, (size_t)N * 32) == hipSuccess &&
              hipMalloc(&c->spins, nslot * g.R0 * 8) == hipSuccess && hipMalloc(&c->perm, nslot * 4) == hipSuccess &&
              hipMalloc(&c->E, nslot * 8) == hipSuccess &&
              hipMalloc(&c->swaps, (size_t)g.runs * 2 * (M - 1) * 8) == hipSuccess &&
              hipMalloc(&c->wtab, dw.size() * 4) == hipSuccess && hipMalloc(&c->ptab, std::max<size_t>(dp.size(), 1) * 4) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        free_pt(c);
        delete c;
        return MICSA_ENOMEM;
    }
    int st = MICSA_OK;
    auto fin = [&](int s) {
        if (s) {
            (void)hipStreamSynchronize(c->stream);
            free_pt(c);
            delete c;
        }
        return s;
    };
    if (hipMemcpyAsync(c->rec, rec.data(), rec.size() * 4, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->wtab, dw.data(), dw.size() * 4, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(c->ptab, dp.data(), dp.size() * 4, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess ||
        hipMemsetAsync(c->swaps, 0, (size_t)g.runs * 2 * (M - 1) * 8, c->stream) != hipSuccess)
        return fin(MICSA_EHIP);
    const int64_t rows_total = (int64_t)nslot * g.R0;
    k_pt_init_spins<<<(unsigned)((rows_total + 255) / 256), 256, 0, c->stream>>>(g, c->spins);
    if (hipGetLastError() != hipSuccess) return fin(MICSA_EHIP);
    if ((st = launch_energy(c))) return fin(st);
    if ((st = identity_perm(c))) return fin(st);
    if (c->lds > 65536u) {
        const EmcsKernel k = emcs_kernel(p->algo, p->houdayer != 0, c->jl);
        if (hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds) !=
            hipSuccess)
            return fin(MICSA_EHIP);
    }
    // register kernel: G temperatures per work-group, one row per thread
    if (reg_kernel(g.Lx, p->algo, p->houdayer != 0) && 2 * g.R0 <= 1024) {
        int G = std::min(M, 1024 / (2 * g.R0));
        while (G > 0 && pt_reg_layout(g, G).total > kPtLdsMax) --G;
        c->G = G;
        if (G > 0) {
            c->reg_lds = pt_reg_layout(g, G).total;
            if (c->reg_lds > 65536u &&
                hipFuncSetAttribute((const void*)reg_kernel(g.Lx, p->algo, p->houdayer != 0),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->reg_lds) != hipSuccess)
                return fin(MICSA_EHIP);
        }
    }
    *out = c;
    return MICSA_OK;
}

int micsa_pt_destroy(micsa_pt* pt)
{
    if (!pt) return MICSA_OK;
    (void)hipStreamSynchronize(pt->stream);
    free_pt(pt);
    delete pt;
    return MICSA_OK;
}

int micsa_pt_step(micsa_pt* pt, int64_t n)
{
    if (!pt || n < 0) return MICSA_EINVAL;
    if ((pt->e + n) * (int64_t)pt->g.S > (int64_t)UINT32_MAX) return pt_fail(pt, MICSA_ERANGE, "EMCS index range");
    const EmcsKernel k = emcs_kernel(pt->p.algo, pt->p.houdayer != 0, pt->jl);
    const dim3 grid((unsigned)pt->g.M, (unsigned)pt->g.runs);
    const bool reg = use_reg(pt);
    const RegKernel kr = reg ? reg_kernel(pt->g.Lx, pt->p.algo, pt->p.houdayer != 0) : nullptr;
    const dim3 rgrid((unsigned)((pt->g.M + pt->G - 1) / std::max(pt->G, 1)), (unsigned)pt->g.runs);
    const unsigned rblock = reg ? (unsigned)(64 * ((2 * pt->G * pt->g.R0 + 63) / 64)) : 0u;
    const unsigned sgrid = (unsigned)((2 * pt->g.runs + 3) / 4);
    for (int64_t i = 0; i < n; ++i) {
        const uint32_t e = (uint32_t)pt->e;
        std::array<hipEvent_t, 3> ev{};
        if (pt->timing) {
            for (auto& x : ev) PT_TRY(pt, hipEventCreate(&x));
            pt->events.push_back(ev);  // owned by the context from here on
            PT_TRY(pt, hipEventRecord(ev[0], pt->stream));
        }
        if (reg)
            kr<<<rgrid, rblock, pt->reg_lds, pt->stream>>>(pt->g, pt->G, pt->rec, pt->spins, pt->perm, pt->E,
                                                           pt->wtab, e);
        else
            k<<<grid, kPtBlock, pt->lds, pt->stream>>>(pt->g, pt->rec, pt->spins, pt->perm, pt->E, pt->wtab, e);
        PT_TRY(pt, hipGetLastError());
        if (pt->timing) PT_TRY(pt, hipEventRecord(ev[1], pt->stream));
        k_pt_swap<<<sgrid, 256, 0, pt->stream>>>(pt->g, pt->perm, pt->E, pt->swaps, pt->ptab, e);
        PT_TRY(pt, hipGetLastError());
        if (pt->timing) PT_TRY(pt, hipEventRecord(ev[2], pt->stream));
        pt->e += 1;
    }
    return MICSA_OK;
}

int micsa_pt_sync(micsa_pt* pt)
{
    if (!pt) return MICSA_EINVAL;
    PT_TRY(pt, hipStreamSynchronize(pt->stream));
    return MICSA_OK;
}

int micsa_pt_get_emcs(const micsa_pt* pt, int64_t* e)
{
    if (!pt || !e) return MICSA_EINVAL;
    *e = pt->e;
    return MICSA_OK;
}

int micsa_pt_read(micsa_pt* pt, int64_t* E, int64_t* Q)
{
    if (!pt) return MICSA_EINVAL;
    const PtGeom& g = pt->g;
    const size_t nslot = (size_t)g.runs * 2 * g.M;
    std::vector<int32_t> perm(nslot);
    std::vector<int64_t> Es(nslot);
    PT_TRY(pt, hipMemcpyAsync(perm.data(), pt->perm, nslot * 4, hipMemcpyDeviceToHost, pt->stream));
    PT_TRY(pt, hipMemcpyAsync(Es.data(), pt->E, nslot * 8, hipMemcpyDeviceToHost, pt->stream));
    std::vector<uint64_t> rows;
    if (Q) {
        rows.resize(nslot * g.R0);
        PT_TRY(pt, hipMemcpyAsync(rows.data(), pt->spins, rows.size() * 8, hipMemcpyDeviceToHost, pt->stream));
    }
    PT_TRY(pt, hipStreamSynchronize(pt->stream));
    for (int u = 0; u < g.runs; ++u)
        for (int t = 0; t < g.M; ++t) {
            const size_t b0 = ((size_t)u * 2 + 0) * g.M, b1 = ((size_t)u * 2 + 1) * g.M;
            if (E) {
                E[b0 + t] = Es[b0 + perm[b0 + t]];
                E[b1 + t] = Es[b1 + perm[b1 + t]];
            }
            if (Q) {  // sum_x s^a s^b = N - 2 (number of differing sites)
                const uint64_t* ra = rows.data() + (b0 + perm[b0 + t]) * g.R0;
                const uint64_t* rb = rows.data() + (b1 + perm[b1 + t]) * g.R0;
                int64_t d = 0;
                for (int r = 0; r < g.R0; ++r) d += __builtin_popcountll((ra[r] ^ rb[r]) & g.xmask);
                Q[(size_t)u * g.M + t] = g.N - 2 * d;
            }
        }
    return MICSA_OK;
}

int micsa_pt_read_spins(micsa_pt* pt, uint8_t* sigma)
{
    if (!pt || !sigma) return MICSA_EINVAL;
    const PtGeom& g = pt->g;
    const size_t nslot = (size_t)g.runs * 2 * g.M;
    std::vector<int32_t> perm(nslot);
    std::vector<uint64_t> rows(nslot * g.R0);
    PT_TRY(pt, hipMemcpyAsync(perm.data(), pt->perm, nslot * 4, hipMemcpyDeviceToHost, pt->stream));
    PT_TRY(pt, hipMemcpyAsync(rows.data(), pt->spins, rows.size() * 8, hipMemcpyDeviceToHost, pt->stream));
    PT_TRY(pt, hipStreamSynchronize(pt->stream));
    for (size_t grp = 0; grp < (size_t)g.runs * 2; ++grp)
        for (int t = 0; t < g.M; ++t) {
            const uint64_t* src = rows.data() + (grp * g.M + perm[grp * g.M + t]) * g.R0;
            uint8_t* dst = sigma + (grp * g.M + t) * g.N;
            for (int r = 0; r < g.R0; ++r)
                for (int x = 0; x < g.Lx; ++x) dst[x + g.Lx * r] = (uint8_t)((src[r] >> x) & 1u);
        }
    return MICSA_OK;
}

int micsa_pt_write_spins(micsa_pt* pt, const uint8_t* sigma)
{
    if (!pt || !sigma) return MICSA_EINVAL;
    const PtGeom& g = pt->g;
    const size_t nslot = (size_t)g.runs * 2 * g.M;
    std::vector<uint64_t> rows(nslot * g.R0, 0);
    for (size_t l = 0; l < nslot; ++l)
        for (int r = 0; r < g.R0; ++r) {
            uint64_t w = 0;
            for (int x = 0; x < g.Lx; ++x) {
                const uint8_t b = sigma[l * g.N + x + g.Lx * r];
                if (b > 1) return pt_fail(pt, MICSA_EINVAL, "spin bits must be 0 or 1");
                w |= (uint64_t)b << x;
            }
            rows[l * g.R0 + r] = w;
        }
    PT_TRY(pt, hipMemcpyAsync(pt->spins, rows.data(), rows.size() * 8, hipMemcpyHostToDevice, pt->stream));
    int st = identity_perm(pt);  // slot t now holds temperature t
    if (!st) st = launch_energy(pt);
    if (!st) PT_TRY(pt, hipStreamSynchronize(pt->stream));
    return st;
}

int micsa_pt_read_swaps(micsa_pt* pt, int64_t* swaps)
{
    if (!pt || !swaps) return MICSA_EINVAL;
    PT_TRY(pt, hipMemcpyAsync(swaps, pt->swaps, (size_t)pt->g.runs * 2 * (pt->g.M - 1) * 8, hipMemcpyDeviceToHost,
                              pt->stream));
    PT_TRY(pt, hipStreamSynchronize(pt->stream));
    return MICSA_OK;
}

int micsa_pt_get_tables(micsa_pt* pt, int32_t kind, int32_t index, uint64_t* t)
{
    if (!pt || !t) return MICSA_EINVAL;
    const std::vector<uint64_t>* src = nullptr;
    if (kind == 0 && index >= 0 && index < pt->g.M) src = &pt->hw;
    if (kind == 1 && index >= 0 && index + 1 < pt->g.M) src = &pt->hp;
    if (!src) return pt_fail(pt, MICSA_EINVAL, "table kind or index out of range");
    for (int d = 0; d < 4; ++d)
        std::memcpy(t + d * 255, src->data() + (size_t)index * 1024 + d * 256, 255 * 8);
    return MICSA_OK;
}

int micsa_pt_get_couplings(micsa_pt* pt, int32_t* Jq)
{
    if (!pt || !Jq) return MICSA_EINVAL;
    std::memcpy(Jq, pt->Jq.data(), pt->Jq.size() * 4);
    return MICSA_OK;
}

int micsa_pt_set_kernel(micsa_pt* pt, int32_t kernel)
{
    if (!pt) return MICSA_EINVAL;
    if (kernel != MICSA_PT_KERNEL_AUTO && kernel != MICSA_PT_KERNEL_ROWS && kernel != MICSA_PT_KERNEL_REGISTER)
        return pt_fail(pt, MICSA_EINVAL, "unknown tempering kernel");
    if (kernel == MICSA_PT_KERNEL_REGISTER && pt->G == 0)
        return pt_fail(pt, MICSA_EINVAL, "the register kernel needs Lx in {4, 6, 8, 10, 12, 16} and 2*Ly*Lz <= 1024");
    pt->kernel = kernel;
    return MICSA_OK;
}

const char* micsa_pt_kernel_name(const micsa_pt* pt)
{
    if (!pt) return "";
    return use_reg(pt) ? "k_pt_emcs_reg" : "k_pt_emcs";
}

int micsa_pt_set_timing(micsa_pt* pt, int32_t enable)
{
    if (!pt || (enable != 0 && enable != 1)) return MICSA_EINVAL;
    pt->timing = enable != 0;
    return MICSA_OK;
}

int micsa_pt_get_timing(micsa_pt* pt, int32_t kind, double* total_ms, int64_t* launches)
{
    if (!pt || kind < 0 || kind > 1) return MICSA_EINVAL;
    PT_TRY(pt, hipStreamSynchronize(pt->stream));
    for (auto& ev : pt->events) {
        for (int kd = 0; kd < 2; ++kd) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, ev[kd], ev[kd + 1]) == hipSuccess) {
                pt->time_ms[kd] += ms;
                pt->launches[kd] += 1;
            }
        }
        for (hipEvent_t x : ev) (void)hipEventDestroy(x);
    }
    pt->events.clear();
    if (total_ms) *total_ms = pt->time_ms[kind];
    if (launches) *launches = pt->launches[kind];
    return MICSA_OK;
}

}  // extern "C"
