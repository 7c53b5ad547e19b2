// picsub.hip -- MI355X (gfx950) implementation of the C ABI in picsub.h.
//
// Sub-cycled relativistic Boris push with order-p temporal Lagrange
// interpolation of E_y and B_z gathered from a 1D Yee grid
// (arXiv:2102.10983, Sec. III, Sec. IV with Algorithm 1, Sec. VI), for a
// batch of independent runs.
//
// Layout in HBM
//   particles: structure of arrays x, px, py, pz (double), k_old (int8),
//              status (uint8) and caller index (int32) per slot; each run's
//              slots are contiguous, sorted by position at load and padded
//              to RUN_ALIGN;
//   fields:    per run a ring of ring_depth levels, E[slot][ncells],
//              B[slot][ncells];
//   weights:   L^E_j, L^B_j for every (k, j) (setup.hpp);
//   runs:      RunDesc table (common.hpp), read once per wavefront;
//   counters:  [run][NSLOT][NCNT] uint64 slots filled with atomics.
//
// Floating point: built with -ffp-contract=off; the PIC_FP64 kernels
// evaluate the equations' expressions in their order with IEEE division and
// square root, so their results equal a plain scalar implementation's.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

#include "picsub.h"
#include "common.hpp"
#include "push_tile.hpp"
#include "push_wave.hpp"
#include "setup.hpp"
#include "mlp.hpp"
#include "push_fast.hpp"
#include "push_f32c.hpp"
#include "fields_yee.hpp"

using namespace picsub;

struct RunHost {
    pic_params prm;
    int64_t np = 0;          // particles of the run
    int64_t caller_off = 0;  // first caller index
    int64_t p_off = 0;       // first slot
    int64_t padded = 0;      // slots reserved
    double *ringE = nullptr, *ringB = nullptr;
    std::vector<int64_t> tags;   // level held by each ring slot
    bool driven = false;         // device-driven source set
    const double *table = nullptr;
    int64_t M = 0, co[6] = {0, 0, 0, 0, 0, 0};
    const double *atab = nullptr;   // potential lattice of the energy error (caller's memory)
    int64_t at[4] = {0, 0, 0, 0};   // its M, A, B, C
    int64_t n_dev = 0;           // level the device-driven counter reaches after queued work
    int64_t n_stop = INT64_MAX;  // device-driven stop level
    double x_origin0 = 0.0;      // x_origin at creation; the grid sits shift cells from it
    int64_t shift = 0;
};

// Staging area of pic_diag_noalloc: a layout of [counter sums: NCNT words,
// padded to 256 B][gamma, px, py, pz, x: PIC_DIAG_NOALLOC_MAX_NP doubles
// each][k_last: int8][status: uint8].  Every GPU the library runs on holds
// its own copy from the load of the code object until the process ends.
// Host code never passes the array's name to a kernel or a copy (on the host
// it only names the symbol): it uses the device address that
// hipGetSymbolAddress returned for the current device.
constexpr size_t NOALLOC_HEAD = 256;
constexpr size_t NOALLOC_BYTES = NOALLOC_HEAD + size_t(PIC_DIAG_NOALLOC_MAX_NP) * (5 * 8 + 2);
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};
hipError_t g_scratch_err[NOALLOC_MAX_DEVICES] = {};

// Once per device, with that device current (pic_batch_create's device):
// the device address of `scratch`.  A failure is kept and reported by
// pic_diag_noalloc; the other entry points do not need the array.
void scratch_setup(int device)
{
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device] || g_scratch_err[device] != hipSuccess) return;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess && p) g_scratch_ptr[device] = static_cast<unsigned char *>(p);
    else g_scratch_err[device] = e != hipSuccess ? e : hipErrorInvalidSymbol;
}

struct pic_ctx {
    std::vector<RunHost> runs;
    int32_t nruns = 0;
    int64_t np = 0;          // caller particles in all runs
    int64_t slots = 0;       // padded slots
    int32_t order = 3, kmax_all = 0, precision = PIC_FP64;
    hipStream_t stream = nullptr;
    int device = 0, ncu = 256;
    pic_tune tune{1, 256, PIC_BIN_NONE, 64, 0};
    bool have_particles = false;
    // particle store
    double *x = nullptr, *px = nullptr, *py = nullptr, *pz = nullptr;
    int8_t *kold = nullptr;
    uint8_t *status = nullptr;
    int32_t *perm = nullptr;
    int32_t *key = nullptr;
    // run table and group maps
    RunDesc *d_runs = nullptr;
    int32_t *group_run = nullptr, *group_order = nullptr;
    int8_t *group_prio = nullptr;
    int32_t ngroups = 0;
    double *wtab = nullptr;
    uint64_t *cnt = nullptr;
    // strict mode: non-finite particle or field input is refused (PIC_E_NUMERIC)
    bool strict = false;
    int32_t *d_flag = nullptr;
    // attached load predictor (pic_predictor_set)
    uint16_t *pred_w = nullptr;
    float *pred_norm = nullptr, *pred_feat = nullptr, *pred_score = nullptr;
    std::vector<float> pred_a0;
    float pred_width = 0.0625f;
    int32_t pred_every = 0;
    int64_t pred_calls = 0;
    uint64_t rebins = 0;
    // trajectory diagnostics (allocated when first switched on)
    double *r0 = nullptr, *rmax = nullptr, *work = nullptr, *werr = nullptr, *gmax = nullptr;
    bool deph = false;
    // energy error against the plane-wave solution: a_i and the running
    // maximum per slot (allocated at the first start; gerr: started for the
    // particles loaded now)
    double *ai = nullptr, *emax = nullptr;
    bool gerr = false;
    // k trace
    int8_t *ktrace = nullptr;
    int64_t kt_n0 = 0, kt_first = 0, kt_count = 0;
    int32_t kt_steps = 0;
    // captured windows
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int64_t graph_steps = 0;
    int32_t graph_S = 1;
    char err[512] = {0};
};

namespace {

pic_status fail(pic_ctx *ctx, pic_status st, const char *fmt, ...)
{
    if (ctx) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(ctx->err, sizeof ctx->err, fmt, ap);
        va_end(ap);
    }
    return st;
}

#define HIP_TRY(ctx, expr)                                                            \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail((ctx), PIC_E_DEVICE, "%s failed: %s", #expr,                  \
                        hipGetErrorString(e_));                                       \
    } while (0)

#define LAUNCH_CHECK(ctx)                                                             \
    do {                                                                              \
        hipError_t e_ = hipGetLastError();                                            \
        if (e_ != hipSuccess)                                                         \
            return fail((ctx), PIC_E_DEVICE, "kernel launch failed: %s",              \
                        hipGetErrorString(e_));                                       \
    } while (0)

#define CTX_CHECK(ctx)                                                                \
    do {                                                                              \
        if (!(ctx)) return PIC_E_ARG;                                                 \
        if (!(ctx)->x) return fail((ctx), PIC_E_STATE, "context not created");        \
    } while (0)

int grid_for(int64_t work, int block, int cap)
{
    int64_t g = (work + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return int(g);
}

size_t cnt_words(const pic_ctx *c) { return size_t(c->nruns) * NSLOT * NCNT; }

void free_all(pic_ctx *c)
{
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    void *ptrs[] = {c->x, c->px, c->py, c->pz, c->kold, c->status, c->perm, c->key,
                    c->d_runs, c->group_run, c->group_order, c->group_prio, c->wtab, c->cnt,
                    c->r0, c->rmax, c->work, c->werr, c->gmax, c->pred_w, c->pred_norm, c->pred_feat,
                    c->pred_score, c->d_flag, c->ai, c->emax};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (RunHost &r : c->runs) {
        if (r.ringE) (void)hipFree(r.ringE);
        if (r.ringB) (void)hipFree(r.ringB);
        r.ringE = r.ringB = nullptr;
    }
    c->x = c->px = c->py = c->pz = c->wtab = nullptr;
    c->kold = nullptr;
    c->status = nullptr;
    c->perm = c->key = c->group_run = c->group_order = nullptr;
    c->group_prio = nullptr;
    c->d_runs = nullptr;
    c->cnt = nullptr;
    c->r0 = c->rmax = c->work = c->werr = c->gmax = nullptr;
    c->deph = false;
    c->ai = c->emax = nullptr;
    c->gerr = false;
    c->pred_w = nullptr;
    c->pred_norm = c->pred_feat = c->pred_score = nullptr;
    c->pred_every = 0;
    c->d_flag = nullptr;
}

pic_status check_params(pic_ctx *ctx, const pic_params *p, int64_t np, int r)
{
    if (!p) return fail(ctx, PIC_E_ARG, "params of run %d are NULL", r);
    if (np < 0 || np > INT32_MAX) return fail(ctx, PIC_E_ARG, "run %d: np out of range", r);
    if (p->ncells < 2) return fail(ctx, PIC_E_ARG, "run %d: ncells must be >= 2", r);
    if (p->order != 1 && p->order != 2 && p->order != 3 && p->order != 5)
        return fail(ctx, PIC_E_ARG, "run %d: order must be 1, 2, 3 or 5 (got %d)", r, p->order);
    if (p->ring_depth < p->order + 1 || p->ring_depth > 1 << 20)
        return fail(ctx, PIC_E_ARG, "run %d: ring_depth must be in [order+1, 2^20]", r);
    if (p->k_max < 0 || p->k_max > PIC_K_MAX_LIMIT)
        return fail(ctx, PIC_E_ARG, "run %d: k_max must be in [0, %d]", r, PIC_K_MAX_LIMIT);
    if (!(p->dx > 0) || !(p->dt > 0)) return fail(ctx, PIC_E_ARG, "run %d: dx, dt must be > 0", r);
    if (!(p->dt <= 64.0 * p->dx)) return fail(ctx, PIC_E_ARG, "run %d: dt / dx must be <= 64", r);
    if (!(p->psi_max > 0)) return fail(ctx, PIC_E_ARG, "run %d: psi_max must be > 0", r);
    if (!(p->qm != 0) || p->qm != p->qm) return fail(ctx, PIC_E_ARG, "run %d: qm must be nonzero", r);
    if (p->x_origin != p->x_origin) return fail(ctx, PIC_E_ARG, "run %d: x_origin is NaN", r);
    if (p->precision != PIC_FP64 && p->precision != PIC_FP32_COMP &&
        p->precision != PIC_FP64_FAST)
        return fail(ctx, PIC_E_ARG, "run %d: unknown precision %d", r, p->precision);
    if (p->binning < PIC_BIN_NONE || p->binning > PIC_BIN_LEARNED)
        return fail(ctx, PIC_E_ARG, "run %d: unknown binning %d", r, p->binning);
    if (p->precision != PIC_FP64 && p->binning == PIC_BIN_BALLOT)
        return fail(ctx, PIC_E_ARG, "the tiled ballot push runs with PIC_FP64 only");
    if (int64_t(p->ring_depth) * p->ncells >= (int64_t(1) << 31))
        return fail(ctx, PIC_E_ARG, "run %d: ring_depth * ncells must stay below 2^31", r);
    if (int64_t(p->ncells) * 256 >= (int64_t(1) << 30))
        return fail(ctx, PIC_E_ARG, "run %d: ncells too large", r);
    return PIC_OK;
}

template <typename T>
pic_status dev_alloc(pic_ctx *ctx, T **p, size_t n)
{
    if (n == 0) n = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), n * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(ctx, PIC_E_NOMEM, "hipMalloc(%zu bytes) failed: %s", n * sizeof(T),
                    hipGetErrorString(e));
    }
    return PIC_OK;
}

// Strict mode: PIC_E_NUMERIC if any of a[0 .. n) (host or device memory)
// is not finite.  Synchronous.
pic_status check_finite(pic_ctx *ctx, pic_mem mem, const double *a, int64_t n, const char *what)
{
    if (!ctx->strict || n <= 0 || !a) return PIC_OK;
    int32_t bad = 0;
    if (mem == PIC_MEM_HOST) {
        for (int64_t i = 0; i < n && !bad; ++i) bad = !std::isfinite(a[i]);
    } else {
        HIP_TRY(ctx, hipMemsetAsync(ctx->d_flag, 0, sizeof(int32_t), ctx->stream));
        nonfinite_kernel<<<grid_for(n, 256, 4096), 256, 0, ctx->stream>>>(a, n, ctx->d_flag);
        LAUNCH_CHECK(ctx);
        HIP_TRY(ctx, hipMemcpyAsync(&bad, ctx->d_flag, sizeof bad, hipMemcpyDeviceToHost,
                                    ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    }
    if (bad) return fail(ctx, PIC_E_NUMERIC, "%s holds a value that is not finite", what);
    return PIC_OK;
}

RunDesc make_desc(const RunHost &r)
{
    RunDesc d{};
    d.ringE = r.ringE;
    d.ringB = r.ringB;
    d.table = r.table;
    d.x_origin = r.prm.x_origin;
    d.dx = r.prm.dx;
    d.dt = r.prm.dt;
    d.qm = r.prm.qm;
    d.psi_max = r.prm.psi_max;
    d.dtdx = r.prm.dt / r.prm.dx;
    d.p_off = r.p_off;
    d.np = r.np;
    d.n_cur = r.n_dev;
    d.n_stop = r.n_stop;
    d.M = r.M;
    d.aE = r.co[0];
    d.bE = r.co[1];
    d.cE = r.co[2];
    d.aB = r.co[3];
    d.bB = r.co[4];
    d.cB = r.co[5];
    d.atab = r.atab;
    d.atM = r.at[0];
    d.atA = r.at[1];
    d.atB = r.at[2];
    d.atC = r.at[3];
    d.D = r.prm.ring_depth;
    d.ncells = r.prm.ncells;
    d.kmax = r.prm.k_max;
    // |v| < c, so a particle crosses fewer than dt / dx cells per step
    d.margin = int32_t(std::ceil(r.prm.dt / r.prm.dx)) + 2;
    return d;
}

pic_status upload_desc(pic_ctx *ctx, int r)
{
    const RunDesc d = make_desc(ctx->runs[size_t(r)]);
    HIP_TRY(ctx, hipMemcpyAsync(ctx->d_runs + r, &d, sizeof d, hipMemcpyHostToDevice, ctx->stream));
    // the host copy goes out of scope: wait for the transfer
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return PIC_OK;
}

PushArgs push_args(pic_ctx *ctx, int64_t n0, int32_t S)
{
    PushArgs a{};
    a.runs = ctx->d_runs;
    a.group_run = ctx->group_run;
    a.group_order = ctx->group_order;
    a.group_prio = ctx->group_prio;
    a.x = ctx->x;
    a.px = ctx->px;
    a.py = ctx->py;
    a.pz = ctx->pz;
    a.kold = ctx->kold;
    a.status = ctx->status;
    a.perm = ctx->perm;
    a.wtab = ctx->wtab;
    a.ktrace = ctx->ktrace;
    a.r0 = ctx->deph ? ctx->r0 : nullptr;
    a.rmax = ctx->deph ? ctx->rmax : nullptr;
    a.work = ctx->deph ? ctx->work : nullptr;
    a.werr = ctx->deph ? ctx->werr : nullptr;
    a.gmax = ctx->deph ? ctx->gmax : nullptr;
    a.ai = ctx->deph && ctx->gerr ? ctx->ai : nullptr;
    a.emax = ctx->deph && ctx->gerr ? ctx->emax : nullptr;
    a.cnt = ctx->cnt;
    a.kt_n0 = ctx->kt_n0;
    a.kt_first = ctx->kt_first;
    a.kt_count = ctx->kt_count;
    a.kt_steps = ctx->kt_steps;
    a.n0 = n0;
    a.S = S;
    a.ngroups = ctx->ngroups;
    return a;
}

// DIAG: the trajectory diagnostics compiled in (only when they are switched
// on, so the kernels without them keep their register budget); the k trace
// is compiled in only for launches with a trace buffer attached.
template <int P, int WPG, bool DIAG>
void launch_wave(const PushArgs &a, int precision, int occupancy, hipStream_t s)
{
    const dim3 grid(unsigned((a.ngroups + WPG - 1) / WPG)), block(64 * WPG);
    if (precision == PIC_FP64) {
        if (a.ktrace) push_wave_kernel<P, WPG, DIAG, true><<<grid, block, 0, s>>>(a);
        else push_wave_kernel<P, WPG, DIAG, false><<<grid, block, 0, s>>>(a);
    } else if (precision == PIC_FP64_FAST && occupancy >= 5 && WPG == 1 && !DIAG && P <= 3) {
        // register budgets for 5, 6 or 7 wavefronts per SIMD
        if (occupancy == 5) {
            if (a.ktrace) push_fast_kernel<P, 1, false, true, 5><<<grid, block, 0, s>>>(a);
            else push_fast_kernel<P, 1, false, false, 5><<<grid, block, 0, s>>>(a);
        } else if (occupancy == 6) {
            if (a.ktrace) push_fast_kernel<P, 1, false, true, 6><<<grid, block, 0, s>>>(a);
            else push_fast_kernel<P, 1, false, false, 6><<<grid, block, 0, s>>>(a);
        } else {
            if (a.ktrace) push_fast_kernel<P, 1, false, true, 7><<<grid, block, 0, s>>>(a);
            else push_fast_kernel<P, 1, false, false, 7><<<grid, block, 0, s>>>(a);
        }
    } else if (precision == PIC_FP64_FAST) {
        if (a.ktrace) push_fast_kernel<P, WPG, DIAG, true><<<grid, block, 0, s>>>(a);
        else push_fast_kernel<P, WPG, DIAG, false><<<grid, block, 0, s>>>(a);
    } else {
        push_wave_fp32c_kernel<P, WPG, DIAG><<<grid, block, 0, s>>>(a);
    }
}

template <int P, bool DIAG>
void launch_shape(const PushArgs &a, const pic_tune &t, int precision, int64_t slots, hipStream_t s)
{
    if (t.binning == PIC_BIN_BALLOT) {
        const dim3 grid(unsigned(slots / t.tile));
        switch (t.tile) {
        case 128: push_tile_kernel<P, 128, DIAG><<<grid, dim3(128), 0, s>>>(a); break;
        case 512: push_tile_kernel<P, 512, DIAG><<<grid, dim3(512), 0, s>>>(a); break;
        default: push_tile_kernel<P, 256, DIAG><<<grid, dim3(256), 0, s>>>(a); break;
        }
        return;
    }
    switch (t.waves_per_group) {
    case 2: launch_wave<P, 2, DIAG>(a, precision, t.occupancy, s); break;
    case 4: launch_wave<P, 4, DIAG>(a, precision, t.occupancy, s); break;
    default: launch_wave<P, 1, DIAG>(a, precision, t.occupancy, s); break;
    }
}

template <int P>
void launch_order(const PushArgs &a, const pic_tune &t, int precision, int64_t slots, hipStream_t s)
{
    if (a.rmax) launch_shape<P, true>(a, t, precision, slots, s);
    else launch_shape<P, false>(a, t, precision, slots, s);
}

pic_status launch_push(pic_ctx *ctx, int64_t n0, int32_t S, hipStream_t s)
{
    const PushArgs a = push_args(ctx, n0, S);
    switch (ctx->order) {
    case 1: launch_order<1>(a, ctx->tune, ctx->precision, ctx->slots, s); break;
    case 2: launch_order<2>(a, ctx->tune, ctx->precision, ctx->slots, s); break;
    case 3: launch_order<3>(a, ctx->tune, ctx->precision, ctx->slots, s); break;
    default: launch_order<5>(a, ctx->tune, ctx->precision, ctx->slots, s); break;
    }
    LAUNCH_CHECK(ctx);
    return PIC_OK;
}

// Device-driven window: fill every run's levels n_cur .. n_cur + S - 1,
// push S steps from n_cur, move n_cur on.  No host state is read, so the
// sequence can be captured into a graph.
pic_status enqueue_window(pic_ctx *ctx, int32_t S, hipStream_t s)
{
    int32_t maxcells = 0;
    for (const RunHost &r : ctx->runs) maxcells = std::max(maxcells, r.prm.ncells);
    const int64_t work = int64_t(S) * maxcells;
    const dim3 lgrid(unsigned(grid_for(work, 256, 4096)), unsigned(ctx->nruns));
    batch_lattice_kernel<<<lgrid, 256, 0, s>>>(ctx->d_runs, S);
    LAUNCH_CHECK(ctx);
    pic_status st = launch_push(ctx, NO_LEVEL, S, s);
    if (st) return st;
    tick_kernel<<<(ctx->nruns + 255) / 256, 256, 0, s>>>(ctx->d_runs, ctx->nruns, S);
    LAUNCH_CHECK(ctx);
    return PIC_OK;
}

pic_status check_window(pic_ctx *ctx, int32_t S)
{
    if (S < 1) return fail(ctx, PIC_E_ARG, "S must be >= 1");
    if (!ctx->have_particles) return fail(ctx, PIC_E_STATE, "particles not loaded");
    for (int r = 0; r < ctx->nruns; ++r) {
        const RunHost &R = ctx->runs[size_t(r)];
        if (!R.driven) return fail(ctx, PIC_E_STATE, "run %d has no field source", r);
        if (int64_t(S) + R.prm.order > R.prm.ring_depth)
            return fail(ctx, PIC_E_LEVEL, "run %d: S + order = %d exceeds ring_depth %d", r,
                        S + R.prm.order, R.prm.ring_depth);
    }
    return PIC_OK;
}

void mirror_advance(pic_ctx *ctx, int64_t steps, int32_t S)
{
    // the device moves in windows of S, each clamped at the run's stop level
    for (RunHost &R : ctx->runs) {
        for (int64_t done = 0; done < steps; done += S) {
            const int64_t left = R.n_stop - R.n_dev;
            const int64_t w = left <= 0 ? 0 : std::min<int64_t>(left, S);
            for (int64_t m = R.n_dev; m < R.n_dev + w; ++m)
                R.tags[size_t(mod_floor(m, R.prm.ring_depth))] = m;
            R.n_dev += w;
        }
    }
}

// pic_counters from the counter words summed over slots (and runs): steps
// per k, clamps, lost; sub-steps are 4^k per step, N* the sub-steps of k > 0
// (Sec. VII).
void counters_from_sums(const uint64_t (&sum)[NCNT], uint64_t rebins, pic_counters *cnt)
{
    std::memset(cnt, 0, sizeof *cnt);
    for (int k = 0; k < PIC_KHIST; ++k) {
        cnt->steps_by_k[k] = sum[k];
        const uint64_t sub = sum[k] << (2 * k);
        cnt->sub_steps_by_k[k] = sub;
        cnt->steps += sum[k];
        cnt->sub_steps += sub;
        if (k > 0) cnt->n_star += sub;
    }
    cnt->clamps = sum[CNT_CLAMPS];
    cnt->lost = sum[CNT_LOST];
    cnt->rebins = rebins;
}

pic_status read_counters(pic_ctx *ctx, int32_t run, pic_counters *cnt)
{
    std::vector<uint64_t> h(cnt_words(ctx));
    HIP_TRY(ctx, hipMemcpyAsync(h.data(), ctx->cnt, h.size() * sizeof(uint64_t),
                                hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    uint64_t sum[NCNT] = {0};
    for (int r = 0; r < ctx->nruns; ++r) {
        if (run >= 0 && r != run) continue;
        for (int b = 0; b < NSLOT; ++b) {
            const uint64_t *v = h.data() + (size_t(r) * NSLOT + b) * NCNT;
            for (int j = 0; j < NCNT; ++j) sum[j] += v[j];
        }
    }
    counters_from_sums(sum, ctx->rebins, cnt);
    return PIC_OK;
}

// The attached predictor before a push: every pred_every-th call scores
// every particle at level n (NO_LEVEL: each run's device-driven level) and
// re-orders the groups, heaviest first (one bucket: particles keep their
// slots).  Synchronises the stream.
pic_status predictor_turn(pic_ctx *ctx, int64_t n)
{
    if (!ctx->pred_w || ctx->pred_every <= 0) return PIC_OK;
    if (ctx->gexec) return PIC_OK;         // no re-binning while a captured graph is held
    if (ctx->pred_calls++ % ctx->pred_every != 0) return PIC_OK;
    pic_status st = pic_features(ctx, n, ctx->pred_a0.data(), ctx->pred_feat);
    if (st) return st;
    st = pic_mlp_forward(ctx->pred_w, ctx->pred_norm, ctx->pred_feat, ctx->pred_score, ctx->np,
                         ctx->stream);
    if (st) return fail(ctx, st, "predictor forward pass failed");
    st = pic_prebin(ctx, ctx->pred_score, 1, ctx->pred_width, 0);
    if (st) return st;
    ++ctx->rebins;
    return PIC_OK;
}

}  // namespace

extern "C" {

pic_status pic_batch_create(const pic_params *per_run, const int64_t *np, int32_t nruns,
                            void *hip_stream, pic_ctx **out)
{
    if (!out) return PIC_E_ARG;
    *out = nullptr;
    pic_ctx *ctx = new (std::nothrow) pic_ctx;
    if (!ctx) return PIC_E_NOMEM;
    *out = ctx;    // a failed create still carries its message
    if (!per_run || !np || nruns < 1 || nruns > 65536)
        return fail(ctx, PIC_E_ARG, "need 1..65536 runs with params and counts");
    for (int r = 0; r < nruns; ++r) {
        pic_status st = check_params(ctx, per_run + r, np[r], r);
        if (st) return st;
        if (per_run[r].order != per_run[0].order || per_run[r].precision != per_run[0].precision ||
            per_run[r].binning != per_run[0].binning)
            return fail(ctx, PIC_E_ARG, "runs of a batch share order, precision and binning");
    }
    ctx->nruns = nruns;
    ctx->order = per_run[0].order;
    ctx->precision = per_run[0].precision;
    ctx->tune.binning = per_run[0].binning == PIC_BIN_BALLOT ? PIC_BIN_BALLOT : PIC_BIN_NONE;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipGetDevice(&ctx->device);
    if (e != hipSuccess) return fail(ctx, PIC_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    (void)hipDeviceGetAttribute(&ctx->ncu, hipDeviceAttributeMultiprocessorCount, ctx->device);
    scratch_setup(ctx->device);
    ctx->runs.resize(size_t(nruns));
    int64_t caller = 0, slot = 0;
    for (int r = 0; r < nruns; ++r) {
        RunHost &R = ctx->runs[size_t(r)];
        R.prm = per_run[r];
        R.x_origin0 = R.prm.x_origin;
        R.np = np[r];
        R.caller_off = caller;
        R.p_off = slot;
        R.padded = (np[r] + RUN_ALIGN - 1) / RUN_ALIGN * RUN_ALIGN;
        if (R.padded == 0) R.padded = RUN_ALIGN;     // every run owns at least one tile
        caller += np[r];
        slot += R.padded;
        ctx->kmax_all = std::max(ctx->kmax_all, R.prm.k_max);
        R.tags.assign(size_t(R.prm.ring_depth), NO_LEVEL);
    }
    ctx->np = caller;
    ctx->slots = slot;
    if (slot / 64 > INT32_MAX) return fail(ctx, PIC_E_ARG, "too many particles");
    ctx->ngroups = int32_t(slot / 64);
    const size_t n = size_t(slot);
    pic_status st;
    if ((st = dev_alloc(ctx, &ctx->x, n)) || (st = dev_alloc(ctx, &ctx->px, n)) ||
        (st = dev_alloc(ctx, &ctx->py, n)) || (st = dev_alloc(ctx, &ctx->pz, n)) ||
        (st = dev_alloc(ctx, &ctx->kold, n)) || (st = dev_alloc(ctx, &ctx->status, n)) ||
        (st = dev_alloc(ctx, &ctx->perm, n)) || (st = dev_alloc(ctx, &ctx->key, size_t(caller))) ||
        (st = dev_alloc(ctx, &ctx->d_runs, size_t(nruns))) ||
        (st = dev_alloc(ctx, &ctx->group_run, size_t(ctx->ngroups))) ||
        (st = dev_alloc(ctx, &ctx->group_order, size_t(ctx->ngroups))) ||
        (st = dev_alloc(ctx, &ctx->group_prio, size_t(ctx->ngroups))) ||
        (st = dev_alloc(ctx, &ctx->wtab, size_t(wtab_entries(ctx->kmax_all)) * 2 * (ctx->order + 1))) ||
        (st = dev_alloc(ctx, &ctx->cnt, cnt_words(ctx))) ||
        (st = dev_alloc(ctx, &ctx->d_flag, 1))) {
        free_all(ctx);
        return st;
    }
    for (RunHost &R : ctx->runs) {
        const size_t ring = size_t(R.prm.ring_depth) * R.prm.ncells;
        if ((st = dev_alloc(ctx, &R.ringE, ring)) || (st = dev_alloc(ctx, &R.ringB, ring))) {
            free_all(ctx);
            return st;
        }
    }
    // group maps: run of each 64-slot group, dispatch in slot order
    std::vector<int32_t> grun(size_t(ctx->ngroups)), gord(size_t(ctx->ngroups));
    for (int r = 0; r < nruns; ++r) {
        const RunHost &R = ctx->runs[size_t(r)];
        for (int64_t g = R.p_off / 64; g < (R.p_off + R.padded) / 64; ++g) grun[size_t(g)] = r;
    }
    std::iota(gord.begin(), gord.end(), 0);
    std::vector<RunDesc> descs;
    for (const RunHost &R : ctx->runs) descs.push_back(make_desc(R));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->group_run, grun.data(), grun.size() * 4, hipMemcpyHostToDevice,
                                ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->group_order, gord.data(), gord.size() * 4,
                                hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->d_runs, descs.data(), descs.size() * sizeof(RunDesc),
                                hipMemcpyHostToDevice, ctx->stream));
    const int64_t went = wtab_entries(ctx->kmax_all);
    weights_kernel<<<grid_for(went, 256, 4096), 256, 0, ctx->stream>>>(ctx->wtab, ctx->order,
                                                                        ctx->kmax_all);
    LAUNCH_CHECK(ctx);
    HIP_TRY(ctx, hipMemsetAsync(ctx->cnt, 0, cnt_words(ctx) * sizeof(uint64_t), ctx->stream));
    HIP_TRY(ctx, hipMemsetAsync(ctx->status, PIC_PARTICLE_LOST, n, ctx->stream));
    HIP_TRY(ctx, hipMemsetAsync(ctx->perm, 0xFF, n * sizeof(int32_t), ctx->stream));
    HIP_TRY(ctx, hipMemsetAsync(ctx->group_prio, 0, size_t(ctx->ngroups), ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return PIC_OK;
}

pic_status pic_create(const pic_params *prm, int64_t np, void *hip_stream, pic_ctx **out)
{
    return pic_batch_create(prm, &np, 1, hip_stream, out);
}

pic_status pic_destroy(pic_ctx *ctx)
{
    if (!ctx) return PIC_E_ARG;
    if (ctx->x) (void)hipStreamSynchronize(ctx->stream);
    free_all(ctx);
    delete ctx;
    return PIC_OK;
}

const char *pic_last_error(const pic_ctx *ctx)
{
    return ctx ? ctx->err : "null context";
}

namespace {
// Load the particle state (caller order, host or device arrays), sort it
// into slots by (run, position bin) and reset counters and group order.
// status may be NULL (every particle live).
pic_status load_particles(pic_ctx *ctx, pic_mem mem, const double *x, const double *px,
                          const double *py, const double *pz, const int8_t *k_old,
                          const uint8_t *status)
{
    const int64_t np = ctx->np;
    if (np > 0 && (!x || !px || !py || !pz)) return fail(ctx, PIC_E_ARG, "null particle array");
    if (mem != PIC_MEM_HOST && mem != PIC_MEM_DEVICE) return fail(ctx, PIC_E_ARG, "bad pic_mem");
    {
        const double *arr[4] = {x, px, py, pz};
        const char *name[4] = {"x", "px", "py", "pz"};
        for (int a = 0; a < 4; ++a) {
            pic_status s = check_finite(ctx, mem, arr[a], np, name[a]);
            if (s) return s;
        }
    }
    const size_t n = size_t(np);
    const double *dx_ = x, *dpx = px, *dpy = py, *dpz = pz;
    const int8_t *dk = k_old;
    const uint8_t *dst = status;
    double *tmp = nullptr;
    int8_t *tmpk = nullptr;
    uint8_t *tmps_ = nullptr;
    int32_t *hist = nullptr, *sums = nullptr;
    LoadRun *dlr = nullptr;
    pic_status result = PIC_OK;
    hipError_t e = hipSuccess;
    std::vector<LoadRun> lr(size_t(ctx->nruns));
    int64_t nb = 0, nchunks = 0;
    if (mem == PIC_MEM_HOST && np > 0) {
        if ((result = dev_alloc(ctx, &tmp, 4 * n))) return result;
        if ((k_old && (result = dev_alloc(ctx, &tmpk, n))) ||
            (status && (result = dev_alloc(ctx, &tmps_, n)))) {
            (void)hipFree(tmp);
            if (tmpk) (void)hipFree(tmpk);
            return result;
        }
        const double *src[4] = {x, px, py, pz};
        for (int a = 0; a < 4 && e == hipSuccess; ++a)
            e = hipMemcpyAsync(tmp + a * n, src[a], n * sizeof(double), hipMemcpyHostToDevice,
                               ctx->stream);
        if (e == hipSuccess && k_old)
            e = hipMemcpyAsync(tmpk, k_old, n, hipMemcpyHostToDevice, ctx->stream);
        if (e == hipSuccess && status)
            e = hipMemcpyAsync(tmps_, status, n, hipMemcpyHostToDevice, ctx->stream);
        dst = tmps_;
        dx_ = tmp;
        dpx = tmp + n;
        dpy = tmp + 2 * n;
        dpz = tmp + 3 * n;
        dk = tmpk;
    }
    // counting sort by (run, position bin)
    for (int r = 0; r < ctx->nruns; ++r) {
        const RunHost &R = ctx->runs[size_t(r)];
        lr[size_t(r)] = LoadRun{R.caller_off, R.np, R.p_off, nb, R.prm.x_origin, R.prm.dx,
                                R.prm.ncells, 0};
        nb += int64_t(R.prm.ncells) * ctx->tune.sort_sub + 1;
    }
    nchunks = (nb + SCAN_CHUNK - 1) / SCAN_CHUNK;
    if (e == hipSuccess) e = hipMemsetAsync(ctx->perm, 0xFF, size_t(ctx->slots) * sizeof(int32_t),
                                            ctx->stream);
    if (e == hipSuccess && np > 0) {
        if ((result = dev_alloc(ctx, &hist, size_t(nb))) ||
            (result = dev_alloc(ctx, &sums, size_t(nchunks))) ||
            (result = dev_alloc(ctx, &dlr, lr.size())))
            goto done;
        e = hipMemcpyAsync(dlr, lr.data(), lr.size() * sizeof(LoadRun), hipMemcpyHostToDevice,
                           ctx->stream);
        if (e == hipSuccess) e = hipMemsetAsync(hist, 0, size_t(nb) * sizeof(int32_t), ctx->stream);
        if (e == hipSuccess) {
            key_kernel<<<grid_for(np, 256, 8192), 256, 0, ctx->stream>>>(
                dx_, np, dlr, ctx->nruns, ctx->tune.sort_sub, ctx->key, hist);
            scan_sums_kernel<<<unsigned(nchunks), 256, 0, ctx->stream>>>(hist, nb, sums);
            scan_top_kernel<<<1, 1024, 0, ctx->stream>>>(sums, int(nchunks));
            scan_chunk_kernel<<<unsigned(nchunks), 256, 0, ctx->stream>>>(hist, nb, sums);
            scatter_kernel<<<grid_for(np, 256, 8192), 256, 0, ctx->stream>>>(ctx->key, np, dlr,
                                                                          ctx->nruns, hist, ctx->perm);
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess) {
        gather_state_kernel<<<grid_for(ctx->slots, 256, 8192), 256, 0, ctx->stream>>>(
            ctx->perm, ctx->slots, dx_, dpx, dpy, dpz, dk, ctx->x, ctx->px, ctx->py, ctx->pz,
            ctx->kold, ctx->status, dst);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemsetAsync(ctx->cnt, 0, cnt_words(ctx) * sizeof(uint64_t), ctx->stream);
    ctx->rebins = 0;
    if (e == hipSuccess)
        e = hipMemsetAsync(ctx->group_prio, 0, size_t(ctx->ngroups), ctx->stream);
    if (e == hipSuccess) {
        std::vector<int32_t> id(size_t(ctx->ngroups));
        std::iota(id.begin(), id.end(), 0);
        e = hipMemcpyAsync(ctx->group_order, id.data(), id.size() * 4, hipMemcpyHostToDevice,
                           ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    }
    ctx->gerr = false;                            // new particles: no a_i for them yet
    if (e == hipSuccess && ctx->r0) {            // new particles: the diagnostics restart
                                                  // (their values belong to slots)
        diag_init_kernel<<<grid_for(ctx->slots, 256, 8192), 256, 0, ctx->stream>>>(
            ctx->slots, ctx->px, ctx->py, ctx->pz, ctx->r0, ctx->rmax, ctx->work, ctx->werr,
            ctx->gmax);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) result = fail(ctx, PIC_E_DEVICE, "particle load: %s", hipGetErrorString(e));
    else ctx->have_particles = true;
done:
    (void)hipStreamSynchronize(ctx->stream);
    void *tmps[] = {tmp, tmpk, tmps_, hist, sums, dlr};
    for (void *p : tmps)
        if (p) (void)hipFree(p);
    return result;
}
}  // namespace

pic_status pic_particles_set(pic_ctx *ctx, pic_mem mem, const double *x, const double *px,
                             const double *py, const double *pz, const int8_t *k_old)
{
    CTX_CHECK(ctx);
    return load_particles(ctx, mem, x, px, py, pz, k_old, nullptr);
}

pic_status pic_fields_load_r(pic_ctx *ctx, int32_t run, int64_t n, pic_mem mem, const double *Ey,
                             const double *Bz)
{
    CTX_CHECK(ctx);
    if (run < 0 || run >= ctx->nruns) return fail(ctx, PIC_E_ARG, "bad run %d", run);
    if (!Ey || !Bz) return fail(ctx, PIC_E_ARG, "null field array");
    if (mem != PIC_MEM_HOST && mem != PIC_MEM_DEVICE) return fail(ctx, PIC_E_ARG, "bad pic_mem");
    RunHost &R = ctx->runs[size_t(run)];
    pic_status fs;
    if ((fs = check_finite(ctx, mem, Ey, R.prm.ncells, "Ey")) ||
        (fs = check_finite(ctx, mem, Bz, R.prm.ncells, "Bz")))
        return fs;
    const int64_t slot = mod_floor(n, R.prm.ring_depth);
    const size_t bytes = size_t(R.prm.ncells) * sizeof(double);
    const hipMemcpyKind kind = mem == PIC_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    HIP_TRY(ctx, hipMemcpyAsync(R.ringE + slot * R.prm.ncells, Ey, bytes, kind, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(R.ringB + slot * R.prm.ncells, Bz, bytes, kind, ctx->stream));
    if (mem == PIC_MEM_HOST) HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    R.tags[size_t(slot)] = n;
    return PIC_OK;
}

pic_status pic_fields_load(pic_ctx *ctx, int64_t n, pic_mem mem, const double *Ey, const double *Bz)
{
    return pic_fields_load_r(ctx, 0, n, mem, Ey, Bz);
}

pic_status pic_fields_load_lattice_r(pic_ctx *ctx, int32_t run, int64_t n_first, int32_t count,
                                     const double *table, int64_t M, int64_t aE, int64_t bE,
                                     int64_t cE, int64_t aB, int64_t bB, int64_t cB)
{
    CTX_CHECK(ctx);
    if (run < 0 || run >= ctx->nruns) return fail(ctx, PIC_E_ARG, "bad run %d", run);
    if (!table || M <= 0) return fail(ctx, PIC_E_ARG, "bad table");
    RunHost &R = ctx->runs[size_t(run)];
    const int D = R.prm.ring_depth;
    if (count < 0 || count > D) return fail(ctx, PIC_E_ARG, "count must be in [0, ring_depth]");
    if (pic_status fs = check_finite(ctx, PIC_MEM_DEVICE, table, M, "the phase table")) return fs;
    if (count == 0) return PIC_OK;
    const int64_t work = int64_t(count) * R.prm.ncells;
    lattice_kernel<<<grid_for(work, 256, 16384), 256, 0, ctx->stream>>>(
        R.ringE, R.ringB, D, R.prm.ncells, n_first, count, table, M, aE, bE, cE, aB, bB, cB);
    LAUNCH_CHECK(ctx);
    for (int32_t c = 0; c < count; ++c) R.tags[size_t(mod_floor(n_first + c, D))] = n_first + c;
    return PIC_OK;
}

pic_status pic_fields_load_lattice(pic_ctx *ctx, int64_t n_first, int32_t count, const double *table,
                                   int64_t M, int64_t aE, int64_t bE, int64_t cE, int64_t aB,
                                   int64_t bB, int64_t cB)
{
    return pic_fields_load_lattice_r(ctx, 0, n_first, count, table, M, aE, bE, cE, aB, bB, cB);
}

pic_status pic_fields_yee_r(pic_ctx *ctx, int32_t run, int64_t n_first, int32_t count,
                           const double *table, int64_t M, int64_t aB, int64_t cB)
{
    CTX_CHECK(ctx);
    if (run < 0 || run >= ctx->nruns) return fail(ctx, PIC_E_ARG, "bad run %d", run);
    if (!table || M <= 0) return fail(ctx, PIC_E_ARG, "bad table");
    RunHost &R = ctx->runs[size_t(run)];
    const int D = R.prm.ring_depth;
    const int32_t N = R.prm.ncells;
    if (pic_status fs = check_finite(ctx, PIC_MEM_DEVICE, table, M, "the phase table")) return fs;
    if (count < 0 || count > D - 1) return fail(ctx, PIC_E_ARG, "count must be in [0, ring_depth - 1]");
    if (N < 2) return fail(ctx, PIC_E_ARG, "the Yee solver needs two or more cells");
    if (count == 0) return PIC_OK;
    if (R.tags[size_t(mod_floor(n_first - 1, D))] != n_first - 1)
        return fail(ctx, PIC_E_LEVEL, "level %lld (the solver's start) is not in the ring",
                    (long long)(n_first - 1));
    const double dx = R.prm.dx, dt = R.prm.dt;
    const double nu = dt / dx, kappa = (dt - dx) / (dt + dx);
    constexpr int WT = 64 * YEE_R - 2 * (YEE_T + 2);
    const unsigned tiles = unsigned((N + WT - 1) / WT);
    const int per = std::min(YEE_T, D - 1);
    for (int32_t c = 0; c < count; c += per) {
        const int cnt = std::min(per, count - c);
        yee_kernel<YEE_R, YEE_T><<<tiles, 64, 0, ctx->stream>>>(R.ringE, R.ringB, D, N,
                                                                 n_first + c, cnt, nu, kappa,
                                                                 table, M, aB, cB);
        LAUNCH_CHECK(ctx);
    }
    for (int32_t c = 0; c < count; ++c) R.tags[size_t(mod_floor(n_first + c, D))] = n_first + c;
    return PIC_OK;
}

pic_status pic_fields_yee(pic_ctx *ctx, int64_t n_first, int32_t count, const double *table,
                         int64_t M, int64_t aB, int64_t cB)
{
    return pic_fields_yee_r(ctx, 0, n_first, count, table, M, aB, cB);
}

pic_status pic_fields_read_r(pic_ctx *ctx, int32_t run, int64_t n, pic_mem mem, double *Ey,
                             double *Bz)
{
    CTX_CHECK(ctx);
    if (run < 0 || run >= ctx->nruns) return fail(ctx, PIC_E_ARG, "bad run %d", run);
    if (mem != PIC_MEM_HOST && mem != PIC_MEM_DEVICE) return fail(ctx, PIC_E_ARG, "bad pic_mem");
    RunHost &R = ctx->runs[size_t(run)];
    const int64_t slot = mod_floor(n, R.prm.ring_depth);
    if (R.driven || R.tags[size_t(slot)] != n)
        return fail(ctx, PIC_E_LEVEL, "level %lld is not in the ring", (long long)n);
    const size_t bytes = size_t(R.prm.ncells) * sizeof(double);
    const hipMemcpyKind kind = mem == PIC_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
    if (Ey) HIP_TRY(ctx, hipMemcpyAsync(Ey, R.ringE + slot * R.prm.ncells, bytes, kind, ctx->stream));
    if (Bz) HIP_TRY(ctx, hipMemcpyAsync(Bz, R.ringB + slot * R.prm.ncells, bytes, kind, ctx->stream));
    if (mem == PIC_MEM_HOST) HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return PIC_OK;
}

pic_status pic_fields_read(pic_ctx *ctx, int64_t n, pic_mem mem, double *Ey, double *Bz)
{
    return pic_fields_read_r(ctx, 0, n, mem, Ey, Bz);
}

pic_status pic_source_set(pic_ctx *ctx, int32_t run, int64_t n_start, int64_t n_stop,
                          const double *table, int64_t M, int64_t aE, int64_t bE, int64_t cE,
                          int64_t aB, int64_t bB, int64_t cB)
{
    CTX_CHECK(ctx);
    if (run < 0 || run >= ctx->nruns) return fail(ctx, PIC_E_ARG, "bad run %d", run);
    if (!table || M <= 0) return fail(ctx, PIC_E_ARG, "bad table");
    if (n_stop < n_start) return fail(ctx, PIC_E_ARG, "n_stop before n_start");
    if (pic_status fs = check_finite(ctx, PIC_MEM_DEVICE, table, M, "the phase table")) return fs;
    RunHost &R = ctx->runs[size_t(run)];
    R.driven = true;
    R.n_stop = n_stop;
    R.table = table;
    R.M = M;
    const int64_t co[6] = {aE, bE, cE, aB, bB, cB};
    std::copy(co, co + 6, R.co);
    R.n_dev = n_start;
    pic_status st = pic_fields_load_lattice_r(ctx, run, n_start - R.prm.order, R.prm.order, table,
                                              M, aE, bE, cE, aB, bB, cB);
    if (st) return st;
    return upload_desc(ctx, run);
}

pic_status pic_advance(pic_ctx *ctx, int32_t S)
{
    CTX_CHECK(ctx);
    pic_status st = check_window(ctx, S);
    if (st) return st;
    if (ctx->np > 0 && (st = predictor_turn(ctx, NO_LEVEL))) return st;
    if (ctx->np > 0 && (st = enqueue_window(ctx, S, ctx->stream))) return st;
    if (ctx->np == 0) {
        // nothing to push, but the device-side levels move on as well
        tick_kernel<<<(ctx->nruns + 255) / 256, 256, 0, ctx->stream>>>(ctx->d_runs, ctx->nruns, S);
        LAUNCH_CHECK(ctx);
    }
    mirror_advance(ctx, S, S);
    return PIC_OK;
}

pic_status pic_run_level(const pic_ctx *ctx, int32_t run, int64_t *n)
{
    if (!ctx || !n || run < 0 || run >= ctx->nruns) return PIC_E_ARG;
    *n = ctx->runs[size_t(run)].n_dev;
    return PIC_OK;
}

pic_status pic_graph_capture(pic_ctx *ctx, int32_t S, int32_t windows)
{
    CTX_CHECK(ctx);
    if (windows < 1) return fail(ctx, PIC_E_ARG, "windows must be >= 1");
    pic_status st = check_window(ctx, S);
    if (st) return st;
    if (ctx->np == 0) return fail(ctx, PIC_E_STATE, "nothing to capture: no particles");
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->gexec = nullptr;
    ctx->graph = nullptr;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    hipStream_t cs = nullptr;       // default priority
    HIP_TRY(ctx, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return fail(ctx, PIC_E_DEVICE, "hipStreamBeginCapture: %s", hipGetErrorString(e));
    }
    for (int32_t w = 0; w < windows && st == PIC_OK; ++w) st = enqueue_window(ctx, S, cs);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(cs, &g);
    (void)hipStreamDestroy(cs);
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(ctx, PIC_E_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(ctx, PIC_E_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    ctx->graph = g;
    ctx->gexec = ge;
    ctx->graph_steps = int64_t(S) * windows;
    ctx->graph_S = S;
    return PIC_OK;
}

pic_status pic_graph_launch(pic_ctx *ctx)
{
    CTX_CHECK(ctx);
    if (!ctx->gexec) return fail(ctx, PIC_E_STATE, "no captured graph");
    HIP_TRY(ctx, hipGraphLaunch(ctx->gexec, ctx->stream));
    mirror_advance(ctx, ctx->graph_steps, ctx->graph_S);
    return PIC_OK;
}

pic_status pic_graph_release(pic_ctx *ctx)
{
    CTX_CHECK(ctx);
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    ctx->gexec = nullptr;
    ctx->graph = nullptr;
    return PIC_OK;
}

pic_status pic_ktrace_set(pic_ctx *ctx, int8_t *buf, int64_t n_first, int32_t steps, int64_t first,
                          int64_t count)
{
    CTX_CHECK(ctx);
    if (buf && (steps <= 0 || count <= 0 || first < 0 || first + count > ctx->np))
        return fail(ctx, PIC_E_ARG, "bad k-trace window");
    ctx->ktrace = buf;
    ctx->kt_n0 = n_first;
    ctx->kt_steps = buf ? steps : 0;
    ctx->kt_first = buf ? first : 0;
    ctx->kt_count = buf ? count : 0;
    return PIC_OK;
}

pic_status pic_push_subcycled(pic_ctx *ctx, int64_t n, int32_t S)
{
    CTX_CHECK(ctx);
    if (!ctx->have_particles) return fail(ctx, PIC_E_STATE, "particles not loaded");
    if (S < 1) return fail(ctx, PIC_E_ARG, "S must be >= 1");
    for (int r = 0; r < ctx->nruns; ++r) {
        const RunHost &R = ctx->runs[size_t(r)];
        const pic_params &p = R.prm;
        if (int64_t(S) + p.order > p.ring_depth)
            return fail(ctx, PIC_E_LEVEL, "S + order = %d exceeds ring_depth %d", S + p.order,
                        p.ring_depth);
        for (int64_t m = n - p.order; m <= n + S - 1; ++m)
            if (R.tags[size_t(mod_floor(m, p.ring_depth))] != m)
                return fail(ctx, PIC_E_LEVEL, "run %d: field level %lld is not in the ring", r,
                            (long long)m);
    }
    if (ctx->np == 0) return PIC_OK;
    const pic_status st = predictor_turn(ctx, n);
    if (st) return st;
    return launch_push(ctx, n, S, ctx->stream);
}

pic_status pic_grid_shift(pic_ctx *ctx, int32_t run, int64_t cells, double *x_origin)
{
    CTX_CHECK(ctx);
    if (run < 0 || run >= ctx->nruns) return fail(ctx, PIC_E_ARG, "bad run %d", run);
    RunHost &R = ctx->runs[size_t(run)];
    if (R.driven) return fail(ctx, PIC_E_STATE, "run %d is in device-driven mode", run);
    if (cells > (int64_t(1) << 40) || cells < -(int64_t(1) << 40))
        return fail(ctx, PIC_E_ARG, "shift out of range");
    R.shift += cells;
    R.prm.x_origin = R.x_origin0 + double(R.shift) * R.prm.dx;
    std::fill(R.tags.begin(), R.tags.end(), NO_LEVEL);
    if (x_origin) *x_origin = R.prm.x_origin;
    return upload_desc(ctx, run);
}

pic_status pic_strict_set(pic_ctx *ctx, int32_t on)
{
    CTX_CHECK(ctx);
    ctx->strict = on != 0;
    return PIC_OK;
}

pic_status pic_counters_reset(pic_ctx *ctx)
{
    CTX_CHECK(ctx);
    HIP_TRY(ctx, hipMemsetAsync(ctx->cnt, 0, cnt_words(ctx) * sizeof(uint64_t), ctx->stream));
    ctx->rebins = 0;
    return PIC_OK;
}

pic_status pic_run_counters(pic_ctx *ctx, int32_t run, pic_counters *cnt)
{
    CTX_CHECK(ctx);
    if (!cnt || run < 0 || run >= ctx->nruns) return fail(ctx, PIC_E_ARG, "bad run or counters");
    return read_counters(ctx, run, cnt);
}

// pic_diag's per-particle outputs for caller indices u_lo .. u_lo + u_n - 1.
pic_status diag_range(pic_ctx *ctx, pic_mem mem, int64_t u_lo, int64_t u_n, double *gamma,
                      double *px, double *py, double *pz, double *x, int8_t *k_last,
                      uint8_t *status)
{
    if (mem != PIC_MEM_HOST && mem != PIC_MEM_DEVICE) return fail(ctx, PIC_E_ARG, "bad pic_mem");
    const size_t n = size_t(u_n);
    const bool any = gamma || px || py || pz || x || k_last || status;
    if (!any || u_n <= 0) return PIC_OK;
    if (!ctx->have_particles) return fail(ctx, PIC_E_STATE, "particles not loaded");
    const int grid = grid_for(ctx->slots, 256, 8192);
    if (mem == PIC_MEM_DEVICE) {
        diag_kernel<<<grid, 256, 0, ctx->stream>>>(ctx->perm, ctx->slots, ctx->x, ctx->px, ctx->py,
                                                   ctx->pz, ctx->kold, ctx->status, u_lo, u_n,
                                                   gamma, px, py, pz, x, k_last, status);
        LAUNCH_CHECK(ctx);
        return PIC_OK;
    }
    double *d = nullptr;
    int8_t *dk = nullptr;
    uint8_t *ds = nullptr;
    pic_status st = dev_alloc(ctx, &d, 5 * n);
    if (st) return st;
    if ((st = dev_alloc(ctx, &dk, n)) || (st = dev_alloc(ctx, &ds, n))) {
        (void)hipFree(d);
        if (dk) (void)hipFree(dk);
        return st;
    }
    diag_kernel<<<grid, 256, 0, ctx->stream>>>(ctx->perm, ctx->slots, ctx->x, ctx->px, ctx->py,
                                               ctx->pz, ctx->kold, ctx->status, u_lo, u_n, d,
                                               d + n, d + 2 * n, d + 3 * n, d + 4 * n, dk, ds);
    hipError_t e = hipGetLastError();
    double *outs[5] = {gamma, px, py, pz, x};
    for (int a = 0; a < 5 && e == hipSuccess; ++a)
        if (outs[a])
            e = hipMemcpyAsync(outs[a], d + a * n, n * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream);
    if (e == hipSuccess && k_last) e = hipMemcpyAsync(k_last, dk, n, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess && status) e = hipMemcpyAsync(status, ds, n, hipMemcpyDeviceToHost, ctx->stream);
    hipError_t e2 = hipStreamSynchronize(ctx->stream);
    (void)hipFree(d);
    (void)hipFree(dk);
    (void)hipFree(ds);
    if (e != hipSuccess || e2 != hipSuccess)
        return fail(ctx, PIC_E_DEVICE, "diag copy: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    return PIC_OK;
}

pic_status pic_diag(pic_ctx *ctx, pic_mem mem, double *gamma, double *px, double *py, double *pz,
                    double *x, int8_t *k_last, uint8_t *status, pic_counters *cnt)
{
    CTX_CHECK(ctx);
    pic_status st = diag_range(ctx, mem, 0, ctx->np, gamma, px, py, pz, x, k_last, status);
    if (st) return st;
    if (cnt) return read_counters(ctx, -1, cnt);
    return PIC_OK;
}

pic_status pic_diag_r(pic_ctx *ctx, int32_t run, pic_mem mem, double *gamma, double *px,
                      double *py, double *pz, double *x, int8_t *k_last, uint8_t *status,
                      pic_counters *cnt)
{
    CTX_CHECK(ctx);
    if (run < 0 || run >= ctx->nruns) return fail(ctx, PIC_E_ARG, "bad run %d", run);
    const RunHost &R = ctx->runs[size_t(run)];
    pic_status st = diag_range(ctx, mem, R.caller_off, R.np, gamma, px, py, pz, x, k_last, status);
    if (st) return st;
    if (cnt) return read_counters(ctx, run, cnt);
    return PIC_OK;
}

pic_status pic_diag_noalloc(pic_ctx *ctx, double *gamma, double *px, double *py, double *pz,
                            double *x, int8_t *k_last, uint8_t *status, pic_counters *cnt)
{
    CTX_CHECK(ctx);
    const int64_t np = ctx->np;
    if (np > PIC_DIAG_NOALLOC_MAX_NP)
        return fail(ctx, PIC_E_ARG, "pic_diag_noalloc: %lld particles exceed its maximum of %d",
                    (long long)np, PIC_DIAG_NOALLOC_MAX_NP);
    unsigned char *base = nullptr;
    if (ctx->device >= 0 && ctx->device < NOALLOC_MAX_DEVICES) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        base = g_scratch_ptr[ctx->device];
        if (!base)
            return fail(ctx, PIC_E_DEVICE, "pic_diag_noalloc: no address of its staging array "
                        "on device %d: %s", ctx->device,
                        hipGetErrorString(g_scratch_err[ctx->device]));
    } else {
        return fail(ctx, PIC_E_DEVICE, "pic_diag_noalloc: device %d out of range", ctx->device);
    }
    const size_t n = size_t(np);
    const bool any = gamma || px || py || pz || x || k_last || status;
    if (any && np > 0 && !ctx->have_particles) return fail(ctx, PIC_E_STATE, "particles not loaded");
    uint64_t *dsum = reinterpret_cast<uint64_t *>(base);
    double *d = reinterpret_cast<double *>(base + NOALLOC_HEAD);
    int8_t *dk = reinterpret_cast<int8_t *>(d + 5 * n);
    uint8_t *ds = reinterpret_cast<uint8_t *>(dk + n);
    if (any && np > 0) {
        diag_kernel<<<grid_for(ctx->slots, 256, 8192), 256, 0, ctx->stream>>>(
            ctx->perm, ctx->slots, ctx->x, ctx->px, ctx->py, ctx->pz, ctx->kold, ctx->status,
            int64_t(0), np, gamma ? d : nullptr, px ? d + n : nullptr, py ? d + 2 * n : nullptr,
            pz ? d + 3 * n : nullptr, x ? d + 4 * n : nullptr, k_last ? dk : nullptr,
            status ? ds : nullptr);
        LAUNCH_CHECK(ctx);
    }
    if (cnt) {
        counter_sum_kernel<<<1, 256, 0, ctx->stream>>>(ctx->cnt, int64_t(ctx->nruns) * NSLOT, dsum);
        LAUNCH_CHECK(ctx);
    }
    uint64_t sum[NCNT] = {0};
    hipError_t e = hipSuccess;
    if (any && np > 0) {
        double *outs[5] = {gamma, px, py, pz, x};
        for (int a = 0; a < 5 && e == hipSuccess; ++a)
            if (outs[a])
                e = hipMemcpyAsync(outs[a], d + a * n, n * sizeof(double), hipMemcpyDeviceToHost,
                                   ctx->stream);
        if (e == hipSuccess && k_last)
            e = hipMemcpyAsync(k_last, dk, n, hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess && status)
            e = hipMemcpyAsync(status, ds, n, hipMemcpyDeviceToHost, ctx->stream);
    }
    if (e == hipSuccess && cnt)
        e = hipMemcpyAsync(sum, dsum, sizeof sum, hipMemcpyDeviceToHost, ctx->stream);
    const hipError_t e2 = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess || e2 != hipSuccess)
        return fail(ctx, PIC_E_DEVICE, "pic_diag_noalloc: %s",
                    hipGetErrorString(e != hipSuccess ? e : e2));
    if (cnt) counters_from_sums(sum, ctx->rebins, cnt);
    return PIC_OK;
}

pic_status pic_predictor_set(pic_ctx *ctx, const uint16_t *w_bf16, const float *norm,
                             const float *run_a0, float width, int32_t every_M)
{
    CTX_CHECK(ctx);
    if (!w_bf16) {                 // detach
        ctx->pred_every = 0;
        return PIC_OK;
    }
    if (!norm || !run_a0) return fail(ctx, PIC_E_ARG, "null normalisation or a0 array");
    if (every_M < 1) return fail(ctx, PIC_E_ARG, "every_M must be >= 1");
    if (!(width > 0.0f)) return fail(ctx, PIC_E_ARG, "width must be > 0");
    for (int r = 0; r < ctx->nruns; ++r)
        if (!(run_a0[r] > 0.0f)) return fail(ctx, PIC_E_ARG, "run %d: a0 must be > 0", r);
    const size_t np = size_t(std::max<int64_t>(ctx->np, 1));
    pic_status st;
    if (!ctx->pred_w &&
        ((st = dev_alloc(ctx, &ctx->pred_w, size_t(PIC_MLP_NPARAM))) ||
         (st = dev_alloc(ctx, &ctx->pred_norm, size_t(2 * PIC_MLP_FEATURES))) ||
         (st = dev_alloc(ctx, &ctx->pred_feat, np * PIC_MLP_FEATURES)) ||
         (st = dev_alloc(ctx, &ctx->pred_score, np)))) {
        void *ps[] = {ctx->pred_w, ctx->pred_norm, ctx->pred_feat, ctx->pred_score};
        for (void *q : ps)
            if (q) (void)hipFree(q);
        ctx->pred_w = nullptr;
        ctx->pred_norm = ctx->pred_feat = ctx->pred_score = nullptr;
        return st;
    }
    HIP_TRY(ctx, hipMemcpyAsync(ctx->pred_w, w_bf16, PIC_MLP_NPARAM * sizeof(uint16_t),
                                hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->pred_norm, norm, 2 * PIC_MLP_FEATURES * sizeof(float),
                                hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    ctx->pred_a0.assign(run_a0, run_a0 + ctx->nruns);
    ctx->pred_width = width;
    ctx->pred_every = every_M;
    ctx->pred_calls = 0;
    return PIC_OK;
}

pic_status pic_diag_track(pic_ctx *ctx, int32_t on)
{
    CTX_CHECK(ctx);
    if (on != 0 && on != 1) return fail(ctx, PIC_E_ARG, "on must be 0 or 1");
    if (!on) {
        ctx->deph = false;
        return PIC_OK;
    }
    const size_t n = size_t(ctx->slots);
    if (!ctx->r0) {
        pic_status st;
        if ((st = dev_alloc(ctx, &ctx->r0, n)) || (st = dev_alloc(ctx, &ctx->rmax, n)) ||
            (st = dev_alloc(ctx, &ctx->work, n)) || (st = dev_alloc(ctx, &ctx->werr, n)) ||
            (st = dev_alloc(ctx, &ctx->gmax, n))) {
            double *ps[5] = {ctx->r0, ctx->rmax, ctx->work, ctx->werr, ctx->gmax};
            for (double *q : ps)
                if (q) (void)hipFree(q);
            ctx->r0 = ctx->rmax = ctx->work = ctx->werr = ctx->gmax = nullptr;
            return st;
        }
    }
    diag_init_kernel<<<grid_for(ctx->slots, 256, 8192), 256, 0, ctx->stream>>>(
        ctx->slots, ctx->px, ctx->py, ctx->pz, ctx->r0, ctx->rmax, ctx->work, ctx->werr,
        ctx->gmax);
    LAUNCH_CHECK(ctx);
    ctx->deph = true;
    ctx->gerr = false;
    return PIC_OK;
}

namespace {
// Two diagnostic arrays out in caller order.
pic_status diag_out(pic_ctx *ctx, pic_mem mem, const double *a, const double *b, double *oa,
                    double *ob)
{
    CTX_CHECK(ctx);
    if (mem != PIC_MEM_HOST && mem != PIC_MEM_DEVICE) return fail(ctx, PIC_E_ARG, "bad pic_mem");
    if (!ctx->r0) return fail(ctx, PIC_E_STATE, "the diagnostics were never switched on");
    const size_t n = size_t(ctx->np);
    if ((oa && !a) || (ob && !b)) return fail(ctx, PIC_E_ARG, "no such diagnostic");
    if (n == 0 || (!oa && !ob)) return PIC_OK;
    const int grid = grid_for(ctx->slots, 256, 8192);
    if (mem == PIC_MEM_DEVICE) {
        slots_to_caller_kernel<<<grid, 256, 0, ctx->stream>>>(ctx->perm, ctx->slots, a, b, oa, ob);
        LAUNCH_CHECK(ctx);
        return PIC_OK;
    }
    double *d = nullptr;
    pic_status st = dev_alloc(ctx, &d, 2 * n);
    if (st) return st;
    // an output slot only for each array the caller asked for (b may be
    // null when ob is)
    slots_to_caller_kernel<<<grid, 256, 0, ctx->stream>>>(ctx->perm, ctx->slots, a, b,
                                                          oa ? d : nullptr, ob ? d + n : nullptr);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && oa) e = hipMemcpyAsync(oa, d, n * 8, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess && ob)
        e = hipMemcpyAsync(ob, d + n, n * 8, hipMemcpyDeviceToHost, ctx->stream);
    const hipError_t e2 = hipStreamSynchronize(ctx->stream);
    (void)hipFree(d);
    if (e != hipSuccess || e2 != hipSuccess)
        return fail(ctx, PIC_E_DEVICE, "diagnostics read: %s",
                    hipGetErrorString(e != hipSuccess ? e : e2));
    return PIC_OK;
}
}  // namespace

pic_status pic_dephasing_read(pic_ctx *ctx, pic_mem mem, double *R0, double *rmax)
{
    if (!ctx) return PIC_E_ARG;
    return diag_out(ctx, mem, ctx->r0, ctx->rmax, R0, rmax);
}

pic_status pic_energy_read(pic_ctx *ctx, pic_mem mem, double *work, double *err_max)
{
    if (!ctx) return PIC_E_ARG;
    return diag_out(ctx, mem, ctx->work, ctx->werr, work, err_max);
}

pic_status pic_ktrace_load(const int8_t *ktrace, int32_t steps, int64_t count, float *score,
                           void *hip_stream)
{
    if (!ktrace || !score || steps < 1 || count < 1) return PIC_E_ARG;
    ktrace_load_kernel<<<grid_for(count, 256, 8192), 256, 0, (hipStream_t)hip_stream>>>(
        ktrace, steps, count, score);
    return hipGetLastError() == hipSuccess ? PIC_OK : PIC_E_DEVICE;
}

pic_status pic_fma_probe(double *out, int32_t blocks, int64_t iters, void *hip_stream)
{
    if (!out || blocks < 1 || iters < 1) return PIC_E_ARG;
    fma_probe_kernel<<<blocks, 256, 0, (hipStream_t)hip_stream>>>(out, iters, 1.0 - 0x1p-30,
                                                                  0x1p-30);
    return hipGetLastError() == hipSuccess ? PIC_OK : PIC_E_DEVICE;
}

pic_status pic_gamma_max_read(pic_ctx *ctx, pic_mem mem, double *gmax)
{
    if (!ctx) return PIC_E_ARG;
    return diag_out(ctx, mem, ctx->gmax, nullptr, gmax, nullptr);
}

pic_status pic_gamma_error_lattice(pic_ctx *ctx, int32_t run, const double *atab, int64_t M,
                                   int64_t A, int64_t B, int64_t C)
{
    CTX_CHECK(ctx);
    if (run < 0 || run >= ctx->nruns) return fail(ctx, PIC_E_ARG, "bad run %d", run);
    RunHost &R = ctx->runs[size_t(run)];
    if (!atab) {
        R.atab = nullptr;
        std::fill(R.at, R.at + 4, int64_t(0));
        return upload_desc(ctx, run);
    }
    if (M <= 0) return fail(ctx, PIC_E_ARG, "bad potential lattice size");
    if (pic_status fs = check_finite(ctx, PIC_MEM_DEVICE, atab, M, "the potential table")) return fs;
    R.atab = atab;
    const int64_t at[4] = {M, A, B, C};
    std::copy(at, at + 4, R.at);
    return upload_desc(ctx, run);
}

pic_status pic_gamma_error_start(pic_ctx *ctx, pic_mem mem, const double *ai)
{
    CTX_CHECK(ctx);
    if (mem != PIC_MEM_HOST && mem != PIC_MEM_DEVICE) return fail(ctx, PIC_E_ARG, "bad pic_mem");
    if (!ai) return fail(ctx, PIC_E_ARG, "null a_i");
    if (!ctx->have_particles) return fail(ctx, PIC_E_STATE, "no particles loaded");
    if (!ctx->r0 || !ctx->deph)
        return fail(ctx, PIC_E_STATE, "the trajectory diagnostics are off (pic_diag_track)");
    const size_t n = size_t(ctx->np);
    if (pic_status fs = check_finite(ctx, mem, ai, int64_t(n), "a_i")) return fs;
    const size_t slots = size_t(ctx->slots);
    if (!ctx->ai) {
        pic_status st;
        if ((st = dev_alloc(ctx, &ctx->ai, slots)) || (st = dev_alloc(ctx, &ctx->emax, slots))) {
            if (ctx->ai) (void)hipFree(ctx->ai);
            if (ctx->emax) (void)hipFree(ctx->emax);
            ctx->ai = ctx->emax = nullptr;
            return st;
        }
    }
    if (n == 0) {                                  // no particles: nothing to start
        ctx->gerr = true;
        return PIC_OK;
    }
    const double *src = ai;
    double *tmp = nullptr;
    if (mem == PIC_MEM_HOST) {
        if (pic_status st = dev_alloc(ctx, &tmp, n)) return st;
        const hipError_t e = hipMemcpyAsync(tmp, ai, n * 8, hipMemcpyHostToDevice, ctx->stream);
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(ctx->stream);
            (void)hipFree(tmp);
            return fail(ctx, PIC_E_DEVICE, "a_i copy: %s", hipGetErrorString(e));
        }
        src = tmp;
    }
    gerr_init_kernel<<<grid_for(ctx->slots, 256, 8192), 256, 0, ctx->stream>>>(
        ctx->perm, ctx->slots, src, ctx->ai, ctx->emax);
    hipError_t e = hipGetLastError();
    if (tmp) {
        const hipError_t e2 = hipStreamSynchronize(ctx->stream);
        (void)hipFree(tmp);
        if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return fail(ctx, PIC_E_DEVICE, "energy error start: %s", hipGetErrorString(e));
    ctx->gerr = true;
    return PIC_OK;
}

pic_status pic_gamma_error_read(pic_ctx *ctx, pic_mem mem, double *emax)
{
    if (!ctx) return PIC_E_ARG;
    return diag_out(ctx, mem, ctx->gerr ? ctx->emax : nullptr, nullptr, emax, nullptr);
}

pic_status pic_tune_set(pic_ctx *ctx, const pic_tune *t)
{
    CTX_CHECK(ctx);
    if (!t) return fail(ctx, PIC_E_ARG, "null tune");
    if (t->waves_per_group != 1 && t->waves_per_group != 2 && t->waves_per_group != 4)
        return fail(ctx, PIC_E_ARG, "waves_per_group must be 1, 2 or 4");
    if (t->tile != 128 && t->tile != 256 && t->tile != 512)
        return fail(ctx, PIC_E_ARG, "tile must be 128, 256 or 512");
    if (t->binning != PIC_BIN_NONE && t->binning != PIC_BIN_BALLOT)
        return fail(ctx, PIC_E_ARG, "binning must be PIC_BIN_NONE or PIC_BIN_BALLOT");
    if (t->binning == PIC_BIN_BALLOT && ctx->precision != PIC_FP64)
        return fail(ctx, PIC_E_ARG, "the tiled ballot push runs with PIC_FP64 only");
    if (t->sort_sub < 1 || t->sort_sub > 256) return fail(ctx, PIC_E_ARG, "sort_sub must be in [1, 256]");
    if (t->occupancy != 0 && (t->occupancy < 5 || t->occupancy > 7))
        return fail(ctx, PIC_E_ARG, "occupancy must be 0, 5, 6 or 7");
    ctx->tune = *t;
    return PIC_OK;
}

pic_status pic_tune_get(const pic_ctx *ctx, pic_tune *t)
{
    if (!ctx || !t) return PIC_E_ARG;
    *t = ctx->tune;
    return PIC_OK;
}

pic_status pic_order_set(pic_ctx *ctx, const int32_t *order, pic_mem mem)
{
    CTX_CHECK(ctx);
    if (mem != PIC_MEM_HOST && mem != PIC_MEM_DEVICE) return fail(ctx, PIC_E_ARG, "bad pic_mem");
    const size_t bytes = size_t(ctx->ngroups) * sizeof(int32_t);
    if (!order) {
        std::vector<int32_t> id(size_t(ctx->ngroups));
        std::iota(id.begin(), id.end(), 0);
        HIP_TRY(ctx, hipMemcpyAsync(ctx->group_order, id.data(), bytes, hipMemcpyHostToDevice,
                                    ctx->stream));
        HIP_TRY(ctx, hipMemsetAsync(ctx->group_prio, 0, size_t(ctx->ngroups), ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        return PIC_OK;
    }
    if (mem == PIC_MEM_HOST) {
        std::vector<char> seen(size_t(ctx->ngroups), 0);
        for (int32_t g = 0; g < ctx->ngroups; ++g) {
            const int32_t v = order[g];
            if (v < 0 || v >= ctx->ngroups || seen[size_t(v)])
                return fail(ctx, PIC_E_ARG, "order is not a permutation of the groups");
            seen[size_t(v)] = 1;
        }
        HIP_TRY(ctx, hipMemcpyAsync(ctx->group_order, order, bytes, hipMemcpyHostToDevice,
                                    ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    } else {
        HIP_TRY(ctx, hipMemcpyAsync(ctx->group_order, order, bytes, hipMemcpyDeviceToDevice,
                                    ctx->stream));
    }
    return PIC_OK;
}

int32_t pic_group_count(const pic_ctx *ctx)
{
    return ctx ? ctx->ngroups : 0;
}

}  // extern "C"

namespace {
// Winners of pic_autotune, per configuration signature, for the process.
std::mutex tune_cache_mu;
std::map<std::vector<int64_t>, std::pair<pic_tune, double>> tune_cache;

std::vector<int64_t> tune_signature(const pic_ctx *ctx, int32_t steps)
{
    auto bits = [](double v) {
        int64_t b;
        std::memcpy(&b, &v, sizeof b);
        return b;
    };
    std::vector<int64_t> k{ctx->device, ctx->precision, ctx->order, ctx->kmax_all, steps,
                           ctx->nruns, ctx->tune.sort_sub};
    for (const RunHost &R : ctx->runs) {
        k.insert(k.end(), {R.np, R.prm.ncells, R.prm.ring_depth, bits(R.prm.dx), bits(R.prm.dt),
                           bits(R.prm.psi_max), bits(R.prm.qm), R.M, R.co[0], R.co[1], R.co[2],
                           R.co[3], R.co[4], R.co[5]});
    }
    return k;
}
}  // namespace

extern "C" {

pic_status pic_autotune_forget(void)
{
    std::lock_guard<std::mutex> lock(tune_cache_mu);
    tune_cache.clear();
    return PIC_OK;
}

pic_status pic_autotune(pic_ctx *ctx, int32_t steps, int32_t reps, pic_tune *best, double *ms_best)
{
    CTX_CHECK(ctx);
    if (steps < 1 || reps < 1) return fail(ctx, PIC_E_ARG, "steps and reps must be >= 1");
    pic_status st = check_window(ctx, steps);
    if (st) return st;
    if (ctx->gexec) return fail(ctx, PIC_E_STATE, "release the captured graph before tuning");
    if (ctx->np == 0) return fail(ctx, PIC_E_STATE, "nothing to tune: no particles");
    const std::vector<int64_t> sig = tune_signature(ctx, steps);
    {
        std::lock_guard<std::mutex> lock(tune_cache_mu);
        const auto it = tune_cache.find(sig);
        if (it != tune_cache.end()) {          // tuned before: no trials
            ctx->tune = it->second.first;
            if (best) *best = it->second.first;
            if (ms_best) *ms_best = it->second.second;
            return PIC_OK;
        }
    }
    // candidates: wavefront kernels with 1, 2, 4 wavefronts per workgroup;
    // compaction kernel with tiles of 128, 256, 512 (FP64 only)
    std::vector<pic_tune> cand;
    const pic_tune &cur = ctx->tune;
    for (int w : {1, 2, 4}) cand.push_back(pic_tune{w, cur.tile, PIC_BIN_NONE, cur.sort_sub, 0});
    if (ctx->precision == PIC_FP64_FAST && ctx->order <= 3)
        for (int occ : {5, 6, 7}) cand.push_back(pic_tune{1, cur.tile, PIC_BIN_NONE, cur.sort_sub, occ});
    if (ctx->precision == PIC_FP64)
        for (int t : {128, 256, 512})
            cand.push_back(pic_tune{cur.waves_per_group, t, PIC_BIN_BALLOT, cur.sort_sub, 0});
    // snapshot of everything a trial changes
    const size_t n = size_t(ctx->slots);
    double *snap = nullptr;
    int8_t *snapk = nullptr;
    uint8_t *snaps = nullptr;
    RunDesc *snapr = nullptr;
    uint64_t *snapc = nullptr;
    if ((st = dev_alloc(ctx, &snap, 4 * n)) || (st = dev_alloc(ctx, &snapk, n)) ||
        (st = dev_alloc(ctx, &snaps, n)) || (st = dev_alloc(ctx, &snapr, size_t(ctx->nruns))) ||
        (st = dev_alloc(ctx, &snapc, cnt_words(ctx)))) {
        void *ps[] = {snap, snapk, snaps, snapr, snapc};
        for (void *p : ps)
            if (p) (void)hipFree(p);
        return st;
    }
    auto copy_state = [&](bool save) -> hipError_t {
        double *soa[4] = {ctx->x, ctx->px, ctx->py, ctx->pz};
        const hipMemcpyKind d2d = hipMemcpyDeviceToDevice;
        hipError_t e = hipSuccess;
        for (int a = 0; a < 4 && e == hipSuccess; ++a)
            e = save ? hipMemcpyAsync(snap + a * n, soa[a], n * 8, d2d, ctx->stream)
                     : hipMemcpyAsync(soa[a], snap + a * n, n * 8, d2d, ctx->stream);
        if (e == hipSuccess)
            e = save ? hipMemcpyAsync(snapk, ctx->kold, n, d2d, ctx->stream)
                     : hipMemcpyAsync(ctx->kold, snapk, n, d2d, ctx->stream);
        if (e == hipSuccess)
            e = save ? hipMemcpyAsync(snaps, ctx->status, n, d2d, ctx->stream)
                     : hipMemcpyAsync(ctx->status, snaps, n, d2d, ctx->stream);
        const size_t rb = size_t(ctx->nruns) * sizeof(RunDesc);
        if (e == hipSuccess)
            e = save ? hipMemcpyAsync(snapr, ctx->d_runs, rb, d2d, ctx->stream)
                     : hipMemcpyAsync(ctx->d_runs, snapr, rb, d2d, ctx->stream);
        const size_t cb = cnt_words(ctx) * sizeof(uint64_t);
        if (e == hipSuccess)
            e = save ? hipMemcpyAsync(snapc, ctx->cnt, cb, d2d, ctx->stream)
                     : hipMemcpyAsync(ctx->cnt, snapc, cb, d2d, ctx->stream);
        return e;
    };
    // the trials write ring slots of levels n_dev .. n_dev + steps - 1,
    // which the next window fills again before reading
    int8_t *keep_trace = ctx->ktrace;
    ctx->ktrace = nullptr;
    const bool keep_deph = ctx->deph;
    ctx->deph = false;
    const pic_tune keep = ctx->tune;
    pic_tune winner = keep;
    double wbest = 1e300;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = copy_state(true);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    for (size_t c = 0; c < cand.size() && e == hipSuccess && st == PIC_OK; ++c) {
        ctx->tune = cand[c];
        double total = 0;
        for (int r = 0; r < reps && e == hipSuccess && st == PIC_OK; ++r) {
            e = copy_state(false);
            if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
            if (e == hipSuccess) st = enqueue_window(ctx, steps, ctx->stream);
            if (e == hipSuccess && st == PIC_OK) e = hipEventRecord(e1, ctx->stream);
            if (e == hipSuccess && st == PIC_OK) e = hipEventSynchronize(e1);
            float ms = 0;
            if (e == hipSuccess && st == PIC_OK) e = hipEventElapsedTime(&ms, e0, e1);
            total += ms;
        }
        if (e == hipSuccess && st == PIC_OK && total / reps < wbest) {
            wbest = total / reps;
            winner = cand[c];
        }
    }
    if (e == hipSuccess) e = copy_state(false);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    void *ps[] = {snap, snapk, snaps, snapr, snapc};
    for (void *p : ps)
        if (p) (void)hipFree(p);
    ctx->ktrace = keep_trace;
    ctx->deph = keep_deph;
    ctx->tune = keep;
    if (st) return st;
    if (e != hipSuccess) return fail(ctx, PIC_E_DEVICE, "autotune: %s", hipGetErrorString(e));
    ctx->tune = winner;
    if (best) *best = winner;
    if (ms_best) *ms_best = wbest;
    std::lock_guard<std::mutex> lock(tune_cache_mu);
    tune_cache[sig] = {winner, wbest};
    return PIC_OK;
}


// ---------------------------------------------------------------------
// Load predictor
// ---------------------------------------------------------------------
pic_status pic_mlp_forward(const uint16_t *w_bf16, const float *norm, const float *feat,
                           float *out, int64_t n, void *hip_stream)
{
    if (!w_bf16 || !norm || (n > 0 && (!feat || !out)) || n < 0) return PIC_E_ARG;
    if (n == 0) return PIC_OK;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    mlp_forward_kernel<<<grid_for(n, 256, 8192), 256, 0, s>>>(w_bf16, norm, feat, out, n);
    return hipGetLastError() == hipSuccess ? PIC_OK : PIC_E_DEVICE;
}

pic_status pic_mlp_grad(const float *w, const float *norm, const float *feat, const float *target,
                        int64_t n, float inv_total, float *grad, float *loss, void *hip_stream)
{
    if (!w || !norm || !grad || !loss || n < 0 || (n > 0 && (!feat || !target))) return PIC_E_ARG;
    if (n == 0) return PIC_OK;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    mlp_grad_kernel<<<grid_for(n, 64, 2048), 64, 0, s>>>(w, norm, feat, target, n, inv_total, grad,
                                                         loss);
    return hipGetLastError() == hipSuccess ? PIC_OK : PIC_E_DEVICE;
}

pic_status pic_mlp_adam(float *w, float *m, float *v, const float *grad, int32_t n, float lr,
                        float beta1, float beta2, float eps, int32_t t, void *hip_stream)
{
    if (!w || !m || !v || !grad || n < 0 || t < 1) return PIC_E_ARG;
    if (n == 0) return PIC_OK;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const float c1 = 1.f / (1.f - std::pow(beta1, float(t)));
    const float c2 = 1.f / (1.f - std::pow(beta2, float(t)));
    adam_kernel<<<(n + 255) / 256, 256, 0, s>>>(w, m, v, grad, n, lr, beta1, beta2, eps, c1, c2);
    return hipGetLastError() == hipSuccess ? PIC_OK : PIC_E_DEVICE;
}

pic_status pic_features(pic_ctx *ctx, int64_t n, const float *run_a0, float *feat)
{
    CTX_CHECK(ctx);
    if (!run_a0 || (!feat && ctx->np > 0)) return fail(ctx, PIC_E_ARG, "null features or a0");
    if (!ctx->have_particles) return fail(ctx, PIC_E_STATE, "particles not loaded");
    for (int r = 0; r < ctx->nruns; ++r) {
        const RunHost &R = ctx->runs[size_t(r)];
        const int64_t lev = n != NO_LEVEL ? n : R.n_dev;
        for (int64_t m = lev - 2; m <= lev - 1; ++m)
            if (R.tags[size_t(mod_floor(m, R.prm.ring_depth))] != m)
                return fail(ctx, PIC_E_LEVEL, "run %d: level %lld is not in the ring", r,
                            (long long)m);
        if (!(run_a0[r] > 0)) return fail(ctx, PIC_E_ARG, "run %d: a0 must be > 0", r);
    }
    if (ctx->np == 0) return PIC_OK;
    float *da0 = nullptr;
    pic_status st = dev_alloc(ctx, &da0, size_t(ctx->nruns));
    if (st) return st;
    hipError_t e = hipMemcpyAsync(da0, run_a0, size_t(ctx->nruns) * 4, hipMemcpyHostToDevice,
                                  ctx->stream);
    if (e == hipSuccess) {
        FeatArgs f{ctx->d_runs, ctx->group_run, ctx->x, ctx->px, ctx->py, ctx->pz, ctx->status,
                   ctx->perm, da0, feat, n, ctx->slots};
        features_kernel<<<grid_for(ctx->slots, 256, 8192), 256, 0, ctx->stream>>>(f);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    (void)hipFree(da0);
    if (e != hipSuccess) return fail(ctx, PIC_E_DEVICE, "features: %s", hipGetErrorString(e));
    return PIC_OK;
}

pic_status pic_prebin(pic_ctx *ctx, const float *score, int32_t nbuckets, float width,
                      int32_t prio_groups)
{
    CTX_CHECK(ctx);
    if (!ctx->have_particles) return fail(ctx, PIC_E_STATE, "particles not loaded");
    if (!score && ctx->np > 0) return fail(ctx, PIC_E_ARG, "null score");
    if (nbuckets < 1 || nbuckets > 64 || !(width > 0) || prio_groups < 0)
        return fail(ctx, PIC_E_ARG, "need 1..64 buckets, width > 0, prio_groups >= 0");
    // a captured graph may stay: the particle arrays, the group order and
    // the priorities are rewritten in place (the launches it recorded hold
    // the same pointers), so its next replay runs in the new order
    if (ctx->np == 0) return PIC_OK;
    const int64_t slots = ctx->slots;
    const size_t n = size_t(slots);
    const int psub = ctx->tune.sort_sub;   // position bins per cell inside a bucket, as at load
    // key space: run-major, then bucket, then position
    std::vector<int64_t> bin_off(size_t(ctx->nruns)), shift(size_t(ctx->nruns));
    int64_t nb = 0;
    for (int r = 0; r < ctx->nruns; ++r) {
        const RunHost &R = ctx->runs[size_t(r)];
        bin_off[size_t(r)] = nb;
        shift[size_t(r)] = R.p_off - R.caller_off;
        nb += int64_t(nbuckets) * (int64_t(R.prm.ncells) * psub + 1);
    }
    if (nb >= INT32_MAX) return fail(ctx, PIC_E_ARG, "too many re-binning bins");
    const int64_t nchunks = (nb + SCAN_CHUNK - 1) / SCAN_CHUNK;
    const bool resort = nbuckets > 1;      // one bucket: the load-time order stays
    int32_t *key = nullptr, *hist = nullptr, *sums = nullptr, *dest = nullptr, *nperm = nullptr;
    int64_t *dbin = nullptr, *dshift = nullptr;
    double *nsoa = nullptr;
    int8_t *nk = nullptr;
    uint8_t *nst = nullptr;
    float *gcost = nullptr, *top = nullptr;
    pic_status st = PIC_OK;
    hipError_t e = hipSuccess;
    std::vector<float> hg;
    std::vector<int32_t> order;
    std::vector<int8_t> prio;
    if ((st = dev_alloc(ctx, &gcost, size_t(ctx->ngroups)))) goto out;
    if (resort &&
        ((st = dev_alloc(ctx, &key, n)) || (st = dev_alloc(ctx, &hist, size_t(nb))) ||
         (st = dev_alloc(ctx, &sums, size_t(nchunks))) || (st = dev_alloc(ctx, &dest, n)) ||
         (st = dev_alloc(ctx, &nperm, n)) || (st = dev_alloc(ctx, &dbin, bin_off.size())) ||
         (st = dev_alloc(ctx, &dshift, shift.size())) || (st = dev_alloc(ctx, &nsoa, 4 * n)) ||
         (st = dev_alloc(ctx, &nk, n)) || (st = dev_alloc(ctx, &nst, n)) ||
         (st = dev_alloc(ctx, &top, size_t(SCORE_MAX_BLOCKS)))))
        goto out;
    if (resort) {
        e = hipMemcpyAsync(dbin, bin_off.data(), bin_off.size() * 8, hipMemcpyHostToDevice,
                           ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(dshift, shift.data(), shift.size() * 8, hipMemcpyHostToDevice,
                               ctx->stream);
        if (e == hipSuccess) e = hipMemsetAsync(hist, 0, size_t(nb) * 4, ctx->stream);
        if (e == hipSuccess) e = hipMemsetAsync(nperm, 0xFF, n * 4, ctx->stream);
        // padding slots keep their contents: start the new arrays as copies
        const double *soa[4] = {ctx->x, ctx->px, ctx->py, ctx->pz};
        for (int a = 0; a < 4 && e == hipSuccess; ++a)
            e = hipMemcpyAsync(nsoa + a * n, soa[a], n * 8, hipMemcpyDeviceToDevice, ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(nk, ctx->kold, n, hipMemcpyDeviceToDevice, ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(nst, ctx->status, n, hipMemcpyDeviceToDevice, ctx->stream);
        if (e == hipSuccess) {
            // top of the score range (max over particles) fixes bucket 0
            score_max_kernel<<<SCORE_MAX_BLOCKS, 256, 0, ctx->stream>>>(score, ctx->np, top);
            score_max_kernel<<<1, 256, 0, ctx->stream>>>(top, SCORE_MAX_BLOCKS, top);
            const int g = grid_for(slots, 256, 8192);
            prebin_key_kernel<<<g, 256, 0, ctx->stream>>>(ctx->d_runs, ctx->group_run, ctx->x,
                                                          ctx->perm, score, dbin, nbuckets, width,
                                                          top, psub, slots, key, hist);
            scan_sums_kernel<<<unsigned(nchunks), 256, 0, ctx->stream>>>(hist, nb, sums);
            scan_top_kernel<<<1, 1024, 0, ctx->stream>>>(sums, int(nchunks));
            scan_chunk_kernel<<<unsigned(nchunks), 256, 0, ctx->stream>>>(hist, nb, sums);
            prebin_scatter_kernel<<<g, 256, 0, ctx->stream>>>(key, ctx->perm, ctx->group_run,
                                                              dshift, slots, hist, dest);
            permute_state_kernel<<<g, 256, 0, ctx->stream>>>(
                dest, slots, ctx->x, ctx->px, ctx->py, ctx->pz, ctx->kold, ctx->status, ctx->perm,
                nsoa, nsoa + n, nsoa + 2 * n, nsoa + 3 * n, nk, nst, nperm);
            e = hipGetLastError();
        }
        double *soa2[4] = {ctx->x, ctx->px, ctx->py, ctx->pz};
        for (int a = 0; a < 4 && e == hipSuccess; ++a)
            e = hipMemcpyAsync(soa2[a], nsoa + a * n, n * 8, hipMemcpyDeviceToDevice, ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ctx->kold, nk, n, hipMemcpyDeviceToDevice, ctx->stream);
        if (e == hipSuccess && ctx->r0) {
            // the diagnostics follow their particles (nsoa is free again;
            // ctx->perm still holds the old slot map)
            double *d4[4] = {ctx->r0, ctx->rmax, ctx->work, ctx->werr};
            for (int a = 0; a < 4 && e == hipSuccess; ++a)
                e = hipMemcpyAsync(nsoa + a * n, d4[a], n * 8, hipMemcpyDeviceToDevice, ctx->stream);
            for (int a = 0; a < 4 && e == hipSuccess; a += 2) {
                permute_pair_kernel<<<grid_for(slots, 256, 8192), 256, 0, ctx->stream>>>(
                    dest, slots, ctx->perm, d4[a], d4[a + 1], nsoa + a * n, nsoa + (a + 1) * n);
                e = hipGetLastError();
            }
            for (int a = 0; a < 4 && e == hipSuccess; ++a)
                e = hipMemcpyAsync(d4[a], nsoa + a * n, n * 8, hipMemcpyDeviceToDevice, ctx->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(nsoa, ctx->gmax, n * 8, hipMemcpyDeviceToDevice, ctx->stream);
            if (e == hipSuccess) {
                permute_one_kernel<<<grid_for(slots, 256, 8192), 256, 0, ctx->stream>>>(
                    dest, slots, ctx->perm, ctx->gmax, nsoa);
                e = hipGetLastError();
            }
            if (e == hipSuccess)
                e = hipMemcpyAsync(ctx->gmax, nsoa, n * 8, hipMemcpyDeviceToDevice, ctx->stream);
            if (e == hipSuccess && ctx->gerr) {
                double *d2[2] = {ctx->ai, ctx->emax};
                for (int a = 0; a < 2 && e == hipSuccess; ++a)
                    e = hipMemcpyAsync(nsoa + a * n, d2[a], n * 8, hipMemcpyDeviceToDevice,
                                       ctx->stream);
                if (e == hipSuccess) {
                    permute_pair_kernel<<<grid_for(slots, 256, 8192), 256, 0, ctx->stream>>>(
                        dest, slots, ctx->perm, nsoa, nsoa + n, ctx->ai, ctx->emax);
                    e = hipGetLastError();
                }
            }
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(ctx->perm, nperm, n * 4, hipMemcpyDeviceToDevice, ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ctx->status, nst, n, hipMemcpyDeviceToDevice, ctx->stream);
    }
    // dispatch order: groups by predicted cost, heaviest first; raised
    // priority for the prio_groups heaviest
    if (e == hipSuccess) {
        group_cost_kernel<<<(ctx->ngroups + 3) / 4, 256, 0, ctx->stream>>>(score, ctx->perm,
                                                                           ctx->ngroups, gcost);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hg.resize(size_t(ctx->ngroups));
        e = hipMemcpyAsync(hg.data(), gcost, hg.size() * 4, hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    }
    if (e == hipSuccess) {
        order.resize(hg.size());
        std::iota(order.begin(), order.end(), 0);
        // heaviest first, in steps of `width`: groups of one cost step keep
        // their slot (position, run) order, so waves that run together still
        // share field data in the caches
        float gtop = -1e30f;
        for (float v : hg) gtop = std::max(gtop, v);
        std::vector<int32_t> gb(hg.size());
        for (size_t g = 0; g < hg.size(); ++g)
            gb[g] = hg[g] > -1e29f ? int32_t(std::min(std::floor((gtop - hg[g]) / width), 1e9f))
                                   : INT32_MAX;
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t a, int32_t b) { return gb[size_t(a)] < gb[size_t(b)]; });
        prio.assign(hg.size(), 0);
        for (int32_t i = 0; i < std::min<int32_t>(prio_groups, ctx->ngroups); ++i)
            if (hg[size_t(order[size_t(i)])] > -1e29f) prio[size_t(order[size_t(i)])] = 1;
        e = hipMemcpyAsync(ctx->group_order, order.data(), order.size() * 4, hipMemcpyHostToDevice,
                           ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ctx->group_prio, prio.data(), prio.size(), hipMemcpyHostToDevice,
                               ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    }
    if (e != hipSuccess) st = fail(ctx, PIC_E_DEVICE, "prebin: %s", hipGetErrorString(e));
out:
    (void)hipStreamSynchronize(ctx->stream);
    void *tmps[] = {key, hist, sums, dest, nperm, dbin, dshift, nsoa, nk, nst, gcost, top};
    for (void *p : tmps)
        if (p) (void)hipFree(p);
    return st;
}


// ---------------------------------------------------------------------
// Checkpoint
// ---------------------------------------------------------------------
namespace {
struct CkptHeader {
    char magic[8];
    uint32_t version;
    int32_t nruns;
    int64_t np;
};
struct CkptRun {
    int64_t np;
    int64_t level;
    int32_t ncells;
    int32_t order;
};
constexpr char CKPT_MAGIC[8] = {'P', 'I', 'C', 'S', 'U', 'B', 'C', 'K'};
constexpr uint32_t CKPT_VERSION = 2;   // 2: pic_counters carries rebins

size_t ckpt_bytes(const pic_ctx *ctx)
{
    const size_t n = size_t(ctx->np);
    return sizeof(CkptHeader) + size_t(ctx->nruns) * (sizeof(CkptRun) + sizeof(pic_counters)) +
           n * (4 * sizeof(double) + 2);
}
}  // namespace

pic_status pic_state_export(pic_ctx *ctx, void *buf, size_t *bytes)
{
    CTX_CHECK(ctx);
    if (!bytes) return fail(ctx, PIC_E_ARG, "null size");
    const size_t need = ckpt_bytes(ctx);
    if (!buf) {
        *bytes = need;
        return PIC_OK;
    }
    if (*bytes < need) return fail(ctx, PIC_E_ARG, "buffer of %zu bytes, need %zu", *bytes, need);
    if (!ctx->have_particles) return fail(ctx, PIC_E_STATE, "particles not loaded");
    const size_t n = size_t(ctx->np);
    std::vector<double> px(n), py(n), pz(n), x(n);
    std::vector<int8_t> k(n);
    std::vector<uint8_t> st(n);
    pic_status s = pic_diag(ctx, PIC_MEM_HOST, nullptr, px.data(), py.data(), pz.data(), x.data(),
                            k.data(), st.data(), nullptr);
    if (s) return s;
    char *o = static_cast<char *>(buf);
    CkptHeader h{};
    std::memcpy(h.magic, CKPT_MAGIC, 8);
    h.version = CKPT_VERSION;
    h.nruns = ctx->nruns;
    h.np = ctx->np;
    std::memcpy(o, &h, sizeof h);
    o += sizeof h;
    for (int r = 0; r < ctx->nruns; ++r) {
        const RunHost &R = ctx->runs[size_t(r)];
        CkptRun cr{R.np, R.n_dev, R.prm.ncells, R.prm.order};
        std::memcpy(o, &cr, sizeof cr);
        o += sizeof cr;
    }
    for (int r = 0; r < ctx->nruns; ++r) {
        pic_counters c;
        if ((s = read_counters(ctx, r, &c))) return s;
        std::memcpy(o, &c, sizeof c);
        o += sizeof c;
    }
    const std::vector<double> *arrs[4] = {&x, &px, &py, &pz};
    for (const auto *a : arrs) {
        std::memcpy(o, a->data(), n * sizeof(double));
        o += n * sizeof(double);
    }
    std::memcpy(o, k.data(), n);
    o += n;
    std::memcpy(o, st.data(), n);
    *bytes = need;
    return PIC_OK;
}

pic_status pic_state_import(pic_ctx *ctx, const void *buf, size_t bytes, int64_t *levels)
{
    CTX_CHECK(ctx);
    if (!buf) return fail(ctx, PIC_E_ARG, "null buffer");
    if (ctx->gexec) return fail(ctx, PIC_E_STATE, "release the captured graph before importing");
    const size_t need = ckpt_bytes(ctx);
    if (bytes < sizeof(CkptHeader)) return fail(ctx, PIC_E_ARG, "truncated checkpoint");
    const char *i = static_cast<const char *>(buf);
    CkptHeader h;
    std::memcpy(&h, i, sizeof h);
    i += sizeof h;
    if (std::memcmp(h.magic, CKPT_MAGIC, 8) != 0 || h.version != CKPT_VERSION)
        return fail(ctx, PIC_E_ARG, "not a checkpoint of this library");
    if (h.nruns != ctx->nruns || h.np != ctx->np || bytes < need)
        return fail(ctx, PIC_E_ARG, "checkpoint of %d runs / %lld particles, context has %d / %lld",
                    h.nruns, (long long)h.np, ctx->nruns, (long long)ctx->np);
    std::vector<int64_t> lev(size_t(ctx->nruns));
    for (int r = 0; r < ctx->nruns; ++r) {
        CkptRun cr;
        std::memcpy(&cr, i, sizeof cr);
        i += sizeof cr;
        const RunHost &R = ctx->runs[size_t(r)];
        if (cr.np != R.np || cr.ncells != R.prm.ncells || cr.order != R.prm.order)
            return fail(ctx, PIC_E_ARG, "run %d does not match the checkpoint", r);
        lev[size_t(r)] = cr.level;
    }
    std::vector<pic_counters> cs(size_t(ctx->nruns));
    for (auto &c : cs) {
        std::memcpy(&c, i, sizeof c);
        i += sizeof c;
    }
    const size_t n = size_t(ctx->np);
    std::vector<double> soa(4 * n);
    std::memcpy(soa.data(), i, 4 * n * sizeof(double));
    i += 4 * n * sizeof(double);
    std::vector<int8_t> k(n);
    std::vector<uint8_t> st(n);
    std::memcpy(k.data(), i, n);
    i += n;
    std::memcpy(st.data(), i, n);
    for (uint8_t v : st)
        if (v != PIC_PARTICLE_LIVE && v != PIC_PARTICLE_LOST)
            return fail(ctx, PIC_E_ARG, "bad status flag in checkpoint");
    pic_status s = load_particles(ctx, PIC_MEM_HOST, soa.data(), soa.data() + n,
                                  soa.data() + 2 * n, soa.data() + 3 * n, k.data(), st.data());
    if (s) return s;
    // counters: each run's totals go to its first slot
    std::vector<uint64_t> w(cnt_words(ctx), 0);
    for (int r = 0; r < ctx->nruns; ++r) {
        uint64_t *v = w.data() + size_t(r) * NSLOT * NCNT;
        for (int kk = 0; kk < PIC_KHIST; ++kk) v[kk] = cs[size_t(r)].steps_by_k[kk];
        v[CNT_CLAMPS] = cs[size_t(r)].clamps;
        v[CNT_LOST] = cs[size_t(r)].lost;
    }
    HIP_TRY(ctx, hipMemcpyAsync(ctx->cnt, w.data(), w.size() * sizeof(uint64_t),
                                hipMemcpyHostToDevice, ctx->stream));
    ctx->rebins = cs.empty() ? 0 : cs[0].rebins;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (levels)
        for (int r = 0; r < ctx->nruns; ++r) levels[r] = lev[size_t(r)];
    return PIC_OK;
}

}  // extern "C"
