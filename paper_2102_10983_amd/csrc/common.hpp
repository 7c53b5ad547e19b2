// common.hpp -- device data layout and helpers shared by the push kernels.
//
// A context is a batch of runs.  Each run has its own grid, time step,
// field ring and particles; its particles occupy a contiguous range of
// slots, padded to RUN_ALIGN so that no 64-slot group (wavefront kernels)
// or tile (compaction kernel) straddles two runs.  Padding slots carry
// perm = -1 and status LOST and are never written back to the caller.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

#include "picsub.h"

namespace picsub {

constexpr int NCNT = PIC_KHIST + 2;   // steps_by_k[16], clamps, lost
constexpr int CNT_CLAMPS = PIC_KHIST;
constexpr int CNT_LOST = PIC_KHIST + 1;
constexpr int NSLOT = 256;            // counter slots per run
constexpr int RUN_ALIGN = 512;        // slot ranges of runs are padded to this
constexpr int WWIN = 64;              // staged nodes per level in a wavefront window
constexpr int64_t NO_LEVEL = INT64_MIN;

// Per-run parameters and state, read by the kernels once per wavefront.
struct RunDesc {
    const double *ringE, *ringB;      // [D][ncells]
    const double *table;              // phase table of the on-device sampler
    double x_origin, dx, dt, qm, psi_max, dtdx;
    int64_t p_off;                    // first slot of the run
    int64_t np;                       // particles of the run (slots p_off .. p_off+np-1)
    int64_t n_cur;                    // current level in device-driven mode
    int64_t n_stop;                   // device-driven mode: no step starts at or past this level
    int64_t M, aE, bE, cE, aB, bB, cB;
    const double *atab;               // potential a on a phase lattice (null: no energy error)
    int64_t atM, atA, atB, atC;       //   entry (atA tau + atB u + atC) mod atM
    int32_t D, ncells, kmax, margin;
};

struct PushArgs {
    const RunDesc *runs;
    const int32_t *group_run;         // run of each 64-slot group
    const int32_t *group_order;       // dispatch position -> group
    const int8_t *group_prio;         // base issue priority of each group (0 or 1)
    double *x, *px, *py, *pz;
    int8_t *kold;
    uint8_t *status;
    const int32_t *perm;              // slot -> caller index (-1: padding)
    const double *wtab;
    int8_t *ktrace;
    const double *r0;                 // trajectory diagnostics (null: off): R = gamma - p_x at
    double *rmax;                     //   the start, running max of |R - R0| / R0,
    double *work, *werr;              //   work of E since the start, largest step energy error,
    double *gmax;                     //   largest gamma after a completed step
    const double *ai;                 // energy error (null: off): a at the start, running
    double *emax;                     //   max of |gamma - gamma_th| / gamma_th
    uint64_t *cnt;                    // [nruns][NSLOT][NCNT]
    int64_t kt_n0, kt_first, kt_count;
    int64_t n0;                       // NO_LEVEL: every run starts at its n_cur
    int32_t kt_steps, S, ngroups;
};

__host__ __device__ inline int64_t mod_floor(int64_t a, int64_t m)
{
    const int64_t r = a % m;
    return r < 0 ? r + m : r;
}

constexpr int64_t wtab_entries(int kmax)
{
    return ((int64_t(1) << (2 * (kmax + 1))) - 1) / 3;   // sum_{k<=kmax} 4^k
}

__host__ __device__ inline int64_t wtab_offset(int k)
{
    return ((int64_t(1) << (2 * k)) - 1) / 3;
}

// Element offsets in the ring of the P+1 levels n-P .. n used at step n.
template <int P>
struct Levels {
    int32_t off[P + 1];
    __device__ __forceinline__ void at(int32_t slot0, int st, int32_t D, int32_t ncells)
    {
#pragma unroll
        for (int j = 0; j <= P; ++j) {
            int s = slot0 + st + j;       // < 2 D since S + P <= D
            s = s >= D ? s - D : s;
            s = s >= D ? s - D : s;
            off[j] = s * ncells;
        }
    }
};

// Temporal interpolation at node i, levels ascending (Eqs. (lagrange1-2),
// (lagrange1-3)): sum_j L_j F_j[i].
template <int P, typename T, typename W>
__device__ __forceinline__ double node_comb(const T *__restrict__ f, const int32_t (&off)[P + 1],
                                            int i, const W &L)
{
    double v = L[0] * f[off[0] + i];
#pragma unroll
    for (int j = 1; j <= P; ++j) v = v + L[j] * f[off[j] + i];
    return v;
}

// Boris momentum update (Sec. III, Eqs. (p)..(gamman)), E along y, B
// along z, IEEE division and square root, equation order.
__device__ __forceinline__ void boris(double qm, double dtp, double E, double B, double &px,
                                      double &py, double &pz)
{
    const double c = 0.5 * qm * dtp;
    const double h = c * E;
    const double mx = px, my = py + h, mz = pz;
    const double g = sqrt(1.0 + ((mx * mx + my * my) + mz * mz));
    const double t = (c * B) / g;
    const double sz = (2.0 * t) / (1.0 + t * t);
    const double ax = mx + my * t;
    const double ay = my - mx * t;
    px = mx + ay * sz;
    py = (my - ax * sz) + h;
    pz = mz;
}

__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e)
{
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// (hi, lo) += d
__device__ __forceinline__ void comp_add(float &hi, float &lo, float d)
{
    const float y = d + lo;
    float s, e;
    two_sum(hi, y, s, e);
    hi = s;
    lo = e;
}

__device__ __forceinline__ void split(double v, float &hi, float &lo)
{
    hi = float(v);
    lo = float(v - double(hi));
}

// Lane masks straight from the compare (no round trip through a vector
// register): the bits of the active lanes where p holds.
__device__ __forceinline__ uint64_t wballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ bool wany(bool p) { return wballot(p) != 0; }
__device__ __forceinline__ bool wall(bool p) { return wballot(!p) == 0; }

__device__ __forceinline__ int wave_min(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ int wave_max(int v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Orders this wavefront's LDS writes before its later LDS reads from other
// lanes (and the reverse); no other wavefront is involved.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Completed steps per k, clamps and lost particles of one lane.
struct Counts {
    uint32_t steps[PIC_K_MAX_LIMIT + 1];
    uint32_t clamps, lost;
    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int k = 0; k <= PIC_K_MAX_LIMIT; ++k) steps[k] = 0;
        clamps = lost = 0;
    }
    __device__ __forceinline__ void step_done(int k)
    {
#pragma unroll
        for (int kk = 0; kk <= PIC_K_MAX_LIMIT; ++kk) steps[kk] += (k == kk);
    }
};

// Counters of a whole wavefront, kept wave-uniform (scalar registers):
// every update is a ballot over the lanes at a point all lanes reach.
struct WaveCounts {
    uint32_t steps[PIC_K_MAX_LIMIT + 1];
    uint32_t clamps, lost;
    __device__ __forceinline__ void zero()
    {
#pragma unroll
        for (int k = 0; k <= PIC_K_MAX_LIMIT; ++k) steps[k] = 0;
        clamps = lost = 0;
    }
    // lanes with `done` completed a step with exponent k
    __device__ __forceinline__ void steps_done(bool done, int k)
    {
        steps[0] += __popcll(wballot(done & (k == 0)));
        if (wany(done & (k > 0))) {
#pragma unroll
            for (int kk = 1; kk <= PIC_K_MAX_LIMIT; ++kk)
                steps[kk] += __popcll(wballot(done & (k == kk)));
        }
    }
    // the same for the lanes with k > 0 only
    __device__ __forceinline__ void steps_heavy(bool done, int k)
    {
#pragma unroll
        for (int kk = 1; kk <= PIC_K_MAX_LIMIT; ++kk)
            steps[kk] += __popcll(wballot(done & (k == kk)));
    }
    __device__ __forceinline__ void flush(uint64_t *__restrict__ slot, int lane) const
    {
        if (lane != 0) return;
#pragma unroll
        for (int k = 0; k <= PIC_K_MAX_LIMIT; ++k)
            if (steps[k]) atomicAdd(reinterpret_cast<unsigned long long *>(slot + k), steps[k]);
        if (clamps) atomicAdd(reinterpret_cast<unsigned long long *>(slot + CNT_CLAMPS), clamps);
        if (lost) atomicAdd(reinterpret_cast<unsigned long long *>(slot + CNT_LOST), lost);
    }
};

// Wavefront reduction, then lane 0 adds into a counter slot.
__device__ __forceinline__ void flush_wave(Counts &c, uint64_t *__restrict__ slot, int lane)
{
#pragma unroll
    for (int k = 0; k <= PIC_K_MAX_LIMIT; ++k) {
        const uint32_t v = wave_sum(c.steps[k]);
        if (lane == 0 && v) atomicAdd(reinterpret_cast<unsigned long long *>(slot + k), v);
    }
    const uint32_t cl = wave_sum(c.clamps), lo = wave_sum(c.lost);
    if (lane == 0 && cl)
        atomicAdd(reinterpret_cast<unsigned long long *>(slot + CNT_CLAMPS), cl);
    if (lane == 0 && lo) atomicAdd(reinterpret_cast<unsigned long long *>(slot + CNT_LOST), lo);
}

// Issue priority of a wavefront: base (0 or 1) from the group's predicted
// load, + 2 inside the sub-step loops of the IEEE and compaction kernels (the
// fast kernel keeps its base priority there: raising it made it slower).
__device__ __forceinline__ void set_prio(int p)
{
    switch (p) {
    case 0: __builtin_amdgcn_s_setprio(0); break;
    case 1: __builtin_amdgcn_s_setprio(1); break;
    case 2: __builtin_amdgcn_s_setprio(2); break;
    default: __builtin_amdgcn_s_setprio(3); break;
    }
}

// A particle whose momentum is not finite is frozen and flagged lost at its
// first step, as one whose x is not finite fails the grid test; its stored
// state is left as it was.
__device__ __forceinline__ bool nonfinite_p(double px, double py, double pz)
{
    return !(__builtin_isfinite(px) & __builtin_isfinite(py) & __builtin_isfinite(pz));
}

// Steps this run takes in a launch of S steps starting at n0.
__device__ __forceinline__ int run_steps(const PushArgs &a, const RunDesc &R, int64_t n0)
{
    if (a.n0 != NO_LEVEL) return a.S;                 // host-driven launch
    const int64_t left = R.n_stop - n0;
    return left <= 0 ? 0 : (left < a.S ? int(left) : a.S);
}

// Dephasing diagnostic (Sec. V, Eq. (R error)): after a completed step,
// R = gamma - p_x of the stored momentum; keep the largest |R - R0| / R0.
// IEEE square root and division, the order of a CPU loop.
__device__ __forceinline__ double gamma_of(double px, double py, double pz)
{
    return sqrt(1.0 + ((px * px + py * py) + pz * pz));
}

// After a completed step: the running maximum of the dephasing error
// |R - R0| / R0, R = gamma - p_x (Eq. (R error)), and of gamma.
__device__ __forceinline__ void dephasing_update(double &rmax, double &gmax, double r0, double px,
                                                 double py, double pz)
{
    const double g = gamma_of(px, py, pz);
    const double d = fabs((g - px) - r0) / r0;
    rmax = d > rmax ? d : rmax;
    gmax = g > gmax ? g : gmax;
}

// After a completed step: the running maximum of the energy error
// |gamma - gamma_th| / gamma_th (Eq. (gamma error)) against the plane-wave
// solution gamma_th = 1 + (a - a_i)^2 / 2 (Eq. (theoretical gamma)) of an
// electron that started at rest where the potential was a_i.  a is taken at
// the phase of the momentum, which lags x by half of the step's last sub-step
// (time tau = n + 1 - dt*/(2 dt) in steps, E-node coordinate u at x - v_x dt*/2)
// and is linear between the points of the run's potential lattice.  The order
// of operations is that of a CPU loop.
__device__ __forceinline__ void gamma_error_update(double &emax, const RunDesc &R, double tau,
                                                   double u, double g, double ai)
{
    const double m = double(R.atA) * tau + double(R.atB) * u + double(R.atC);
    const double mf = floor(m);
    int64_t j0 = int64_t(mf) % R.atM;
    if (j0 < 0) j0 += R.atM;
    const int64_t j1 = j0 + 1 == R.atM ? 0 : j0 + 1;
    const double av = R.atab[j0] + (m - mf) * (R.atab[j1] - R.atab[j0]);
    const double d = av - ai;
    const double gth = 1.0 + 0.5 * (d * d);
    const double e = fabs(g - gth) / gth;
    emax = e > emax ? e : emax;
}

// Energy accounting (App. B): the work of E over a sub-step is
// q dt_p / 2 E . (v_before + v_after), with E along y here (c = q dt_p / 2);
// after a completed step the change of gamma is set against the step's
// work.  The order of operations is that of a CPU loop.
__device__ __forceinline__ double sub_step_work(double c, double E, double vy_before,
                                                double vy_after)
{
    return (c * E) * (vy_before + vy_after);
}

__device__ __forceinline__ void energy_close(double &work, double &werr, double g_start,
                                             double g_end, double step_work)
{
    const double d = fabs((g_end - g_start) - step_work);
    werr = d > werr ? d : werr;
    work += step_work;
}

__device__ __forceinline__ void ktrace_put(const PushArgs &a, int64_t kt_u, int64_t n, int8_t v)
{
    if (kt_u >= 0) {
        const int64_t r = n - a.kt_n0;
        if (r >= 0 && r < a.kt_steps) a.ktrace[r * a.kt_count + kt_u] = v;
    }
}

}  // namespace picsub
