// push_fast.hpp -- FP64 push with refined hardware reciprocal and inverse
// square root (pic_precision PIC_FP64_FAST) and a step-ahead field window.
//
// Same schedule as the IEEE wavefront kernel: one wavefront per 64-slot
// group, all S steps of the launch, no waiting on other wavefronts.  What
// differs is where the fields come from.  Lanes of a group are sorted by
// position and a particle moves less than one cell per step (c dt < dx), so
// while the group stays narrow, the nodes every lane can touch in step n+1
// lie in a window of PF_NW nodes fixed by the cells of step n.  During step
// n each lane loads its share of that window for the levels of step n+1
// (2 (p + 1) rows of PF_NW nodes: two FP64 values per lane for p = 3) into
// registers; at the end of step n they go to the wavefront's LDS.  The
// decision, the k = 0 step and every sub-step then read LDS, and the global
// load latency hides behind a whole step of arithmetic.  A group that has
// spread wider falls back to direct gathers (k = 0) or a synchronously
// staged window of up to WWIN nodes (sub-cycled steps).
//
// Arithmetic: the temporal combination (Eqs. (lagrange1-2), (lagrange1-3)),
// the tent weights and the Boris update (Sec. III) with fused multiply-adds,
// 1/gamma from v_rsq_f64 and the Boris denominator from v_rcp_f64, each
// refined by one Newton step; x is carried in node units.  p_z never
// changes in this geometry (E along y, B along z), so 1 + p_z^2 is a
// constant of each lane.  At orders 1 to 3, when a wavefront sub-cycles, its
// LDS window is rewritten once per step as the coefficients of each node's
// interpolating polynomial in u = s - 1/2 (the same polynomial as the
// Lagrange form), so a sub-step evaluates it by Horner's rule at
// u = (j - 1) / 4^k instead of loading the weights of (k, j); order 5 keeps
// the weights.  Completed sub-cycled steps are counted per
// k in the wavefront's LDS, one distinct k at a time.
#pragma once

#include "common.hpp"

namespace picsub {

constexpr int PF_NW = 16;   // nodes per row of the step-ahead window (lane bits 0..3)

// Field rings live in global memory; saying so lets the loads be global
// (not generic) loads.
typedef const __attribute__((address_space(1))) double *gdptr;

// Lagrange weights of the B levels (nodes s = 1 - p .. 1) at s = 1/2, the
// decision's time (Eq. (lagrange1-3)); exact dyadic values, the same the
// weight table holds for (k = 0, j = 1).
template <int P> struct HalfStepB;
template <> struct HalfStepB<1> {
    __device__ constexpr double operator[](int) const { return 0.5; }
};
template <> struct HalfStepB<2> {
    __device__ constexpr double operator[](int j) const
    {
        return j == 0 ? -1.0 / 8 : j == 1 ? 6.0 / 8 : 3.0 / 8;
    }
};
template <> struct HalfStepB<3> {
    __device__ constexpr double operator[](int j) const
    {
        return j == 0 ? 1.0 / 16 : j == 1 ? -5.0 / 16 : j == 2 ? 15.0 / 16 : 5.0 / 16;
    }
};
template <> struct HalfStepB<5> {
    __device__ constexpr double operator[](int j) const
    {
        return j == 0 ? 7.0 / 256 : j == 1 ? -45.0 / 256 : j == 2 ? 126.0 / 256
             : j == 3 ? -210.0 / 256 : j == 4 ? 315.0 / 256 : 63.0 / 256;
    }
};

template <int P, typename T, typename W>
__device__ __forceinline__ double comb_fma(const T *__restrict__ f, const int32_t (&off)[P + 1],
                                           int i, const W &L)
{
    double v = L[0] * f[off[0] + i];
#pragma unroll
    for (int j = 1; j <= P; ++j) v = fma(L[j], f[off[j] + i], v);
    return v;
}

// 1 / sqrt(a), a >= 1, and 1 / b, b >= 1: the hardware estimates refined
// by Newton steps (each squares the relative error).
#ifndef PICSUB_RSQ_NEWTON
#define PICSUB_RSQ_NEWTON 1
#endif
#ifndef PICSUB_RCP_NEWTON
#define PICSUB_RCP_NEWTON 1
#endif
__device__ __forceinline__ double rsq_1nr(double a)
{
    double y = __builtin_amdgcn_rsq(a);
    const double h = -0.5 * a;
#pragma unroll
    for (int i = 0; i < PICSUB_RSQ_NEWTON; ++i) y = fma(y, fma(h * y, y, 0.5), y);
    return y;
}

__device__ __forceinline__ double rcp_1nr(double b)
{
    double r = __builtin_amdgcn_rcp(b);
#pragma unroll
    for (int i = 0; i < PICSUB_RCP_NEWTON; ++i) r = fma(r, fma(-b, r, 1.0), r);
    return r;
}

__device__ __forceinline__ double tent_fma(double w, double f0, double f1)
{
    return fma(w, f1 - f0, f0);
}

// Boris update with c = q dt_p / 2 (Sec. III): half kick, rotation by
// t = c B / gamma, half kick.  p_z is untouched.
__device__ __forceinline__ void boris_fma(double c, double E, double B, double onepz, double &px,
                                          double &py)
{
    const double h = c * E;
    const double mx = px, my = py + h;
    const double ig = rsq_1nr(fma(mx, mx, fma(my, my, onepz)));
    const double t = (c * B) * ig;
    const double sz = (2.0 * t) * rcp_1nr(fma(t, t, 1.0));
    const double ax = fma(my, t, mx);
    const double ay = fma(-mx, t, my);
    px = fma(ay, sz, mx);
    py = fma(-ax, sz, my) + h;
}

// Sum_j L_j F_j at one node from the LDS window: p points at the node in
// row 0, rows 2j (E) and 2j + 1 (B) are WWIN doubles apart.
template <int P, typename W>
__device__ __forceinline__ double comb_lds(const double *p, int field, const W &L)
{
    double v = L[0] * p[field * WWIN];
#pragma unroll
    for (int j = 1; j <= P; ++j) v = fma(L[j], p[(2 * j + field) * WWIN], v);
    return v;
}

// The temporal interpolant of one node over the levels n - P .. n
// (Eqs. (lagrange1-2), (lagrange1-3)) written in the monomial basis of
// u = s - 1/2 (u = 0 at the time of x_n, u in [0, 1) over a sub-cycled step):
// N(u) = sum_m a_m u^m with a = C F, F the level values, C the inverse of the
// Vandermonde matrix of the level times (E: u = j - P, B: u = j - P + 1/2).
// The entries are exact rationals; C[B][0][.] are the weights at s = 1/2.
template <int P>
__device__ constexpr double mono_c(int field, int m, int j)
{
    if constexpr (P == 1) {
        constexpr double e[2][2] = {{0.0, 1.0}, {-1.0, 1.0}};
        constexpr double b[2][2] = {{0.5, 0.5}, {-1.0, 1.0}};
        return field ? b[m][j] : e[m][j];
    } else if constexpr (P == 2) {
        constexpr double e[3][3] = {{0.0, 0.0, 1.0}, {0.5, -2.0, 1.5}, {0.5, -1.0, 0.5}};
        constexpr double b[3][3] = {{-1.0 / 8, 3.0 / 4, 3.0 / 8}, {0.0, -1.0, 1.0}, {0.5, -1.0, 0.5}};
        return field ? b[m][j] : e[m][j];
    } else if constexpr (P == 3) {
        constexpr double e[4][4] = {{0.0, 0.0, 0.0, 1.0},
                                    {-1.0 / 3, 3.0 / 2, -3.0, 11.0 / 6},
                                    {-1.0 / 2, 2.0, -5.0 / 2, 1.0},
                                    {-1.0 / 6, 1.0 / 2, -1.0 / 2, 1.0 / 6}};
        constexpr double b[4][4] = {{1.0 / 16, -5.0 / 16, 15.0 / 16, 5.0 / 16},
                                    {1.0 / 24, -1.0 / 8, -7.0 / 8, 23.0 / 24},
                                    {-1.0 / 4, 5.0 / 4, -7.0 / 4, 3.0 / 4},
                                    {-1.0 / 6, 1.0 / 2, -1.0 / 2, 1.0 / 6}};
        return field ? b[m][j] : e[m][j];
    } else {
        constexpr double e[6][6] = {{0.0, 0.0, 0.0, 0.0, 0.0, 1.0},
                                    {-1.0 / 5, 5.0 / 4, -10.0 / 3, 5.0, -5.0, 137.0 / 60},
                                    {-5.0 / 12, 61.0 / 24, -13.0 / 2, 107.0 / 12, -77.0 / 12, 15.0 / 8},
                                    {-7.0 / 24, 41.0 / 24, -49.0 / 12, 59.0 / 12, -71.0 / 24, 17.0 / 24},
                                    {-1.0 / 12, 11.0 / 24, -1.0, 13.0 / 12, -7.0 / 12, 1.0 / 8},
                                    {-1.0 / 120, 1.0 / 24, -1.0 / 12, 1.0 / 12, -1.0 / 24, 1.0 / 120}};
        constexpr double b[6][6] = {{7.0 / 256, -45.0 / 256, 63.0 / 128, -105.0 / 128, 315.0 / 256, 63.0 / 256},
                                    {71.0 / 1920, -29.0 / 128, 37.0 / 64, -143.0 / 192, -67.0 / 128, 563.0 / 640},
                                    {-3.0 / 32, 59.0 / 96, -85.0 / 48, 49.0 / 16, -269.0 / 96, 95.0 / 96},
                                    {-7.0 / 48, 43.0 / 48, -55.0 / 24, 71.0 / 24, -91.0 / 48, 23.0 / 48},
                                    {-1.0 / 16, 17.0 / 48, -19.0 / 24, 7.0 / 8, -23.0 / 48, 5.0 / 48},
                                    {-1.0 / 120, 1.0 / 24, -1.0 / 12, 1.0 / 12, -1.0 / 24, 1.0 / 120}};
        return field ? b[m][j] : e[m][j];
    }
}

// a_m = sum_j C[m][j] F_j, j ascending, leaving out the zero entries of C
// (E's a_0 is the newest level itself): the entries are compile-time
// constants once the loops are unrolled, so the tests fold away.  Dropping a
// zero term changes no value (only, at most, the sign of an exact zero).
template <int P, int FIELD>
__device__ __forceinline__ double mono_row(const double (&F)[P + 1], int m)
{
    double v = 0.0;
    bool first = true;
#pragma unroll
    for (int j = 0; j <= P; ++j) {
        const double c = mono_c<P>(FIELD, m, j);
        if (c != 0.0) {
            v = first ? c * F[j] : fma(c, F[j], v);
            first = false;
        }
    }
    return v;
}

// Replace the level rows of the LDS window (row 2j: E of level j, 2j + 1: B,
// nodes 0 .. nn - 1) by the monomial coefficients (row 2m: a_m of E, 2m + 1:
// of B), one node per lane, both fields (the field is then known at compile
// time, so every entry of C is a constant operand rather than a per-lane
// selection the compiler may keep in registers across the step loop).
template <int P, int FIELD>
__device__ __forceinline__ void column_to_monomial(double *col)
{
    double F[P + 1];
#pragma unroll
    for (int j = 0; j <= P; ++j) F[j] = col[2 * j * WWIN];
#pragma unroll
    for (int m = 0; m <= P; ++m) col[2 * m * WWIN] = mono_row<P, FIELD>(F, m);
}

template <int P>
__device__ __forceinline__ void window_to_monomial(double *sw, int nn, int lane)
{
    for (int c = lane; c < nn; c += 64) {
        column_to_monomial<P, 0>(sw + c);
        column_to_monomial<P, 1>(sw + WWIN + c);
    }
}

// The same for a node read straight from the ring (a group too wide for a
// window): the coefficients are formed with the operations of
// window_to_monomial, so the value does not depend on which path the
// particle's group takes.
template <int P>
__device__ __forceinline__ double horner_ring(gdptr ring, const int32_t (&off)[P + 1], int i,
                                              int field, double u)
{
    double F[P + 1];
#pragma unroll
    for (int j = 0; j <= P; ++j) F[j] = ring[off[j] + i];
    // each coefficient is formed just before Horner's rule takes it (the
    // same operations; fewer values live at once)
    auto coeff = [&](int m) {
        return field ? mono_row<P, 1>(F, m) : mono_row<P, 0>(F, m);
    };
    double v = coeff(P);
#pragma unroll
    for (int m = P - 1; m >= 0; --m) v = fma(v, u, coeff(m));
    return v;
}

// N(u) of one node from its coefficient column (rows 2m + field).
template <int P>
__device__ __forceinline__ double horner_lds(const double *p, int field, double u)
{
    double v = p[(2 * P + field) * WWIN];
#pragma unroll
    for (int m = P - 1; m >= 0; --m) v = fma(v, u, p[(2 * m + field) * WWIN]);
    return v;
}

// Register budget: the compiler's own allocation (94 VGPRs at order 1, 120 at
// order 3, 124 at order 5) gives 5, 4 and 4 wavefronts per SIMD; OCC > 0 asks
// for OCC wavefronts per SIMD (pic_tune.occupancy), paid for with spills.  KT: the k trace compiled in
// (launches with a trace buffer attached); its per-step bookkeeping costs
// about 5 % of a launch that does not record.
template <int P, int WPG, bool DIAG = false, bool KT = true, int OCC = 0>
__global__ void __launch_bounds__(64 * WPG)
    __attribute__((amdgpu_waves_per_eu(OCC > 0 ? OCC : 1))) push_fast_kernel(PushArgs a)
{
    constexpr int ROWS = 2 * (P + 1);                 // row 2j: E of level j, 2j+1: B
    constexpr int NPF = (ROWS * PF_NW + 63) / 64;     // window values per lane
    // Sub-steps evaluate each node's polynomial by Horner's rule from
    // coefficients formed once per sub-cycled step (orders 1 to 3), or weight the
    // window's levels with the (k, j) entry of the weight table (order 5, where
    // forming 2 (P + 1)^2 products per node costs more than it saves).
    constexpr bool MONO = P <= 3;
    constexpr int STRIDE = 2 * (P + 1);               // weight-table entry
    static_assert(PF_NW == 16, "the step-ahead load maps lane bits 4, 5 to field, level");
    __shared__ double sw_all[WPG][ROWS * WWIN];
    __shared__ uint32_t shist_all[WPG][PIC_K_MAX_LIMIT + 1];   // completed steps per k > 0
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int pos = blockIdx.x * WPG + wv;
    if (pos >= a.ngroups) return;                      // whole wavefront: no barrier below
    double *sw = sw_all[wv];
    uint32_t *shist = shist_all[wv];
    if (lane <= PIC_K_MAX_LIMIT) shist[lane] = 0;
    wave_lds_sync();
    const int g = __builtin_amdgcn_readfirstlane(a.group_order[pos]);
    const int run = __builtin_amdgcn_readfirstlane(a.group_run[g]);
    const int prio = __builtin_amdgcn_readfirstlane(a.group_prio[g]);
    if (prio) set_prio(prio);
    // the run's constants, once, in scalar registers
    const RunDesc &RD = a.runs[run];
    const gdptr ringE = (gdptr)RD.ringE;
    const gdptr ringB = (gdptr)RD.ringB;
    const double x_origin = RD.x_origin, dx = RD.dx, dt = RD.dt, qm = RD.qm;
    const double psi_max = RD.psi_max, dtdx = RD.dtdx;
    const int32_t D = RD.D, ncells = RD.ncells, kmax = RD.kmax, margin = RD.margin;
    const int64_t n0 = a.n0 != NO_LEVEL ? a.n0 : RD.n_cur;
    const int S_run = run_steps(a, RD, n0);
    const int64_t p_off = RD.p_off, np = RD.np;
    const int32_t slot0 = int32_t(mod_floor(n0 - P, D));
    const double ncm1 = double(ncells - 1);
    const double c0 = 0.5 * qm * dt;
    const double q4 = 0.25 * qm * dt;
    const HalfStepB<P> LB1;                            // B weights at s = 1/2
    const int rad = (PF_NW - 2 * margin - 4) / 2;      // cell spread the window allows
    WaveCounts cnt;
    cnt.zero();

    const int64_t s = int64_t(g) * 64 + lane;
    const bool mine = s - p_off < np;
    double x = 0, px = 0, py = 0, pz = 0, onepz = 1, ig = 1;   // x in node units
    int kold = 0;
    // q dt_p / 2 of a k = 0 step: dt_p = (dt*_old + dt) / 2 (Sec. IV), which is
    // dt unless the previous step was sub-cycled
    double c1k0 = c0;
    uint8_t status = PIC_PARTICLE_LOST;
    int64_t kt_u = -1;
    if (mine) {
        x = (a.x[s] - x_origin) / dx;
        px = a.px[s];
        py = a.py[s];
        pz = a.pz[s];
        onepz = fma(pz, pz, 1.0);
        ig = rsq_1nr(fma(px, px, fma(py, py, onepz)));
        kold = a.kold[s];
        if (kold > 0) c1k0 = q4 * (ldexp(1.0, -2 * kold) + 1.0);
        status = a.status[s];
        if (nonfinite_p(px, py, pz)) x = __builtin_nan("");
        if (KT && a.ktrace) {
            const int64_t u = a.perm[s] - a.kt_first;
            if (u >= 0 && u < a.kt_count) kt_u = u;
        }
    }
    bool moved = false;
    const bool tracing = KT && a.ktrace != nullptr;
    constexpr bool deph = DIAG;   // trajectory diagnostics compiled in
    double r0v = 1.0, rmx = 0.0, wacc = 0.0, wem = 0.0, gmx = 1.0;
    if (deph && mine) {
        r0v = a.r0[s];
        rmx = a.rmax[s];
        gmx = a.gmax[s];
        wacc = a.work[s];
        wem = a.werr[s];
    }
    const bool gerr = deph && a.emax != nullptr && RD.atab != nullptr;   // energy error
    double aiv = 0.0, emx = 0.0;
    if (gerr && mine) {
        aiv = a.ai[s];
        emx = a.emax[s];
    }
    // launch steps whose k is recorded: [kt_lo, kt_hi)
    int kt_lo = 0, kt_hi = 0;
    if (tracing) {
        const int64_t lo = a.kt_n0 - n0, hi = lo + a.kt_steps;
        kt_lo = int(lo < 0 ? 0 : (lo > S_run ? S_run : lo));
        kt_hi = int(hi < 0 ? 0 : (hi > S_run ? S_run : hi));
    }
    bool win = false;        // LDS holds this step's levels on nodes [wlo, wlo + PF_NW)
    int wlo = 0;
    // this lane's share of the window: field (lane bit 4), level pair (bit
    // 5), node (bits 0..3); where it goes in LDS
    const gdptr pf_src = (lane & 16) ? ringB : ringE;
    const int pf_q = lane & (PF_NW - 1);
    const bool pf_hi = (lane & 32) != 0;          // odd level of each pair
    double *const pf_dst = sw + (lane >> 4) * WWIN + pf_q;

    // ring offsets of levels n - P .. n + 1 (scalar registers), moved on by
    // one slot per step
    int32_t lvo[P + 2];
#pragma unroll
    for (int j = 0; j <= P + 1; ++j) lvo[j] = int32_t(mod_floor(slot0 + j, D)) * ncells;
    const int32_t ring_end = D * ncells;

    for (int st = 0; st < S_run; ++st) {
        const int64_t n = n0 + st;
        Levels<P> lv;
#pragma unroll
        for (int j = 0; j <= P; ++j) lv.off[j] = lvo[j];
        // masks of compares, combined on the scalar unit
        const uint64_t amask = wballot(status == PIC_PARTICLE_LIVE);
        const uint64_t lmask = amask & wballot(x >= 0.5) & wballot(x < ncm1);
        const bool live = (status == PIC_PARTICLE_LIVE) & (x >= 0.5) & (x < ncm1);
        if (amask != lmask) {                      // some lane left the grid
            cnt.lost += __popcll(amask & ~lmask);
            if ((status == PIC_PARTICLE_LIVE) & !live) status = PIC_PARTICLE_LOST;
        }
        // k trace: the row of this step, if it is recorded (wave-uniform)
        const bool trace_now = KT && st >= kt_lo && st < kt_hi;
        const int64_t kt_row = n - a.kt_n0;
        if (trace_now) {
            if (!live && kt_u >= 0) a.ktrace[kt_row * a.kt_count + kt_u] = -1;
        }
        // A wavefront with no live lane left runs on to the end: the rest
        // of each step then changes nothing but the (clamped, in-bounds)
        // step-ahead window.  An early exit costs more: the compiler's phi
        // copies and lane reads for it run on every step (4-10 % of the
        // launch).
        const double fl = floor(x);
        const int cell = int(fl);
        // reference cell: the first live lane's
        const int cref =
            __builtin_amdgcn_readlane(cell, (__ffsll((unsigned long long)lmask) - 1) & 63);

        // Step-ahead loads: the levels of step n+1 on the nodes any lane can
        // reach from this step's cells (all within rad of cref).
        const bool pf_next = st + 1 < S_run && rad >= 0 && ncells >= PF_NW &&
                             (lmask & ~(wballot(cell >= cref - rad) & wballot(cell <= cref + rad))) == 0;
        // first node of the window, kept inside the grid on the scalar unit
        // (near an end the window may then miss a lane, which the coverage
        // check of the next step sends to direct gathers of the same values)
        const int nlo = min(max(cref - rad - margin - 1, 0), ncells - PF_NW);
        double pf[NPF];
        if (pf_next) {
#pragma unroll
            for (int h = 0; h < NPF; ++h) {
                // value e = lane + 64 h: row e / 16 (level e / 32, field
                // (e / 16) & 1), node nlo + e % 16
                if (lane + 64 * h < ROWS * PF_NW) {
                    const int node = nlo + pf_q;
                    // (an odd number of levels, p = 2, leaves the last pair
                    // half empty: those lanes have no value to load)
                    const int32_t o_even = lvo[2 * h + 1];
                    const int32_t o_odd = 2 * h + 2 <= P + 1 ? lvo[2 * h + 2] : o_even;
                    const int32_t off = pf_hi ? o_odd : o_even;
                    pf[h] = pf_src[off + node];
                }
            }
        }

        // Does the window loaded during the previous step cover every lane?
        const bool use_win =
            win && (lmask & ~(wballot(cell - margin >= wlo) &
                             wballot(cell + margin + 1 < wlo + PF_NW))) == 0;

        // decision: B at (x_n, s = 1/2), 1/gamma of the stored momentum
        int k = 0;
        double Bd = 0.0, psi0 = 0.0;
        bool clamped = false;
        if (live) {
            double b0, b1;
            if (use_win) {
                const double *p = sw + (cell - wlo);
                b0 = comb_lds<P>(p, 1, LB1);
                b1 = comb_lds<P>(p + 1, 1, LB1);
            } else {
                b0 = comb_fma<P>(ringB, lv.off, cell, LB1);
                b1 = comb_fma<P>(ringB, lv.off, cell + 1, LB1);
            }
            Bd = tent_fma(x - fl, b0, b1);
            psi0 = fabs(c0 * Bd) * ig;
        }
        // lanes over the threshold: with kmax > 0 exactly the sub-cycled ones
        const uint64_t omask = lmask & wballot(psi0 > psi_max);
        const uint64_t hmask = kmax > 0 ? omask : 0;
        if (omask) {
            if (live) {
                double lim = psi_max;
                while (psi0 > lim && k < kmax) {
                    ++k;
                    lim = lim * 4.0;
                }
                clamped = psi0 > lim;
            }
            cnt.clamps += __popcll(wballot(clamped));
        }
        if (trace_now) {
            if (live && kt_u >= 0) a.ktrace[kt_row * a.kt_count + kt_u] = int8_t(k);
        }
        const bool heavy = live && k > 0;

        // E of level n at x_n (s = 1/2 is the time of level n: E's weights are
        // (0, .., 0, 1)), for a k = 0 step and for the first sub-step of a
        // sub-cycled one; read before the window is converted
        double Ek = 0.0;
        if (live) {
            const double uE = x - 0.5;
            const double flE = floor(uE);
            const int iE = int(flE);
            // the tent is taken inside each branch, so the window path does
            // not wait for the rare branch's loads (nor for the step-ahead
            // loads in flight) where the branches meet
            if (use_win) {
                const double *p = sw + (2 * P) * WWIN + (iE - wlo);
                Ek = tent_fma(uE - flE, p[0], p[1]);
            } else {
                Ek = tent_fma(uE - flE, ringE[lv.off[P] + iE], ringE[lv.off[P] + iE + 1]);
            }
        }

        // A sub-cycled step outside the step-ahead window stages its own.
        bool lds = use_win;
        int base = wlo;
        int nwin = PF_NW;
        if (!use_win && wany(heavy)) {
            const int lo = max(__builtin_amdgcn_readfirstlane(
                                   wave_min(heavy ? cell - margin : INT_MAX)), 0);
            const int hi = min(__builtin_amdgcn_readfirstlane(
                                   wave_max(heavy ? cell + margin : INT_MIN)), ncells - 1);
            if (hi - lo + 1 <= WWIN) {
                wave_lds_sync();
                for (int q = lane; q <= hi - lo; q += 64) {
#pragma unroll
                    for (int j = 0; j <= P; ++j) {
                        sw[(2 * j) * WWIN + q] = ringE[lv.off[j] + lo + q];
                        sw[(2 * j + 1) * WWIN + q] = ringB[lv.off[j] + lo + q];
                    }
                }
                wave_lds_sync();
                base = lo;
                nwin = hi - lo + 1;
                lds = true;
            }
        }
        // sub-steps read the window's nodes as polynomials in u
        if (MONO && lds && hmask) {
            wave_lds_sync();
            window_to_monomial<P>(sw, nwin, lane);
            wave_lds_sync();
        }

        bool done = false;
        double gst = 1.0, swork = 0.0;     // diagnostics: gamma at the step start, step work
        if (live) {
            moved = true;
            const int kprev = kold;
            kold = k;
            if (deph) gst = gamma_of(px, py, pz);
            if (k == 0) {
                const double c1 = c1k0;
                c1k0 = c0;
                const double vb = deph ? py * ig : 0.0;
                boris_fma(c1, Ek, Bd, onepz, px, py);
                ig = rsq_1nr(fma(px, px, fma(py, py, onepz)));
                x = fma(dtdx, px * ig, x);
                if (deph) swork = sub_step_work(c1, Ek, vb, py * ig);
                done = true;
            } else {
                // dt*_new / dt and dt*_old / dt (cold start: p lags x by half
                // of this step's sub-step)
                const double fnew = ldexp(1.0, -2 * k);
                const double fold = kprev < 0 ? fnew : ldexp(1.0, -2 * kprev);
                const double c1 = q4 * (fold + fnew);          // transition push
                c1k0 = q4 * (fnew + 1.0);                      // for a k = 0 step next
                const double rdx = dtdx * fnew;
                const double dt_new = dt * fnew;
                const int nsub = 1 << (2 * k);
                const double cn = 0.5 * qm * dt_new;
                double u = 0.0;                                // s - 1/2 of sub-step j
                const double *Wk = MONO ? nullptr : a.wtab + wtab_offset(k) * STRIDE;
                done = true;
                for (int j = 1; j <= nsub; ++j, u += fnew) {
                    // sub-step 1 is at x_n and s = 1/2: its fields are the
                    // decision's B and level n's E (the same operations on the
                    // same values as the interpolant's evaluation at u = 0)
                    if (j == 1) {
                        const double vb = deph ? py * ig : 0.0;
                        boris_fma(c1, Ek, Bd, onepz, px, py);
                        ig = rsq_1nr(fma(px, px, fma(py, py, onepz)));
                        x = fma(rdx, px * ig, x);
                        if (deph) swork += sub_step_work(c1, Ek, vb, py * ig);
                        continue;
                    }
                    if (!(x >= 0.5 && x < ncm1)) {
                        done = false;
                        break;
                    }
                    const double fb = floor(x);
                    const int ib = int(fb);
                    const double uE = x - 0.5;
                    const double fe = floor(uE);
                    const int ie = int(fe);
                    double bb0, bb1, e0, e1;
                    if constexpr (MONO) {
                        if (lds) {
                            const double *pb = sw + (ib - base);
                            const double *pe = sw + (ie - base);
                            bb0 = horner_lds<P>(pb, 1, u);
                            bb1 = horner_lds<P>(pb + 1, 1, u);
                            e0 = horner_lds<P>(pe, 0, u);
                            e1 = horner_lds<P>(pe + 1, 0, u);
                        } else {
                            bb0 = horner_ring<P>(ringB, lv.off, ib, 1, u);
                            bb1 = horner_ring<P>(ringB, lv.off, ib + 1, 1, u);
                            e0 = horner_ring<P>(ringE, lv.off, ie, 0, u);
                            e1 = horner_ring<P>(ringE, lv.off, ie + 1, 0, u);
                        }
                    } else {
                        const double *W = Wk + (j - 1) * STRIDE;   // weights of (k, j)
                        if (lds) {
                            const double *pb = sw + (ib - base);
                            const double *pe = sw + (ie - base);
                            bb0 = comb_lds<P>(pb, 1, W + P + 1);
                            bb1 = comb_lds<P>(pb + 1, 1, W + P + 1);
                            e0 = comb_lds<P>(pe, 0, W);
                            e1 = comb_lds<P>(pe + 1, 0, W);
                        } else {
                            bb0 = comb_fma<P>(ringB, lv.off, ib, W + P + 1);
                            bb1 = comb_fma<P>(ringB, lv.off, ib + 1, W + P + 1);
                            e0 = comb_fma<P>(ringE, lv.off, ie, W);
                            e1 = comb_fma<P>(ringE, lv.off, ie + 1, W);
                        }
                    }
                    const double Es = tent_fma(uE - fe, e0, e1);
                    const double vb = deph ? py * ig : 0.0;
                    boris_fma(cn, Es, tent_fma(x - fb, bb0, bb1), onepz, px, py);
                    ig = rsq_1nr(fma(px, px, fma(py, py, onepz)));
                    x = fma(rdx, px * ig, x);
                    if (deph) swork += sub_step_work(cn, Es, vb, py * ig);
                }
                if (!done) status = PIC_PARTICLE_LOST;
            }
        }
        // a k = 0 step always completes; only sub-cycled lanes can leave the
        // grid inside a step
        cnt.steps[0] += __popcll(lmask & ~hmask);
        if (hmask) {
            // completed sub-cycled steps per k, one distinct k at a time
            uint64_t m = wballot(done & (k > 0));
            while (m) {
                const int kk = __builtin_amdgcn_readlane(k, __ffsll((unsigned long long)m) - 1);
                const uint64_t mk = m & wballot(k == kk);
                if (lane == 0) atomicAdd(&shist[kk], uint32_t(__popcll(mk)));
                m &= ~mk;
            }
            cnt.lost += __popcll(wballot(live & !done));
        }
        if (deph && done) {
            dephasing_update(rmx, gmx, r0v, px, py, pz);
            energy_close(wacc, wem, gst, gamma_of(px, py, pz), swork);
            if (gerr) {
                const double g = gamma_of(px, py, pz);
                const double half = 0.5 * ldexp(1.0, -2 * k);      // dt* / 2, in dt
                gamma_error_update(emx, RD, double(n + 1) - half,
                                   x - half * dtdx * (px / g) - 0.5, g, aiv);
            }
        }

        // hand the step-ahead window to LDS for the next step
        if (pf_next) {
            wave_lds_sync();
#pragma unroll
            for (int h = 0; h < NPF; ++h) {
                const int e = lane + 64 * h;
                if (e < ROWS * PF_NW) pf_dst[4 * h * WWIN] = pf[h];
            }
            wave_lds_sync();
            wlo = nlo;
        }
        win = pf_next;
#pragma unroll
        for (int j = 0; j <= P; ++j) lvo[j] = lvo[j + 1];
        lvo[P + 1] = lvo[P] + ncells == ring_end ? 0 : lvo[P] + ncells;
    }
    if (mine) {
        if (moved) {
            a.x[s] = x_origin + x * dx;
            a.px[s] = px;
            a.py[s] = py;
        }
        a.kold[s] = int8_t(kold);
        a.status[s] = status;
        if (deph) {
            a.rmax[s] = rmx;
            a.gmax[s] = gmx;
            a.work[s] = wacc;
            a.werr[s] = wem;
        }
        if (gerr) a.emax[s] = emx;
    }
    uint64_t *slot = a.cnt + (int64_t(run) * NSLOT + pos % NSLOT) * NCNT;
    if (lane >= 1 && lane <= PIC_K_MAX_LIMIT) {
        const uint32_t v = shist[lane];
        if (v) atomicAdd(reinterpret_cast<unsigned long long *>(slot + lane), v);
    }
    cnt.flush(slot, lane);
}

}  // namespace picsub
