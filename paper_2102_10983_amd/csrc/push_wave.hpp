// push_wave.hpp -- asynchronous wavefront push kernels.
//
// Every wavefront owns one group of 64 consecutive slots of one run and
// carries it through all S steps of the launch; wavefronts never wait for
// each other (a workgroup holds WPG independent wavefronts), so a deeply
// sub-cycled group delays only itself while the rest of the machine keeps
// advancing.  Slots are sorted by position at load: the lanes of a group
// hold particles with nearly the same phase history and mostly choose the
// same k.
//
// Per step and lane: the decision (Sec. IV) from B at (x_n, s = 1/2),
// gathered straight from the ring; a k = 0 step is one Boris step with E at
// level n; when any lane sub-cycles, the group's node window is staged once
// in the wavefront's LDS and the 4^k sub-steps of Algorithm 1 read it,
// with the wavefront's issue priority raised (these are the launch's
// longest dependency chains).
#pragma once

#include "common.hpp"

namespace picsub {

// IEEE FP64 throughout (PIC_FP64): the operations and their order are those
// of the CPU oracle, so the results are bit-identical to it.
// KT: the k trace compiled in (launches with a trace buffer attached).
template <int P, int WPG, bool DIAG = false, bool KT = true>
__global__ void __launch_bounds__(64 * WPG) push_wave_kernel(PushArgs a)
{
    constexpr int STRIDE = 2 * (P + 1);
    __shared__ double sE_all[WPG][(P + 1) * WWIN];
    __shared__ double sB_all[WPG][(P + 1) * WWIN];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int pos = blockIdx.x * WPG + wv;
    if (pos >= a.ngroups) return;              // whole wavefront: no barrier below
    double *sE = sE_all[wv];
    double *sB = sB_all[wv];
    const int g = __builtin_amdgcn_readfirstlane(a.group_order[pos]);
    const int run = __builtin_amdgcn_readfirstlane(a.group_run[g]);
    const RunDesc R = a.runs[run];                 // wave-uniform: scalar registers
    const int prio = __builtin_amdgcn_readfirstlane(a.group_prio[g]);
    if (prio) set_prio(prio);
    const int64_t n0 = a.n0 != NO_LEVEL ? a.n0 : R.n_cur;
    const int32_t slot0 = int32_t(mod_floor(n0 - P, R.D));
    const double ncm1 = double(R.ncells - 1);
    const double c0 = 0.5 * R.qm * R.dt;
    const double *LB1 = a.wtab + (P + 1);      // B weights of (k = 0, j = 1): s = 1/2
    WaveCounts cnt;
    cnt.zero();

    const int64_t s = int64_t(g) * 64 + lane;
    const bool mine = s - R.p_off < R.np;
    double x = 0, px = 0, py = 0, pz = 0;
    int kold = 0;
    uint8_t status = PIC_PARTICLE_LOST;
    int64_t kt_u = -1;
    if (mine) {
        x = a.x[s];
        px = a.px[s];
        py = a.py[s];
        pz = a.pz[s];
        kold = a.kold[s];
        status = a.status[s];
        if (KT && a.ktrace) {
            const int64_t u = a.perm[s] - a.kt_first;
            if (u >= 0 && u < a.kt_count) kt_u = u;
        }
    }
    bool moved = false;
    constexpr bool deph = DIAG;   // trajectory diagnostics compiled in
    double r0v = 1.0, rmx = 0.0, wacc = 0.0, wem = 0.0;
    if (deph && mine) {
        r0v = a.r0[s];
        rmx = a.rmax[s];
        wacc = a.work[s];
        wem = a.werr[s];
    }

    const int S_run = run_steps(a, R, n0);
    for (int st = 0; st < S_run; ++st) {
        const int64_t n = n0 + st;
        Levels<P> lv;
        lv.at(slot0, st, R.D, R.ncells);
        double xi = (x - R.x_origin) / R.dx;
        const bool live = status == PIC_PARTICLE_LIVE && xi >= 0.5 && xi < ncm1;
        const bool left = status == PIC_PARTICLE_LIVE && !live;
        cnt.lost += __popcll(__ballot(left));
        if (left) status = PIC_PARTICLE_LOST;
        if (KT && !live) ktrace_put(a, kt_u, n, -1);
        // A wavefront with no live lane left runs on to the end (every
        // access below is behind a live lane); an early exit costs its phi
        // copies on every step.
        // decision: B at (x_n, s = 1/2), gamma of the stored momentum
        int k = 0, cell = 0;
        double Bd = 0.0;
        bool clamped = false;
        double gst = 1.0, sw = 0.0;        // diagnostics: gamma at the step start, step work
        if (live) {
            const double flB = floor(xi);
            cell = int(flB);
            const double wB = xi - flB;
            const double b0 = node_comb<P>(R.ringB, lv.off, cell, LB1);
            const double b1 = node_comb<P>(R.ringB, lv.off, cell + 1, LB1);
            Bd = (1.0 - wB) * b0 + wB * b1;
            const double g0 = sqrt(1.0 + ((px * px + py * py) + pz * pz));
            const double psi0 = fabs(c0 * Bd) / g0;
            gst = g0;
            double lim = R.psi_max;
            while (psi0 > lim && k < R.kmax) {
                ++k;
                lim = lim * 4.0;
            }
            clamped = psi0 > lim;
            if (KT) ktrace_put(a, kt_u, n, int8_t(k));
        }
        cnt.clamps += __popcll(__ballot(clamped));
        const bool heavy = live && k > 0;
        const uint64_t hmask = __ballot(heavy);
        bool use_lds = false;
        int lo = 0;
        if (hmask) {
            lo = max(wave_min(heavy ? cell - R.margin : INT_MAX), 0);
            const int hi = min(wave_max(heavy ? cell + R.margin : INT_MIN), R.ncells - 1);
            use_lds = hi - lo + 1 <= WWIN;
            if (use_lds) {
                wave_lds_sync();
                for (int q = lane; q <= hi - lo; q += 64) {
#pragma unroll
                    for (int j = 0; j <= P; ++j) {
                        sE[j * WWIN + q] = R.ringE[lv.off[j] + lo + q];
                        sB[j * WWIN + q] = R.ringB[lv.off[j] + lo + q];
                    }
                }
                wave_lds_sync();
            }
        }
        bool done = false;
        if (live) {
        moved = true;
        const int ko = kold < 0 ? k : kold;
        kold = k;
        const double dt_new = ldexp(R.dt, -2 * k);
        const double dt_old = ldexp(R.dt, -2 * ko);
        if (k == 0) {
            // s = 1/2 is the time of level n: E's weights are (0, .., 0, 1)
            const double uE = xi - 0.5;
            const double flE = floor(uE);
            const int iE = int(flE);
            const double wE = uE - flE;
            const double e0 = R.ringE[lv.off[P] + iE];
            const double e1 = R.ringE[lv.off[P] + iE + 1];
            const double E = (1.0 - wE) * e0 + wE * e1;
            const double dtp = 0.5 * (dt_old + dt_new);
            const double vb = deph ? py / gst : 0.0;
            boris(R.qm, dtp, E, Bd, px, py, pz);
            const double g2 = sqrt(1.0 + ((px * px + py * py) + pz * pz));
            x = x + dt_new * (px / g2);
            if (deph) sw = sub_step_work((0.5 * R.qm) * dtp, E, vb, py / g2);
            done = true;
        } else {
            set_prio(prio + 2);
            int32_t vo[P + 1];
#pragma unroll
            for (int j = 0; j <= P; ++j) vo[j] = j * WWIN - lo;
            const int nsub = 1 << (2 * k);
            const double *Wk = a.wtab + wtab_offset(k) * STRIDE;
            done = true;
            double gcur = gst;                 // gamma of the momentum before the sub-step
            for (int j = 1; j <= nsub; ++j, Wk += STRIDE) {
                if (j > 1) {
                    xi = (x - R.x_origin) / R.dx;
                    if (!(xi >= 0.5 && xi < ncm1)) {
                        done = false;
                        break;
                    }
                }
                const double fl = floor(xi);
                const int ib = int(fl);
                const double wb = xi - fl;
                const double uE = xi - 0.5;
                const double flE = floor(uE);
                const int ie = int(flE);
                const double we = uE - flE;
                double bb0, bb1, e0, e1;
                if (use_lds) {
                    bb0 = node_comb<P>(sB, vo, ib, Wk + P + 1);
                    bb1 = node_comb<P>(sB, vo, ib + 1, Wk + P + 1);
                    e0 = node_comb<P>(sE, vo, ie, Wk);
                    e1 = node_comb<P>(sE, vo, ie + 1, Wk);
                } else {
                    bb0 = node_comb<P>(R.ringB, lv.off, ib, Wk + P + 1);
                    bb1 = node_comb<P>(R.ringB, lv.off, ib + 1, Wk + P + 1);
                    e0 = node_comb<P>(R.ringE, lv.off, ie, Wk);
                    e1 = node_comb<P>(R.ringE, lv.off, ie + 1, Wk);
                }
                const double B = (1.0 - wb) * bb0 + wb * bb1;
                const double E = (1.0 - we) * e0 + we * e1;
                const double dtp = j == 1 ? 0.5 * (dt_old + dt_new) : dt_new;
                const double vb = deph ? py / gcur : 0.0;
                boris(R.qm, dtp, E, B, px, py, pz);
                const double g2 = sqrt(1.0 + ((px * px + py * py) + pz * pz));
                x = x + dt_new * (px / g2);
                if (deph) {
                    sw += sub_step_work((0.5 * R.qm) * dtp, E, vb, py / g2);
                    gcur = g2;
                }
            }
            set_prio(prio);
            if (!done) status = PIC_PARTICLE_LOST;
        }
        }
        // a k = 0 step always completes; only sub-cycled lanes can leave the
        // grid inside a step
        cnt.steps[0] += __popcll(__ballot(live) & ~hmask);
        if (hmask) {
            cnt.steps_heavy(done, k);
            cnt.lost += __popcll(__ballot(live && !done));
        }
        if (deph && done) {
            dephasing_update(rmx, r0v, px, py, pz);
            energy_close(wacc, wem, gst, gamma_of(px, py, pz), sw);
        }
    }
    if (mine) {
        if (moved) {
            a.x[s] = x;
            a.px[s] = px;
            a.py[s] = py;
            a.pz[s] = pz;
        }
        a.kold[s] = int8_t(kold);
        a.status[s] = status;
        if (deph) {
            a.rmax[s] = rmx;
            a.work[s] = wacc;
            a.werr[s] = wem;
        }
    }
    cnt.flush(a.cnt + (int64_t(run) * NSLOT + pos % NSLOT) * NCNT, lane);
}

// ---------------------------------------------------------------------
// FP32 bulk push (pic_precision PIC_FP32_COMP).
//
// Registers hold x as an int32 node index `cell`, an FP32 fraction `fr` of
// a cell and its FP32 carry, and each momentum component as an FP32 pair
// (hi, lo).  A k = 0 step runs in FP32: the fields come from the FP64
// temporal combination rounded once to FP32, the Boris update is formed as
// increments of p added to (hi, lo) with TwoSum, and the position
// increment uses 1 - |v| = (1 + p_y^2 + p_z^2) / (gamma (gamma + |p_x|)),
// free of cancellation for ultra-relativistic electrons.  A sub-cycled
// step (the stopping points, gamma near 1) runs in FP64 with the FP64
// weights, in node units, then is split back.  The state in HBM stays
// FP64.  For an electron riding the wave the transverse force is a
// cancellation of size E / gamma, so the FP32 rounding here is amplified
// by gamma: this mode trades accuracy (a few 1e-5 at a0 ~ 10..150) for
// arithmetic width.
// ---------------------------------------------------------------------
template <int P, int WPG, bool DIAG = false>
__global__ void __launch_bounds__(64 * WPG) push_wave_fp32c_kernel(PushArgs a)
{
    constexpr int STRIDE = 2 * (P + 1);
    __shared__ double sE_all[WPG][(P + 1) * WWIN];
    __shared__ double sB_all[WPG][(P + 1) * WWIN];
    __shared__ float sBh_all[WPG][WWIN];
    __shared__ float sEn_all[WPG][WWIN];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int pos = blockIdx.x * WPG + wv;
    if (pos >= a.ngroups) return;
    double *sE = sE_all[wv];
    double *sB = sB_all[wv];
    float *sBh = sBh_all[wv];
    float *sEn = sEn_all[wv];
    const int g = __builtin_amdgcn_readfirstlane(a.group_order[pos]);
    const int run = __builtin_amdgcn_readfirstlane(a.group_run[g]);
    const RunDesc R = a.runs[run];                 // wave-uniform: scalar registers
    const int prio = __builtin_amdgcn_readfirstlane(a.group_prio[g]);
    if (prio) set_prio(prio);
    const int64_t n0 = a.n0 != NO_LEVEL ? a.n0 : R.n_cur;
    const int32_t slot0 = int32_t(mod_floor(n0 - P, R.D));
    const int ncm2 = R.ncells - 2;
    const double *W1 = a.wtab;
    const float c0f = float(0.5 * R.qm * R.dt);
    const float psif = float(R.psi_max);
    const float dtdx_hi = float(R.dtdx);
    const float dtdx_lo = float(R.dtdx - double(dtdx_hi));
    WaveCounts cnt;
    cnt.zero();

    const int64_t s = int64_t(g) * 64 + lane;
    const bool mine = s - R.p_off < R.np;
    int cell = 0;
    float fr = 0.f, frc = 0.f, pxh = 0.f, pxl = 0.f, pyh = 0.f, pyl = 0.f, pzh = 0.f, pzl = 0.f;
    int kold = 0;
    uint8_t status = PIC_PARTICLE_LOST;
    int64_t kt_u = -1;
    constexpr bool deph = DIAG;   // trajectory diagnostics compiled in
    double r0v = 1.0, rmx = 0.0, wacc = 0.0, wem = 0.0;
    if (deph && mine) {
        r0v = a.r0[s];
        rmx = a.rmax[s];
        wacc = a.work[s];
        wem = a.werr[s];
    }
    if (mine) {
        const double xi = (a.x[s] - R.x_origin) / R.dx;
        status = a.status[s];
        if (status == PIC_PARTICLE_LIVE && xi >= 0.0 && xi < double(R.ncells)) {
            const double fl = floor(xi);
            cell = int(fl);
            split(xi - fl, fr, frc);
        } else if (status == PIC_PARTICLE_LIVE) {
            cell = -1;     // outside: flagged at the first step
        }
        split(a.px[s], pxh, pxl);
        split(a.py[s], pyh, pyl);
        split(a.pz[s], pzh, pzl);
        kold = a.kold[s];
        if (a.ktrace) {
            const int64_t u = a.perm[s] - a.kt_first;
            if (u >= 0 && u < a.kt_count) kt_u = u;
        }
    }
    bool moved = false;

    const int S_run = run_steps(a, R, n0);
    for (int st = 0; st < S_run; ++st) {
        const int64_t n = n0 + st;
        Levels<P> lv;
        lv.at(slot0, st, R.D, R.ncells);
        const bool live = status == PIC_PARTICLE_LIVE && cell >= 0 && cell <= ncm2 &&
                          (cell > 0 || fr >= 0.5f);
        const bool left = status == PIC_PARTICLE_LIVE && !live;
        cnt.lost += __popcll(__ballot(left));
        if (left) status = PIC_PARTICLE_LOST;
        if (!live) ktrace_put(a, kt_u, n, -1);
        if (!__any(live)) {
            for (int s2 = st + 1; s2 < S_run; ++s2) ktrace_put(a, kt_u, n0 + s2, -1);
            break;
        }
        const int lo = max(wave_min(live ? cell - R.margin : INT_MAX), 0);
        const int hi = min(wave_max(live ? cell + R.margin : INT_MIN), R.ncells - 1);
        const bool use_lds = hi - lo + 1 <= WWIN;
        if (use_lds) {
            wave_lds_sync();
            for (int q = lane; q <= hi - lo; q += 64) {
                const double b = node_comb<P>(R.ringB, lv.off, lo + q, W1 + P + 1);
                sBh[q] = float(b);
                sEn[q] = float(R.ringE[lv.off[P] + lo + q]);
            }
            wave_lds_sync();
        }
        int k = 0;
        float Bd = 0.f;
        bool clamped = false;
        const float wB = fr;
        int iE;
        float wE;
        if (fr >= 0.5f) {
            iE = cell;
            wE = fr - 0.5f;
        } else {
            iE = cell - 1;
            wE = fr + 0.5f;
        }
        if (live) {
            float b0, b1;
            if (use_lds) {
                b0 = sBh[cell - lo];
                b1 = sBh[cell + 1 - lo];
            } else {
                b0 = float(node_comb<P>(R.ringB, lv.off, cell, W1 + P + 1));
                b1 = float(node_comb<P>(R.ringB, lv.off, cell + 1, W1 + P + 1));
            }
            Bd = (1.f - wB) * b0 + wB * b1;
            const float p2 = (pxh * pxh + pyh * pyh) + pzh * pzh;
            const float psi0 = fabsf(c0f * Bd) * __builtin_amdgcn_rsqf(1.f + p2);
            float lim = psif;
            while (psi0 > lim && k < R.kmax) {
                ++k;
                lim = lim * 4.f;
            }
            clamped = psi0 > lim;
            ktrace_put(a, kt_u, n, int8_t(k));
        }
        cnt.clamps += __popcll(__ballot(clamped));
        const bool heavy = live && k > 0;
        if (__any(heavy) && use_lds) {
            wave_lds_sync();
            for (int q = lane; q <= hi - lo; q += 64) {
#pragma unroll
                for (int j = 0; j <= P; ++j) {
                    sE[j * WWIN + q] = R.ringE[lv.off[j] + lo + q];
                    sB[j * WWIN + q] = R.ringB[lv.off[j] + lo + q];
                }
            }
            wave_lds_sync();
        }
        bool done = false;
        double gst = 1.0, sw = 0.0;        // diagnostics: gamma at the step start, step work
        if (live) {
        moved = true;
        const int ko = kold < 0 ? k : kold;
        kold = k;
        if (deph)
            gst = gamma_of(double(pxh) + double(pxl), double(pyh) + double(pyl),
                           double(pzh) + double(pzl));
        if (!heavy) {
            float e0, e1;
            if (use_lds) {
                e0 = sEn[iE - lo];
                e1 = sEn[iE + 1 - lo];
            } else {
                e0 = float(R.ringE[lv.off[P] + iE]);
                e1 = float(R.ringE[lv.off[P] + iE + 1]);
            }
            const float E = (1.f - wE) * e0 + wE * e1;
            const float cf = float(0.5 * R.qm * (0.5 * (ldexp(R.dt, -2 * ko) + R.dt)));
            const double vb = deph ? (double(pyh) + double(pyl)) / gst : 0.0;
            const float h = cf * E;
            const float mx = pxh, my = pyh + h, mz = pzh;
            const float igf = __builtin_amdgcn_rsqf(1.f + ((mx * mx + my * my) + mz * mz));
            const float t = cf * Bd * igf;
            const float sz = 2.f * t * __builtin_amdgcn_rcpf(1.f + t * t);
            const float ax = mx + my * t;
            const float ay = my - mx * t;
            comp_add(pxh, pxl, ay * sz);
            comp_add(pyh, pyl, (h + h) - ax * sz);
            if (deph) {
                const double pya = double(pyh) + double(pyl);
                const double ga = gamma_of(double(pxh) + double(pxl), pya, double(pzh) + double(pzl));
                sw = sub_step_work((0.5 * R.qm) * (0.5 * (ldexp(R.dt, -2 * ko) + R.dt)), double(E),
                                   vb, pya / ga);
            }
            const float q2 = (pyh * pyh + pzh * pzh);
            const float g2 = __builtin_amdgcn_sqrtf(1.f + (pxh * pxh + q2));
            const float omv = (1.f + q2) * __builtin_amdgcn_rcpf(g2 * (g2 + fabsf(pxh)));  // 1 - |v|
            const float sgn = pxh < 0.f ? -1.f : 1.f;
            float s1, e1c;
            two_sum(fr, sgn * dtdx_hi, s1, e1c);
            const float y = ((sgn * (dtdx_lo - dtdx_hi * omv)) + e1c) + frc;
            float s2, e2;
            two_sum(s1, y, s2, e2);
            const float adj = s2 >= 1.f ? -1.f : (s2 < 0.f ? 1.f : 0.f);
            cell -= int(adj);
            float e3;
            two_sum(s2, adj, fr, e3);
            frc = e2 + e3;
            done = true;
        } else {
            set_prio(prio + 2);
            double xi = double(cell) + (double(fr) + double(frc));
            double px = double(pxh) + double(pxl);
            double py = double(pyh) + double(pyl);
            double pz = double(pzh) + double(pzl);
            const double dt_new = ldexp(R.dt, -2 * k);
            const double dt_old = ldexp(R.dt, -2 * ko);
            const double rdx = ldexp(R.dtdx, -2 * k);
            const int nsub = 1 << (2 * k);
            const double *Wk = a.wtab + wtab_offset(k) * STRIDE;
            int32_t vo[P + 1];
#pragma unroll
            for (int j = 0; j <= P; ++j) vo[j] = j * WWIN - lo;
            const double ncm1 = double(R.ncells - 1);
            done = true;
            double gcur = gst;
            for (int j = 1; j <= nsub; ++j, Wk += STRIDE) {
                if (!(xi >= 0.5 && xi < ncm1)) {
                    done = false;
                    break;
                }
                const double fl = floor(xi);
                const int ib = int(fl);
                const double wb = xi - fl;
                const double uE = xi - 0.5;
                const double flE = floor(uE);
                const int ie = int(flE);
                const double we = uE - flE;
                double bb0, bb1, ee0, ee1;
                if (use_lds) {
                    bb0 = node_comb<P>(sB, vo, ib, Wk + P + 1);
                    bb1 = node_comb<P>(sB, vo, ib + 1, Wk + P + 1);
                    ee0 = node_comb<P>(sE, vo, ie, Wk);
                    ee1 = node_comb<P>(sE, vo, ie + 1, Wk);
                } else {
                    bb0 = node_comb<P>(R.ringB, lv.off, ib, Wk + P + 1);
                    bb1 = node_comb<P>(R.ringB, lv.off, ib + 1, Wk + P + 1);
                    ee0 = node_comb<P>(R.ringE, lv.off, ie, Wk);
                    ee1 = node_comb<P>(R.ringE, lv.off, ie + 1, Wk);
                }
                const double B = (1.0 - wb) * bb0 + wb * bb1;
                const double E = (1.0 - we) * ee0 + we * ee1;
                const double dtp = j == 1 ? 0.5 * (dt_old + dt_new) : dt_new;
                const double vb = deph ? py / gcur : 0.0;
                boris(R.qm, dtp, E, B, px, py, pz);
                const double g2 = sqrt(1.0 + ((px * px + py * py) + pz * pz));
                xi = xi + rdx * (px / g2);
                if (deph) {
                    sw += sub_step_work((0.5 * R.qm) * dtp, E, vb, py / g2);
                    gcur = g2;
                }
            }
            set_prio(prio);
            if (!done) status = PIC_PARTICLE_LOST;
            const double fl = floor(xi);
            cell = (xi >= 0.0 && xi < double(R.ncells)) ? int(fl) : -1;
            split(xi - fl, fr, frc);
            split(px, pxh, pxl);
            split(py, pyh, pyl);
            split(pz, pzh, pzl);
        }
        }
        cnt.steps_done(done, k);
        cnt.lost += __popcll(__ballot(live && !done));
        if (deph && done) {
            const double qx = double(pxh) + double(pxl), qy = double(pyh) + double(pyl);
            const double qz = double(pzh) + double(pzl);
            dephasing_update(rmx, r0v, qx, qy, qz);
            energy_close(wacc, wem, gst, gamma_of(qx, qy, qz), sw);
        }
    }
    if (mine) {
        if (deph) {
            a.rmax[s] = rmx;
            a.work[s] = wacc;
            a.werr[s] = wem;
        }
        if (moved) {
            const double xi = double(cell) + (double(fr) + double(frc));
            a.x[s] = R.x_origin + xi * R.dx;
            a.px[s] = double(pxh) + double(pxl);
            a.py[s] = double(pyh) + double(pyl);
            a.pz[s] = double(pzh) + double(pzl);
        }
        a.kold[s] = int8_t(kold);
        a.status[s] = status;
    }
    cnt.flush(a.cnt + (int64_t(run) * NSLOT + pos % NSLOT) * NCNT, lane);
}

}  // namespace picsub
