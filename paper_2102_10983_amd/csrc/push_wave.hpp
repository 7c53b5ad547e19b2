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
        if (nonfinite_p(px, py, pz)) x = __builtin_nan("");
        if (KT && a.ktrace) {
            const int64_t u = a.perm[s] - a.kt_first;
            if (u >= 0 && u < a.kt_count) kt_u = u;
        }
    }
    bool moved = false;
    constexpr bool deph = DIAG;   // trajectory diagnostics compiled in
    double r0v = 1.0, rmx = 0.0, wacc = 0.0, wem = 0.0, gmx = 1.0;
    if (deph && mine) {
        r0v = a.r0[s];
        rmx = a.rmax[s];
        gmx = a.gmax[s];
        wacc = a.work[s];
        wem = a.werr[s];
    }
    const bool gerr = deph && a.emax != nullptr && R.atab != nullptr;   // energy error
    double aiv = 0.0, emx = 0.0;
    if (gerr && mine) {
        aiv = a.ai[s];
        emx = a.emax[s];
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
            dephasing_update(rmx, gmx, r0v, px, py, pz);
            energy_close(wacc, wem, gst, gamma_of(px, py, pz), sw);
            if (gerr) {
                const double g = gamma_of(px, py, pz);
                const double half = 0.5 * ldexp(1.0, -2 * k);      // dt* / 2, in dt
                const double xp = x - half * R.dt * (px / g);
                gamma_error_update(emx, R, double(n + 1) - half, (xp - R.x_origin) / R.dx - 0.5,
                                   g, aiv);
            }
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
            a.gmax[s] = gmx;
            a.work[s] = wacc;
            a.werr[s] = wem;
        }
        if (gerr) a.emax[s] = emx;
    }
    cnt.flush(a.cnt + (int64_t(run) * NSLOT + pos % NSLOT) * NCNT, lane);
}

}  // namespace picsub
