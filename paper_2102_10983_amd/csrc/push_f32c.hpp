// push_f32c.hpp -- the FP32-compensated push (pic_precision PIC_FP32_COMP).
//
// Same schedule as the other wavefront kernels: one wavefront per 64-slot
// group for all S steps of the launch.  Registers hold x as an int32 node
// index `cell`, an FP32 fraction `fr` of a cell and its FP32 carry `frc`, and
// each momentum component as an FP32 pair (hi, lo) whose sum is the value.
//
// Precision policy:
//  * FP64: the field levels, the Lagrange weights, the temporal combination
//    and the tent gather, the sub-cycling decision (Sec. IV: B at
//    (x_n, s = 1/2) and gamma of the stored momentum, both from the FP64
//    value of the compensated state), and every sub-cycled step (the
//    stopping points, where gamma is near 1): those run the IEEE FP64 Boris
//    update in node units and are split back into the pairs.
//  * FP32: the Boris update of a k = 0 step (Sec. III, Eqs. (p)..(gamman)),
//    formed as increments of p that TwoSum adds to the (hi, lo) pairs, and
//    the position increment.  Reciprocals and inverse square roots are the
//    hardware estimates refined by one Newton step.
//
// Three rearrangements keep the FP32 increments free of cancellation; each
// is algebraically the Boris update of the equations:
//  * the y increment 2h - a_x s (h = c E, s = 2t / (1 + t^2), t = c B /
//    gamma) is written 2c [(E - B) + B w] with w = 1 - a_x / (gamma (1 +
//    t^2)); E - B is formed in FP64 before rounding, and w's numerator
//    gamma - m_x + t (c B - m_y) uses gamma - m_x = (1 + m_y^2 + m_z^2) /
//    (gamma + m_x) when m_x >= 0.  For an electron riding the wave both
//    terms of 2h - a_x s are about |q E dt| while their difference is of
//    order |q E dt| / gamma, so FP32 rounding of the difference would be
//    amplified by gamma;
//  * the position moves by dt/dx - dt/dx (1 - |v_x|) with 1 - |v_x| =
//    (1 + p_y^2 + p_z^2) / (gamma (gamma + |p_x|)), dt/dx held as an FP32
//    pair: for |v_x| near 1 an FP32 v_x would lose the phase velocity
//    1 - v_x that sets where the electron sees the wave;
//  * c = q dt_p / 2 is an FP32 pair as well (a rounded c would scale every
//    k = 0 step's kicks by the same factor), and the low words of p enter
//    the first operation that uses them.
// What remains is the FP32 rounding of each increment (relative 2^-24),
// which acts on a trajectory like a perturbation of the initial position of
// about 1e-10 relative; electrons whose FP64 trajectory is that sensitive
// (a long ride ending next to a stopping point) differ from the FP64 result
// by the same amount.
#pragma once

#include "common.hpp"
#include "push_fast.hpp"

namespace picsub {

// 1 / b and 1 / sqrt(a) in FP32 (b, a >= 1 here): hardware estimate plus one
// Newton step.
__device__ __forceinline__ float rcpf_nr(float b)
{
    const float r = __builtin_amdgcn_rcpf(b);
    return fmaf(r, fmaf(-b, r, 1.f), r);
}

__device__ __forceinline__ float rsqf_nr(float a)
{
    const float y = __builtin_amdgcn_rsqf(a);
    return fmaf(y, fmaf(-0.5f * a * y, y, 0.5f), y);
}

template <int P, int WPG, bool DIAG = false>
__global__ void __launch_bounds__(64 * WPG) push_wave_fp32c_kernel(PushArgs a)
{
    constexpr int STRIDE = 2 * (P + 1);
    __shared__ double sE_all[WPG][(P + 1) * WWIN];
    __shared__ double sB_all[WPG][(P + 1) * WWIN];
    __shared__ double sBh_all[WPG][WWIN];
    __shared__ double sEn_all[WPG][WWIN];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int pos = blockIdx.x * WPG + wv;
    if (pos >= a.ngroups) return;
    double *sE = sE_all[wv];
    double *sB = sB_all[wv];
    double *sBh = sBh_all[wv];
    double *sEn = sEn_all[wv];
    const int g = __builtin_amdgcn_readfirstlane(a.group_order[pos]);
    const int run = __builtin_amdgcn_readfirstlane(a.group_run[g]);
    const RunDesc R = a.runs[run];                 // wave-uniform: scalar registers
    const int prio = __builtin_amdgcn_readfirstlane(a.group_prio[g]);
    if (prio) set_prio(prio);
    const int64_t n0 = a.n0 != NO_LEVEL ? a.n0 : R.n_cur;
    const int32_t slot0 = int32_t(mod_floor(n0 - P, R.D));
    const int ncm2 = R.ncells - 2;
    const double *W1 = a.wtab;
    const double c0 = 0.5 * R.qm * R.dt;
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
    if (mine) {
        const double xi = (a.x[s] - R.x_origin) / R.dx;
        status = a.status[s];
        if (status == PIC_PARTICLE_LIVE && xi >= 0.0 && xi < double(R.ncells) &&
            !nonfinite_p(a.px[s], a.py[s], a.pz[s])) {
            const double fl = floor(xi);
            cell = int(fl);
            split(xi - fl, fr, frc);
        } else if (status == PIC_PARTICLE_LIVE) {
            cell = -1;     // outside or not finite: flagged at the first step
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
    const float onepz = fmaf(pzh, pzh, 1.f);       // p_z never changes in this geometry

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
        // node window of this step: B at s = 1/2 (the decision's and the k = 0
        // step's) and E of level n, both FP64
        const int lo = max(wave_min(live ? cell - R.margin : INT_MAX), 0);
        const int hi = min(wave_max(live ? cell + R.margin : INT_MIN), R.ncells - 1);
        const bool use_lds = hi - lo + 1 <= WWIN;
        if (use_lds) {
            wave_lds_sync();
            for (int q = lane; q <= hi - lo; q += 64) {
                sBh[q] = node_comb<P>(R.ringB, lv.off, lo + q, W1 + P + 1);
                sEn[q] = R.ringE[lv.off[P] + lo + q];
            }
            wave_lds_sync();
        }
        // tent weights in FP64 from the compensated position
        const double wB = double(fr) + double(frc);
        int iE;
        double wE;
        if (fr >= 0.5f) {
            iE = cell;
            wE = (double(fr) - 0.5) + double(frc);
        } else {
            iE = cell - 1;
            wE = (double(fr) + 0.5) + double(frc);
        }
        // decision (FP64): B at (x_n, s = 1/2), gamma of the stored momentum
        int k = 0;
        double Bd = 0.0;
        bool clamped = false;
        if (live) {
            double b0, b1;
            if (use_lds) {
                b0 = sBh[cell - lo];
                b1 = sBh[cell + 1 - lo];
            } else {
                b0 = node_comb<P>(R.ringB, lv.off, cell, W1 + P + 1);
                b1 = node_comb<P>(R.ringB, lv.off, cell + 1, W1 + P + 1);
            }
            Bd = (1.0 - wB) * b0 + wB * b1;
            const double qx = double(pxh) + double(pxl), qy = double(pyh) + double(pyl);
            const double qz = double(pzh) + double(pzl);
            const double psi0 = fabs(c0 * Bd) * rsq_1nr(1.0 + ((qx * qx + qy * qy) + qz * qz));
            double lim = R.psi_max;
            while (psi0 > lim && k < R.kmax) {
                ++k;
                lim = lim * 4.0;
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
            double e0, e1;
            if (use_lds) {
                e0 = sEn[iE - lo];
                e1 = sEn[iE + 1 - lo];
            } else {
                e0 = R.ringE[lv.off[P] + iE];
                e1 = R.ringE[lv.off[P] + iE + 1];
            }
            const double E = (1.0 - wE) * e0 + wE * e1;
            const float Ef = float(E), Bf = float(Bd), Df = float(E - Bd);
            const double c64 = 0.5 * R.qm * (0.5 * (ldexp(R.dt, -2 * ko) + R.dt));
            const float ch = float(c64), cl = float(c64 - double(ch));
            const double vb = deph ? (double(pyh) + double(pyl)) / gst : 0.0;
            // Boris update as increments (Sec. III), FP32
            const float h = fmaf(cl, Ef, ch * Ef);
            const float my = (pyh + h) + pyl;
            float gg = fmaf(my, my, onepz);
            gg = fmaf(pxh, pxh, gg);
            gg = fmaf(pxh + pxh, pxl, gg);                 // 1 + |m|^2
            const float ig = rsqf_nr(gg);
            const float cB = fmaf(cl, Bf, ch * Bf);
            const float t = cB * ig;
            const float opt = fmaf(t, t, 1.f);
            const float sz = (t + t) * rcpf_nr(opt);
            const float ax = fmaf(my, t, pxh) + pxl;
            const float ay = fmaf(-pxh, t, my);
            const float dpx = ay * sz;
            const float gm = gg * ig;                       // gamma of m
            float num;                                      // gamma (1 + t^2) - a_x
            if (pxh >= 0.f)
                num = fmaf(t, cB - my, fmaf(my, my, onepz) * rcpf_nr(gm + pxh));
            else
                num = fmaf(gm, opt, -ax);
            const float w = num * rcpf_nr(gm * opt);
            const float fy = fmaf(Bf, w, Df);               // (E - B) + B w
            const float dpy = fmaf(cl + cl, fy, (ch + ch) * fy);
            comp_add(pxh, pxl, dpx);
            comp_add(pyh, pyl, dpy);
            if (deph) {
                const double pya = double(pyh) + double(pyl);
                const double ga = gamma_of(double(pxh) + double(pxl), pya, double(pzh) + double(pzl));
                sw = sub_step_work(c64, E, vb, pya / ga);
            }
            // position: dt/dx (1 - (1 - |v_x|)) with the sign of v_x
            float q2 = fmaf(pyh, pyh, pzh * pzh);
            q2 = fmaf(pyh + pyh, pyl, q2);
            float gg2 = 1.f + fmaf(pxh, pxh, q2);
            gg2 = fmaf(pxh + pxh, pxl, gg2);
            const float g2 = gg2 * rsqf_nr(gg2);
            const float omv = (1.f + q2) * rcpf_nr(g2 * (g2 + fabsf(pxh)));   // 1 - |v_x|
            const float sgn = pxh < 0.f ? -1.f : 1.f;
            float s1, e1c;
            two_sum(fr, sgn * dtdx_hi, s1, e1c);
            const float y = (sgn * fmaf(-dtdx_hi, omv, dtdx_lo) + e1c) + frc;
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
            dephasing_update(rmx, gmx, r0v, qx, qy, qz);
            energy_close(wacc, wem, gst, gamma_of(qx, qy, qz), sw);
            if (gerr) {
                const double g = gamma_of(qx, qy, qz);
                const double half = 0.5 * ldexp(1.0, -2 * k);      // dt* / 2, in dt
                const double xi = double(cell) + (double(fr) + double(frc));
                gamma_error_update(emx, R, double(n + 1) - half,
                                   xi - half * R.dtdx * (qx / g) - 0.5, g, aiv);
            }
        }
    }
    if (mine) {
        if (deph) {
            a.rmax[s] = rmx;
            a.gmax[s] = gmx;
            a.work[s] = wacc;
            a.werr[s] = wem;
        }
        if (gerr) a.emax[s] = emx;
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
