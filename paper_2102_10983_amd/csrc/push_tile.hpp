// push_tile.hpp -- tiled push with per-step compaction by k
// (pic_binning PIC_BIN_BALLOT, FP64).
//
// A workgroup of TILE threads owns TILE consecutive slots of one run (one
// particle per thread) for all S steps of a launch.  Per step:
//   1. the node window its live particles can touch during the step (a
//      particle crosses fewer than dt/dx cells per step) is reduced over the
//      workgroup and the P+1 levels of E and B on it are staged in LDS,
//      together with B interpolated to s = 1/2;
//   2. every thread takes the decision for its particle; k = 0 particles
//      do their single sub-step in place;
//   3. sub-cycled particles leave their state in LDS and are appended to a
//      per-k queue with a ballot and a lane rank (mbcnt), so each queue is
//      a dense list; full 64-lane chunks of one k are run by the
//      workgroup's wavefronts, heaviest k first, with wave-uniform weights;
//   4. owners pick their updated state back up.
// Every particle sees exactly the arithmetic of the IEEE wavefront kernel;
// only the lane doing it changes.  The price is a workgroup barrier per
// step, which ties a tile to its slowest chunk.
#pragma once

#include "common.hpp"

namespace picsub {

constexpr int WMAX = 256;   // staged nodes per field level

template <int P, int TILE, bool DIAG = false>
__global__ void __launch_bounds__(TILE) push_tile_kernel(PushArgs a)
{
    constexpr int STRIDE = 2 * (P + 1);
    constexpr int NWAVE = TILE / 64;
    __shared__ double sE[(P + 1) * WMAX];
    __shared__ double sB[(P + 1) * WMAX];
    __shared__ double sBh[WMAX];
    __shared__ double sx[TILE], spx[TILE], spy[TILE], spz[TILE];
    __shared__ uint8_t sst[TILE];
    __shared__ double swk[DIAG ? TILE : 1];    // work of a sub-cycled step (diagnostics)
    __shared__ uint16_t sq[PIC_K_MAX_LIMIT + 1][TILE];
    __shared__ int sqn[PIC_K_MAX_LIMIT + 1];
    __shared__ int slo[2], shi[2];   // window bounds, double-buffered by step parity

    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int64_t first = int64_t(blockIdx.x) * TILE;
    const int run = a.group_run[first / 64];
    const RunDesc &R = a.runs[run];
    const int64_t n0 = a.n0 != NO_LEVEL ? a.n0 : R.n_cur;
    const int32_t slot0 = int32_t(mod_floor(n0 - P, R.D));
    const double ncm1 = double(R.ncells - 1);
    const double c0 = 0.5 * R.qm * R.dt;
    const double *W1 = a.wtab;
    Counts cnt;
    cnt.zero();

    if (t <= PIC_K_MAX_LIMIT) sqn[t] = 0;
    if (t < 2) {
        slo[t] = INT_MAX;
        shi[t] = INT_MIN;
    }
    const int64_t i = first + t;
    const bool mine = i - R.p_off < R.np;
    double x = 0, px = 0, py = 0, pz = 0;
    int kold = 0;
    uint8_t status = PIC_PARTICLE_LOST;
    int64_t kt_u = -1;
    constexpr bool deph = DIAG;   // trajectory diagnostics compiled in
    double r0v = 1.0, rmx = 0.0, wacc = 0.0, wem = 0.0, gmx = 1.0;
    if (deph && mine) {
        r0v = a.r0[i];
        rmx = a.rmax[i];
        gmx = a.gmax[i];
        wacc = a.work[i];
        wem = a.werr[i];
    }
    const bool gerr = deph && a.emax != nullptr && R.atab != nullptr;   // energy error
    double aiv = 0.0, emx = 0.0;
    if (gerr && mine) {
        aiv = a.ai[i];
        emx = a.emax[i];
    }
    // the energy error after a completed step of level n at level k
    auto gerr_step = [&](int64_t n, int k) {
        const double g = gamma_of(px, py, pz);
        const double half = 0.5 * ldexp(1.0, -2 * k);      // dt* / 2, in dt
        const double xp = x - half * R.dt * (px / g);
        gamma_error_update(emx, R, double(n + 1) - half, (xp - R.x_origin) / R.dx - 0.5, g, aiv);
    };
    if (mine) {
        x = a.x[i];
        px = a.px[i];
        py = a.py[i];
        pz = a.pz[i];
        kold = a.kold[i];
        status = a.status[i];
        if (a.ktrace) {
            const int64_t u = a.perm[i] - a.kt_first;
            if (u >= 0 && u < a.kt_count) kt_u = u;
        }
    }
    __syncthreads();

    const int S_run = run_steps(a, R, n0);
    if (S_run > 0 && status == PIC_PARTICLE_LIVE && nonfinite_p(px, py, pz)) {
        status = PIC_PARTICLE_LOST;
        ++cnt.lost;
    }
    for (int st = 0; st < S_run; ++st) {
        const int64_t n = n0 + st;
        Levels<P> lv;
        lv.at(slot0, st, R.D, R.ncells);
        // -- 1. window of nodes the tile may touch during the step
        double xi = (x - R.x_origin) / R.dx;
        const bool live = status == PIC_PARTICLE_LIVE && xi >= 0.5 && xi < ncm1;
        if (status == PIC_PARTICLE_LIVE && !live) {
            status = PIC_PARTICLE_LOST;
            ++cnt.lost;
        }
        if (!live) ktrace_put(a, kt_u, n, -1);
        const int par = st & 1;
        const int cell = live ? int(floor(xi)) : 0;
        const int wlo = wave_min(live ? cell - R.margin : INT_MAX);
        const int whi = wave_max(live ? cell + R.margin : INT_MIN);
        if (lane == 0 && wlo <= whi) {
            atomicMin(&slo[par], wlo);
            atomicMax(&shi[par], whi);
        }
        __syncthreads();
        const int lo = max(slo[par], 0);
        const int hi = min(shi[par], R.ncells - 1);
        const bool any = slo[par] <= shi[par];
        const bool use_lds = any && hi - lo + 1 <= WMAX;
        if (use_lds) {
            for (int q = t; q <= hi - lo; q += TILE) {
                double bh = 0;
#pragma unroll
                for (int j = 0; j <= P; ++j) {
                    const double e = R.ringE[lv.off[j] + lo + q];
                    const double b = R.ringB[lv.off[j] + lo + q];
                    sE[j * WMAX + q] = e;
                    sB[j * WMAX + q] = b;
                    bh = j == 0 ? W1[P + 1] * b : bh + W1[P + 1 + j] * b;
                }
                sBh[q] = bh;
            }
        }
        __syncthreads();
        // every thread has read this parity's bounds; the next writes to
        // them come two steps on, after the next step's first barrier
        if (t == 0) {
            slo[par] = INT_MAX;
            shi[par] = INT_MIN;
        }
        if (!any) {                    // uniform: nothing live in this tile any more
            for (int s2 = st + 1; s2 < S_run; ++s2) ktrace_put(a, kt_u, n0 + s2, -1);
            break;
        }
        int32_t vo[P + 1];
#pragma unroll
        for (int j = 0; j <= P; ++j) vo[j] = j * WMAX - lo;

        // -- 2. decision, k = 0 steps in place
        bool heavy = false;
        int k = 0;
        double gst = 1.0;                  // diagnostics: gamma at the step start
        if (live) {
            const double flB = floor(xi);
            const int iB = int(flB);
            const double wB = xi - flB;
            double f0, f1;
            if (use_lds) {
                f0 = sBh[iB - lo];
                f1 = sBh[iB + 1 - lo];
            } else {
                f0 = node_comb<P>(R.ringB, lv.off, iB, W1 + P + 1);
                f1 = node_comb<P>(R.ringB, lv.off, iB + 1, W1 + P + 1);
            }
            const double Bd = (1.0 - wB) * f0 + wB * f1;
            const double g0 = sqrt(1.0 + ((px * px + py * py) + pz * pz));
            const double psi0 = fabs(c0 * Bd) / g0;
            gst = g0;
            double lim = R.psi_max;
            while (psi0 > lim && k < R.kmax) {
                ++k;
                lim = lim * 4.0;
            }
            cnt.clamps += psi0 > lim;
            ktrace_put(a, kt_u, n, int8_t(k));
            const int ko = kold < 0 ? k : kold;
            kold = k;
            if (k == 0) {
                const double uE = xi - 0.5;
                const double flE = floor(uE);
                const int iE = int(flE);
                const double wE = uE - flE;
                double e0, e1;
                if (use_lds) {
                    e0 = sE[vo[P] + iE];
                    e1 = sE[vo[P] + iE + 1];
                } else {
                    e0 = R.ringE[lv.off[P] + iE];
                    e1 = R.ringE[lv.off[P] + iE + 1];
                }
                const double E = (1.0 - wE) * e0 + wE * e1;
                const double dto = ldexp(R.dt, -2 * ko);
                const double vb = deph ? py / g0 : 0.0;
                boris(R.qm, 0.5 * (dto + R.dt), E, Bd, px, py, pz);
                const double g2 = sqrt(1.0 + ((px * px + py * py) + pz * pz));
                x = x + R.dt * (px / g2);
                cnt.step_done(0);
                if (deph) {
                    dephasing_update(rmx, gmx, r0v, px, py, pz);
                    energy_close(wacc, wem, g0, gamma_of(px, py, pz),
                                 sub_step_work((0.5 * R.qm) * (0.5 * (dto + R.dt)), E, vb, py / g2));
                    if (gerr) gerr_step(n, 0);
                }
            } else {
                heavy = true;
                sx[t] = x;
                spx[t] = px;
                spy[t] = py;
                spz[t] = pz;
                sst[t] = uint8_t(ko);      // dt*_old travels with the state
            }
        }
        // -- 3. per-k queues: ballot + lane rank
        if (__syncthreads_or(heavy)) {
            for (int kk = 1; kk <= R.kmax; ++kk) {
                const uint64_t m = __ballot(heavy && k == kk);
                if (m) {
                    int base = 0;
                    if (lane == 0) base = atomicAdd(&sqn[kk], __popcll(m));
                    base = __shfl(base, 0);
                    if (heavy && k == kk) {
                        const uint32_t below = __builtin_amdgcn_mbcnt_hi(
                            uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
                        sq[kk][base + below] = uint16_t(t);
                    }
                }
            }
            __syncthreads();
            int total = 0;
            for (int kk = R.kmax; kk >= 1; --kk) total += (sqn[kk] + 63) >> 6;
            for (int gch = wave; gch < total; gch += NWAVE) {
                int kk = R.kmax, c = gch;
                while (c >= ((sqn[kk] + 63) >> 6)) {
                    c -= (sqn[kk] + 63) >> 6;
                    --kk;
                }
                kk = __builtin_amdgcn_readfirstlane(kk);
                const int e = c * 64 + lane;
                if (e >= sqn[kk]) continue;
                const int who = sq[kk][e];
                double hx = sx[who], hpx = spx[who], hpy = spy[who], hpz = spz[who];
                const int ko = sst[who];
                const double dt_new = ldexp(R.dt, -2 * kk);
                const double dt_old = ldexp(R.dt, -2 * ko);
                const int nsub = 1 << (2 * kk);
                const double *Wk = a.wtab + wtab_offset(kk) * STRIDE;
                uint8_t hst = PIC_PARTICLE_LIVE;
                double hsw = 0.0, hg = deph ? gamma_of(hpx, hpy, hpz) : 1.0;
                for (int j = 1; j <= nsub; ++j, Wk += STRIDE) {
                    const double hxi = (hx - R.x_origin) / R.dx;
                    if (!(hxi >= 0.5 && hxi < ncm1)) {
                        hst = PIC_PARTICLE_LOST;
                        break;
                    }
                    const double flB = floor(hxi);
                    const int iB = int(flB);
                    const double wB = hxi - flB;
                    const double uE = hxi - 0.5;
                    const double flE = floor(uE);
                    const int iE = int(flE);
                    const double wE = uE - flE;
                    double b0, b1, e0, e1;
                    if (use_lds) {
                        b0 = node_comb<P>(sB, vo, iB, Wk + P + 1);
                        b1 = node_comb<P>(sB, vo, iB + 1, Wk + P + 1);
                        e0 = node_comb<P>(sE, vo, iE, Wk);
                        e1 = node_comb<P>(sE, vo, iE + 1, Wk);
                    } else {
                        b0 = node_comb<P>(R.ringB, lv.off, iB, Wk + P + 1);
                        b1 = node_comb<P>(R.ringB, lv.off, iB + 1, Wk + P + 1);
                        e0 = node_comb<P>(R.ringE, lv.off, iE, Wk);
                        e1 = node_comb<P>(R.ringE, lv.off, iE + 1, Wk);
                    }
                    const double B = (1.0 - wB) * b0 + wB * b1;
                    const double E = (1.0 - wE) * e0 + wE * e1;
                    const double dtp = j == 1 ? 0.5 * (dt_old + dt_new) : dt_new;
                    const double vb = deph ? hpy / hg : 0.0;
                    boris(R.qm, dtp, E, B, hpx, hpy, hpz);
                    const double g2 = sqrt(1.0 + ((hpx * hpx + hpy * hpy) + hpz * hpz));
                    hx = hx + dt_new * (hpx / g2);
                    if (deph) {
                        hsw += sub_step_work((0.5 * R.qm) * dtp, E, vb, hpy / g2);
                        hg = g2;
                    }
                }
                if (deph) swk[who] = hsw;
                sx[who] = hx;
                spx[who] = hpx;
                spy[who] = hpy;
                spz[who] = hpz;
                sst[who] = hst == PIC_PARTICLE_LIVE ? uint8_t(0xFF) : hst;
            }
            __syncthreads();
            if (heavy) {
                x = sx[t];
                px = spx[t];
                py = spy[t];
                pz = spz[t];
                if (sst[t] == 0xFF) {
                    cnt.step_done(k);
                    if (deph) {
                        dephasing_update(rmx, gmx, r0v, px, py, pz);
                        energy_close(wacc, wem, gst, gamma_of(px, py, pz), swk[t]);
                        if (gerr) gerr_step(n, k);
                    }
                } else {
                    status = PIC_PARTICLE_LOST;
                    ++cnt.lost;
                }
            }
            if (t <= PIC_K_MAX_LIMIT) sqn[t] = 0;   // ordered before new queues by the next barrier
        }
    }
    if (mine) {
        a.x[i] = x;
        a.px[i] = px;
        a.py[i] = py;
        a.pz[i] = pz;
        a.kold[i] = int8_t(kold);
        a.status[i] = status;
        if (deph) {
            a.rmax[i] = rmx;
            a.gmax[i] = gmx;
            a.work[i] = wacc;
            a.werr[i] = wem;
        }
        if (gerr) a.emax[i] = emx;
    }
    flush_wave(cnt, a.cnt + (int64_t(run) * NSLOT + blockIdx.x % NSLOT) * NCNT, lane);
}

}  // namespace picsub
