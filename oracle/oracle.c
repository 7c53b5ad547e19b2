/*
 * oracle.c -- plain FP64 CPU reference of the sub-cycled Boris push.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Written for readability: one
 * particle at a time, every step in the order the paper states it, no
 * blocking, fusion or reordering.  Build with -ffp-contract=off so that no
 * multiply-add is fused.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ */
/* Lagrange coefficients, Sec. VI.                                     */
/* The field is wanted at t = (n - 1/2) dt + dt' and s = dt'/dt.       */
/* Eq. (lagrange2-2): L^B_j = prod_{k != j} (p - k - 1 + s) / (j - k)  */
/* Eq. (lagrange2-3): L^E_j = prod_{k != j} (p - k - 1/2 + s) / (j - k) */
/* The numerator is multiplied with k ascending and divided once by    */
/* the integer denominator.                                            */
/* ------------------------------------------------------------------ */
int orc_lagrange(int32_t p, double s, double *LE, double *LB)
{
    if (p < 0 || p > ORC_MAX_ORDER) return -1;
    for (int j = 0; j <= p; ++j) {
        double numB = 1.0, numE = 1.0, den = 1.0;
        for (int k = 0; k <= p; ++k) {
            if (k == j) continue;
            numB = numB * ((double)(p - k - 1) + s);
            numE = numE * (((double)(p - k) - 0.5) + s);
            den = den * (double)(j - k);
        }
        LB[j] = numB / den;
        LE[j] = numE / den;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Field storage.  Level m holds E_y at t = m dt on nodes (i+1/2) dx   */
/* and B_z at t = (m+1/2) dt on nodes i dx: the Yee staggering of      */
/* Sec. III, Eqs. (Ey) and (Bz).                                       */
/* ------------------------------------------------------------------ */
static int level_value(const orc_fields *f, int32_t ncells, int32_t which,
                       int64_t m, int32_t i, double *v)
{
    if (f->mode == 0) {
        if (m < f->lev0 || m >= f->lev0 + f->nlev) return -2;
        const double *a = which == 0 ? f->E : f->B;
        *v = a[(m - f->lev0) * (int64_t)ncells + i];
        return 0;
    }
    int64_t a = which == 0 ? f->aE : f->aB;
    int64_t b = which == 0 ? f->bE : f->bB;
    int64_t c = which == 0 ? f->cE : f->cB;
    int64_t idx = (a * m + b * (int64_t)i + c) % f->M;
    if (idx < 0) idx += f->M;
    *v = f->table[idx];
    return 0;
}

/* Temporal interpolation at one node, Eqs. (lagrange1-2) and           */
/* (lagrange1-3): F' = sum_j F|_{level n+j-p} L_j, j ascending.         */
static int node_value(const orc_fields *f, int32_t ncells, int32_t p,
                      int32_t which, int64_t n, int32_t i, const double *L,
                      double *out)
{
    double v, acc;
    if (level_value(f, ncells, which, n - p, i, &v)) return -2;
    acc = L[0] * v;
    for (int j = 1; j <= p; ++j) {
        if (level_value(f, ncells, which, n + j - p, i, &v)) return -2;
        acc = acc + L[j] * v;
    }
    *out = acc;
    return 0;
}

/* Fractional node coordinate of a particle: B nodes sit at i dx, E nodes
 * at (i+1/2) dx, measured from x_origin. */
static double grid_coord(const orc_params *prm, double x)
{
    return (x - prm->x_origin) / prm->dx;
}

/* Both tent nodes of E and of B exist iff 1/2 <= xi < ncells - 1. */
static int in_grid(const orc_params *prm, double xi)
{
    return xi >= 0.5 && xi < (double)(prm->ncells - 1);
}

/* Tent (triangular) shape, Eqs. (Enp) and (Bnp): the two nearest nodes
 * with weights 1 - w and w. */
static int tent(const orc_params *prm, const orc_fields *f, int32_t which,
                int64_t n, double xi, const double *L, double *out)
{
    double u = which == 0 ? xi - 0.5 : xi;
    double fl = floor(u);
    int32_t i0 = (int32_t)fl;
    double w = u - fl;
    double f0, f1;
    if (node_value(f, prm->ncells, prm->order, which, n, i0, L, &f0)) return -2;
    if (node_value(f, prm->ncells, prm->order, which, n, i0 + 1, L, &f1)) return -2;
    *out = (1.0 - w) * f0 + w * f1;
    return 0;
}

int orc_gather(const orc_params *prm, const orc_fields *f, int32_t which,
               int64_t n, double s, double x, double *out)
{
    double LE[ORC_MAX_ORDER + 1], LB[ORC_MAX_ORDER + 1];
    if (orc_lagrange(prm->order, s, LE, LB)) return -3;
    double xi = grid_coord(prm, x);
    if (!in_grid(prm, xi)) return -1;
    return tent(prm, f, which, n, xi, which == 0 ? LE : LB, out);
}

/* ------------------------------------------------------------------ */
/* Sub-cycling criterion, Sec. IV: dt* = dt / 4^k with k the smallest   */
/* whole number that brings the rotation |Psi| = psi0 / 4^k within      */
/* psi_max.  Algorithm 1 divides dt*_new by 4 while |Psi| > psi_max;    */
/* scaling psi_max by 4^k instead is exact (a power of two).            */
/* ------------------------------------------------------------------ */
int32_t orc_decide_k(double psi0, double psi_max, int32_t k_max,
                     int32_t *clamped)
{
    int32_t k = 0;
    double lim = psi_max;
    while (psi0 > lim && k < k_max) {
        k = k + 1;
        lim = lim * 4.0;
    }
    *clamped = psi0 > lim;
    return k;
}

/* ------------------------------------------------------------------ */
/* Relativistic Boris push, Sec. III, Eqs. (p)..(gamman), with E = E_y   */
/* y-hat and B = B_z z-hat (1D model problem):                          */
/*   p-  = p + q E dt/2                                                 */
/*   Psi = q B dt / (2 gamma_n m),  gamma_n from p-                     */
/*   p'  = p- + p- x Psi,  s = 2 Psi / (1 + Psi^2),  p+ = p- + p' x s   */
/*   p   = p+ + q E dt/2                                                */
/* ------------------------------------------------------------------ */
void orc_boris(double qm, double dtp, double E, double B,
               double *px, double *py, double *pz)
{
    double c = 0.5 * qm * dtp;
    double h = c * E;                            /* q E dt / 2 along y */
    double mx = *px, my = *py + h, mz = *pz;     /* p- */
    double g = sqrt(1.0 + ((mx * mx + my * my) + mz * mz)); /* gamma_n */
    double t = (c * B) / g;                      /* Psi (z component) */
    double sz = (2.0 * t) / (1.0 + t * t);       /* s (z component) */
    double ax = mx + my * t;                     /* p' = p- + p- x Psi */
    double ay = my - mx * t;
    *px = mx + ay * sz;                          /* p+ = p- + p' x s */
    *py = (my - ax * sz) + h;                    /* ... + q E dt / 2 */
    *pz = mz;
}

/* Position update, Eqs. (gamma)..(x): x += dt v_x, v = p / gamma. */
static double advance_x(double x, double dtn, double px, double py, double pz)
{
    double g = sqrt(1.0 + ((px * px + py * py) + pz * pz));
    return x + dtn * (px / g);
}

/* ------------------------------------------------------------------ */
/* One particle over one step of size dt (x: n dt -> (n+1) dt), as in  */
/* Algorithm 1 with the reading counter = dt / dt*_new = 4^k.          */
/* Returns 0, 1 when the particle left the grid, -2 on a missing level. */
/* ------------------------------------------------------------------ */
typedef struct {
    uint64_t steps, sub_steps, n_star, clamps, lost;
    uint64_t steps_by_k[ORC_KHIST], sub_steps_by_k[ORC_KHIST];
} local_cnt;

static int one_step(const orc_params *prm, const orc_fields *f, int64_t n,
                    double *x, double *px, double *py, double *pz,
                    int8_t *k_old, int forced, int32_t *k_out,
                    double *psi_ratio, double *step_work, local_cnt *lc)
{
    double LE[ORC_MAX_ORDER + 1], LB[ORC_MAX_ORDER + 1];
    double Ep, Bp;
    int rc;

    /* a state that is not finite is frozen and flagged like a particle that
     * left the grid (the paper's electrons always have a finite state; the
     * rule only keeps bad input from spreading) */
    if (!isfinite(*x) || !isfinite(*px) || !isfinite(*py) || !isfinite(*pz)) return 1;
    /* decision: Psi over a full dt with B at (x_n, s = 1/2) and gamma of
     * the stored momentum (Sec. IV) */
    double xi = grid_coord(prm, *x);
    if (!in_grid(prm, xi)) return 1;
    orc_lagrange(prm->order, 0.5, LE, LB);
    if ((rc = tent(prm, f, 1, n, xi, LB, &Bp))) return rc;
    double g0 = sqrt(1.0 + ((*px * *px + *py * *py) + *pz * *pz));
    double psi0 = fabs((0.5 * prm->qm * prm->dt) * Bp) / g0;
    int32_t clamped = 0;
    int32_t k = orc_decide_k(psi0, prm->psi_max, prm->k_max, &clamped);
    if (forced >= 0) { k = forced; clamped = 0; }
    *psi_ratio = psi0 / prm->psi_max;
    *k_out = k;

    int32_t kold = *k_old < 0 ? k : (int32_t)*k_old;
    double dt_new = ldexp(prm->dt, -2 * k);     /* dt / 4^k */
    double dt_old = ldexp(prm->dt, -2 * kold);
    int64_t nsub = (int64_t)1 << (2 * k);
    double ds = ldexp(1.0, -2 * k);              /* 4^-k */

    lc->clamps += (uint64_t)clamped;
    *k_old = (int8_t)k;

    for (int64_t j = 1; j <= nsub; ++j) {
        /* fields at the time of x before this sub-step */
        double s = 0.5 + (double)(j - 1) * ds;
        /* first push after a change of dt*: (dt*_old + dt*_new) / 2 */
        double dtp = j == 1 ? 0.5 * (dt_old + dt_new) : dt_new;
        xi = grid_coord(prm, *x);
        if (!in_grid(prm, xi)) return 1;
        orc_lagrange(prm->order, s, LE, LB);
        if ((rc = tent(prm, f, 0, n, xi, LE, &Ep))) return rc;
        if ((rc = tent(prm, f, 1, n, xi, LB, &Bp))) return rc;
        /* work of E over the sub-step (App. B): q dt_p / 2 E . (v_before +
         * v_after); E has only a y component here */
        double vb = 0.0;
        if (step_work) vb = *py / sqrt(1.0 + ((*px * *px + *py * *py) + *pz * *pz));
        orc_boris(prm->qm, dtp, Ep, Bp, px, py, pz);
        if (step_work) {
            double ga = sqrt(1.0 + ((*px * *px + *py * *py) + *pz * *pz));
            *step_work += ((0.5 * prm->qm) * dtp * Ep) * (vb + *py / ga);
        }
        *x = advance_x(*x, dt_new, *px, *py, *pz);
    }
    /* a step is counted once all its sub-steps are done */
    lc->steps += 1;
    lc->sub_steps += (uint64_t)nsub;
    if (k > 0) lc->n_star += (uint64_t)nsub;  /* sub-steps with dt* < dt */
    lc->steps_by_k[k] += 1;
    lc->sub_steps_by_k[k] += (uint64_t)nsub;
    return 0;
}

static int levels_present(const orc_params *prm, const orc_fields *f,
                          int64_t n0, int32_t nsteps)
{
    if (f->mode != 0) return 1;
    return n0 - prm->order >= f->lev0 &&
           n0 + nsteps - 1 < f->lev0 + f->nlev;
}

int orc_push(const orc_params *prm, const orc_fields *f, int64_t np,
             double *x, double *px, double *py, double *pz,
             int8_t *k_old, uint8_t *status, int64_t n0, int32_t nsteps,
             const int8_t *forced_k, int8_t *k_trace, double *psi_trace,
             double *work, double *werr, const double *r0, double *rmax, double *gmax,
             const double *ai, double *emax, orc_counters *cnt, int32_t nthreads)
{
    if (!prm || !f || np < 0 || nsteps < 0) return -1;
    if (prm->order < 1 || prm->order > ORC_MAX_ORDER) return -1;
    if (prm->ncells < 2 || !(prm->dx > 0) || !(prm->dt > 0)) return -1;
    if (prm->k_max < 0 || prm->k_max > 12) return -1;
    if (f->mode == 1 && f->M <= 0) return -1;
    if (emax && (!ai || f->mode != 1 || !f->atab)) return -1;
    if (!levels_present(prm, f, n0, nsteps)) return -2;

    local_cnt total;
    memset(&total, 0, sizeof total);
    int bad = 0;

#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel num_threads(nt)
#endif
    {
        local_cnt lc;
        memset(&lc, 0, sizeof lc);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
        for (int64_t i = 0; i < np; ++i) {
            for (int32_t st = 0; st < nsteps; ++st) {
                int64_t tix = (int64_t)st * np + i;
                if (status[i] != ORC_LIVE) {
                    if (k_trace) k_trace[tix] = -1;
                    if (psi_trace) psi_trace[tix] = -1.0;
                    continue;
                }
                int32_t k = -1;
                double ratio = -1.0;
                int forced = forced_k ? (int)forced_k[tix] : -1;
                double g_start = sqrt(1.0 + ((px[i] * px[i] + py[i] * py[i]) + pz[i] * pz[i]));
                double sw = 0.0;
                int rc = one_step(prm, f, n0 + st, &x[i], &px[i], &py[i],
                                  &pz[i], &k_old[i], forced, &k, &ratio,
                                  (work || werr) ? &sw : NULL, &lc);
                if (k_trace) k_trace[tix] = (int8_t)k;
                if (psi_trace) psi_trace[tix] = ratio;
                if (rc == 0 && (work || werr)) {
                    /* a completed step: kinetic energy change against work */
                    double g_end = sqrt(1.0 + ((px[i] * px[i] + py[i] * py[i]) + pz[i] * pz[i]));
                    double d = fabs((g_end - g_start) - sw);
                    if (work) work[i] += sw;
                    if (werr && d > werr[i]) werr[i] = d;
                }
                if (rc == 0 && ((r0 && rmax) || gmax)) {
                    /* a completed step: dephasing error |R - R0| / R0, R = gamma -
                     * p_x (Sec. IV, Eq. (R error)), and the largest gamma */
                    double g_end = sqrt(1.0 + ((px[i] * px[i] + py[i] * py[i]) + pz[i] * pz[i]));
                    if (r0 && rmax) {
                        double dr = fabs((g_end - px[i]) - r0[i]) / r0[i];
                        if (dr > rmax[i]) rmax[i] = dr;
                    }
                    if (gmax && g_end > gmax[i]) gmax[i] = g_end;
                }
                if (rc == 0 && emax) {
                    /* energy error against gamma_th = 1 + (a - a_i)^2 / 2 at
                     * the phase of the momentum, which lags x by half of the
                     * step's last sub-step */
                    double g_end = sqrt(1.0 + ((px[i] * px[i] + py[i] * py[i]) + pz[i] * pz[i]));
                    double half = 0.5 * ldexp(1.0, -2 * k);          /* dt* / 2, in dt */
                    double tau = (double)(n0 + st + 1) - half;
                    double xp = x[i] - half * prm->dt * (px[i] / g_end);
                    double u = (xp - prm->x_origin) / prm->dx - 0.5;  /* E-node coordinate */
                    double m = (double)f->aE * tau + (double)f->bE * u + (double)f->cE;
                    double mf = floor(m);
                    int64_t j0 = (int64_t)mf % f->M;
                    if (j0 < 0) j0 += f->M;
                    int64_t j1 = j0 + 1 == f->M ? 0 : j0 + 1;
                    double a = f->atab[j0] + (m - mf) * (f->atab[j1] - f->atab[j0]);
                    double d = a - ai[i];
                    double g_th = 1.0 + 0.5 * (d * d);
                    double e = fabs(g_end - g_th) / g_th;
                    if (e > emax[i]) emax[i] = e;
                }
                if (rc == 1) {
                    status[i] = ORC_LOST;
                    lc.lost += 1;
                } else if (rc != 0) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
                    bad = 1;
                }
            }
        }
#ifdef _OPENMP
#pragma omp critical
#endif
        {
            total.steps += lc.steps;
            total.sub_steps += lc.sub_steps;
            total.n_star += lc.n_star;
            total.clamps += lc.clamps;
            total.lost += lc.lost;
            for (int k = 0; k < ORC_KHIST; ++k) {
                total.steps_by_k[k] += lc.steps_by_k[k];
                total.sub_steps_by_k[k] += lc.sub_steps_by_k[k];
            }
        }
    }
    if (cnt) {
        cnt->steps += total.steps;
        cnt->sub_steps += total.sub_steps;
        cnt->n_star += total.n_star;
        cnt->clamps += total.clamps;
        cnt->lost += total.lost;
        for (int k = 0; k < ORC_KHIST; ++k) {
            cnt->steps_by_k[k] += total.steps_by_k[k];
            cnt->sub_steps_by_k[k] += total.sub_steps_by_k[k];
        }
    }
    return bad ? -2 : 0;
}

int32_t orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
