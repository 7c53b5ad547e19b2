/*
 * oracle.h -- plain FP64 CPU reference of the sub-cycled Boris push.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product
 * (libpicsub and its Python binding) never calls it and shares no code,
 * header, table or helper with it.
 *
 * What it computes (Tangtartharakul, Chen & Arefiev, "Particle integrator
 * for particle-in-cell simulations of ultra-high intensity laser-plasma
 * interactions", arXiv:2102.10983):
 *   - Yee staggering of the 1D fields, Sec. III, Eqs. (Ey), (Bz);
 *   - temporal Lagrange interpolation of E and B, Sec. VI,
 *     Eqs. (lagrange1-2)..(lagrange2-3);
 *   - the tent (triangular) shape gather, Sec. III, Eqs. (Enp), (Bnp);
 *   - the relativistic Boris push, Sec. III, Eqs. (p)..(x);
 *   - adaptive sub-cycling with the Psi_max rotation criterion and the
 *     leapfrog-consistent transition push, Sec. IV and Algorithm 1;
 *   - the step counters N and N* of Sec. VII (delta_steps).
 *
 * Units are normalised: t in 1/omega, x in c/omega, p in m c, E and B in
 * m omega c / |e|; qm is the charge-to-mass ratio in electron units (-1
 * for an electron).
 *
 * Readings of passages that are ambiguous or garbled are listed in the
 * project design notes; the ones that shape this code:
 *   - a field level m holds E_y at t = m dt (nodes (i+1/2) dx) and B_z at
 *     t = (m+1/2) dt (nodes i dx);
 *   - x sits at integer multiples of dt; p lags x by half the current
 *     sub-step (Algorithm 1), so sub-step j of a step at level n uses the
 *     fields at relative time s_j = 1/2 + (j-1)/4^k, with
 *     s = (t - (n-1/2) dt) / dt;
 *   - the loop count of Algorithm 1 is dt / dt*_new = 4^k;
 *   - Psi for the decision uses B gathered at (x_n, s = 1/2) and gamma of
 *     the stored momentum;
 *   - a particle leaving the gatherable range is frozen and flagged.
 */
#ifndef PICSUB_ORACLE_H
#define PICSUB_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_ORDER 7
#define ORC_KHIST 16

/* status flags of a particle (same meaning as in the product library) */
#define ORC_LIVE 0
#define ORC_LOST 1 /* left the range where both tent nodes exist, or its
                     state (x, p) is not finite at the start of a step */

typedef struct {
    int32_t ncells;   /* number of E and of B nodes on the 1D grid */
    int32_t order;    /* temporal interpolation order p (1..ORC_MAX_ORDER) */
    int32_t k_max;    /* cap of the sub-cycling exponent k */
    int32_t pad_;
    double x_origin;  /* x of B node 0; E node i is at x_origin + (i+1/2) dx */
    double dx, dt;
    double qm;        /* charge / mass in electron units */
    double psi_max;   /* maximum rotation per sub-step, Sec. IV */
} orc_params;

/* Field source.  Level m: E at t = m dt, B at t = (m + 1/2) dt.
 * mode 0: explicit arrays E[(m - lev0) * ncells + i], same for B;
 * mode 1: lattice table, F = table[((a m + b i + c) mod M)].
 * atab (mode 1, may be NULL): the wave's vector potential a on the same
 * lattice (atab[j] at the phase of table[j]), for the energy error. */
typedef struct {
    int32_t mode;
    int32_t nlev;
    int64_t lev0;
    const double *E, *B;
    const double *table;
    int64_t M;
    int64_t aE, bE, cE, aB, bB, cB;
    const double *atab;
} orc_fields;

/* Steps are counted when all their sub-steps are done (a particle lost
 * in the middle of a step adds to `lost` only). */
typedef struct {
    uint64_t steps;          /* N: completed particle-steps of size dt */
    uint64_t sub_steps;      /* Boris sub-steps of completed steps */
    uint64_t n_star;         /* N*: those with dt* < dt (Sec. VII) */
    uint64_t clamps;         /* decisions that hit k_max unmet */
    uint64_t lost;           /* particles flagged ORC_LOST */
    uint64_t steps_by_k[ORC_KHIST];
    uint64_t sub_steps_by_k[ORC_KHIST];
} orc_counters;

/* Lagrange weights for order p at relative time s, Eqs. (lagrange2-2) and
 * (lagrange2-3): LE[j] multiplies E at level n+j-p, LB[j] multiplies B at
 * level n+j-p (time n+1/2+j-p).  Returns 0, or -1 on a bad order. */
int orc_lagrange(int32_t p, double s, double *LE, double *LB);

/* Field at a particle: temporal interpolation on the two tent nodes, then
 * the tent weights.  which = 0 for E_y, 1 for B_z.  Returns 0, -1 when the
 * node range is outside the grid, -2 when a level is missing. */
int orc_gather(const orc_params *prm, const orc_fields *f, int32_t which,
               int64_t n, double s, double x, double *out);

/* Sub-cycling exponent for one particle from psi0 = |Psi| at dt:
 * smallest k >= 0 with psi0 <= psi_max 4^k, capped at k_max.
 * *clamped is set when the cap was hit with the criterion unmet. */
int32_t orc_decide_k(double psi0, double psi_max, int32_t k_max,
                     int32_t *clamped);

/* One relativistic Boris momentum update, Eqs. (p)..(gamman), with the
 * geometry of the model problem (E along y, B along z). */
void orc_boris(double qm, double dtp, double E, double B,
               double *px, double *py, double *pz);

/* Advance np particles over nsteps steps of size dt starting at level n0
 * (x at n0 dt on entry, at (n0+nsteps) dt on exit).
 * work and werr (np each, may be NULL): after every completed step, the
 * work of E over its sub-steps (App. B: q dt_p / 2 E . (v_before +
 * v_after) per sub-step) is added to work[i], and werr[i] keeps the
 * largest |(gamma_end - gamma_start) - step work| (kinetic energy change
 * against work, in m c^2).
 * r0, rmax (np each, may be NULL): after every completed step rmax[i]
 * keeps the largest |R - r0[i]| / r0[i], R = gamma - p_x of the momentum
 * (the dephasing error of Sec. IV, Eq. (R error)); gmax (may be NULL) keeps
 * the largest gamma.
 * ai, emax (np each, may be NULL; need f->atab): after every completed
 * step emax[i] keeps the largest |gamma - gamma_th| / gamma_th (the energy
 * error of Sec. IV, Eq. (gamma error)), gamma_th = 1 + (a - ai[i])^2 / 2
 * (Eq. (theoretical gamma) for an electron that started at rest where
 * a = ai[i]) with a taken at the phase of the momentum: t_p = (n + 1) dt -
 * dt* / 2 and x(t_p) = x - v_x dt* / 2 (dt* of the step just completed), a
 * linear between lattice points.
 * k_old[i] < 0 means "no previous sub-step": the first transition push
 * then uses dt*_new.  forced_k ([nsteps][np], may be NULL) replaces the
 * decision; k_trace and psi_trace ([nsteps][np], may be NULL) record the
 * decision and psi0 / psi_max (-1 where the particle was not live).
 * nthreads <= 0 uses the OpenMP default.  Returns 0, -1 on bad arguments,
 * -2 when a needed field level is missing (nothing is advanced then). */
int orc_push(const orc_params *prm, const orc_fields *f, int64_t np,
             double *x, double *px, double *py, double *pz,
             int8_t *k_old, uint8_t *status, int64_t n0, int32_t nsteps,
             const int8_t *forced_k, int8_t *k_trace, double *psi_trace,
             double *work, double *werr, const double *r0, double *rmax, double *gmax,
             const double *ai, double *emax, orc_counters *cnt, int32_t nthreads);

/* number of OpenMP threads the library would use */
int32_t orc_max_threads(void);

#ifdef __cplusplus
}
#endif

#endif
