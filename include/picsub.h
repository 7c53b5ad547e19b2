/*
 * picsub.h -- C ABI of the MI355X sub-cycled Boris particle push.
 *
 * The library advances test electrons through prescribed 1D Yee-grid
 * fields with the relativistic Boris pusher, adaptive per-particle
 * sub-cycling (dt* = dt / 4^k, k from the Psi_max rotation criterion) and
 * order-p temporal Lagrange interpolation of E_y and B_z, following
 * Tangtartharakul, Chen & Arefiev, arXiv:2102.10983:
 *   Sec. III  Yee staggering (Eqs. (Ey), (Bz)), tent gather (Eqs. (Enp),
 *             (Bnp)) and the Boris push (Eqs. (p)..(x));
 *   Sec. IV   the Psi_max criterion, the leapfrog-consistent transition
 *             push and Algorithm 1 ("Sub-Cycling");
 *   Sec. VI   Lagrange interpolation during sub-cycling
 *             (Eqs. (lagrange1-2)..(lagrange2-3));
 *   Sec. VII  the step counters N and N* (delta_steps).
 *
 * Conventions
 *   Units: t in 1/omega, x in c/omega, p in m c, E and B in
 *   m omega c / |e|; qm = charge / mass in electron units (-1: electron).
 *   Field level m: E_y at t = m dt on nodes x_origin + (i + 1/2) dx and
 *   B_z at t = (m + 1/2) dt on nodes x_origin + i dx, i = 0..ncells-1.
 *   Particle state at step n: x at t = n dt; p at t = n dt - dt*_old / 2
 *   where dt*_old = dt / 4^k_old (k_old < 0: p lags x by half of the
 *   sub-step chosen at the next step, e.g. an electron at rest).
 *   Sub-step j (1..4^k) of the step at level n uses the fields at the
 *   time of x before that sub-step, s_j = 1/2 + (j-1) / 4^k in units of dt
 *   after (n - 1/2) dt; the first sub-step's momentum push uses
 *   (dt*_old + dt*_new) / 2 (Sec. IV).
 *
 * Ownership and errors
 *   Every call returns pic_status; nothing throws or aborts across the
 *   ABI.  pic_last_error() returns a message for the last failure on a
 *   context (the HIP error string for PIC_E_DEVICE).  The library owns the
 *   device state it allocates in pic_create; the caller owns every array it
 *   passes in or receives.  Work is enqueued on the stream given to
 *   pic_create; calls with PIC_MEM_HOST buffers synchronise that stream,
 *   calls with PIC_MEM_DEVICE buffers are asynchronous and the caller keeps
 *   the buffers valid until the stream has passed them.  A context is not
 *   thread-safe; distinct contexts are independent.  A particle whose
 *   tent nodes leave the grid is frozen and flagged PIC_PARTICLE_LOST; it
 *   is not an error.
 */
#ifndef PICSUB_H
#define PICSUB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PIC_OK = 0,
    PIC_E_ARG = 1,     /* invalid argument (null pointer, size, parameter) */
    PIC_E_DEVICE = 2,  /* a HIP call failed */
    PIC_E_NOMEM = 3,   /* device or host allocation failed */
    PIC_E_LEVEL = 4,   /* a field level the push needs is not in the ring */
    PIC_E_STATE = 5,   /* call out of order (e.g. push before particles) */
    PIC_E_NUMERIC = 6  /* strict mode (pic_strict_set): particle or field input
                          holds a value that is not finite */
} pic_status;

typedef enum { PIC_MEM_HOST = 0, PIC_MEM_DEVICE = 1 } pic_mem;

/* arithmetic of the push */
typedef enum {
    PIC_FP64 = 0,       /* IEEE FP64 in the operation order of the equations:
                           bit-identical to a plain scalar implementation */
    PIC_FP32_COMP = 1,  /* k = 0 steps in FP32: the Boris update (Sec. III)
                           formed as cancellation-free increments added to p
                           held as FP32 (hi, lo) pairs by TwoSum, x as node
                           index + FP32 fraction + carry; FP64 fields,
                           weights, decision (Sec. IV) and sub-cycled steps.
                           Within 1e-5 of FP64 except on electrons whose
                           trajectory is as sensitive as a 1e-10 relative
                           change of the initial position (a long ride
                           ending next to a stopping point) */
    PIC_FP64_FAST = 2   /* FP64 with fused multiply-adds, the hardware
                           reciprocal / rsqrt estimates refined by one Newton
                           step, positions in node units, 1/gamma reused by
                           the next decision, and the next step's field
                           window loaded into LDS one step ahead.  Not
                           bit-identical to PIC_FP64: rounding differences
                           grow along trajectories (observed up to 5e-7
                           relative on p, well inside 1e-5) */
} pic_precision;

/* how particles are grouped onto wavefronts for the sub-step loop */
typedef enum {
    PIC_BIN_NONE = 0,    /* one particle per lane, no regrouping */
    PIC_BIN_BALLOT = 1,  /* per-step compaction by k inside a workgroup */
    PIC_BIN_LEARNED = 2  /* the wavefront kernels of NONE; the caller re-bins
                            by predicted load with pic_prebin (below) */
} pic_binning;

#define PIC_PARTICLE_LIVE 0u
#define PIC_PARTICLE_LOST 1u   /* left the grid (its tent nodes are not all on
                                  it), or its x or p was not finite at the start
                                  of a step; frozen from then on */

#define PIC_KHIST 16
#define PIC_K_MAX_LIMIT 12

typedef struct {
    int32_t ncells;      /* nodes per field, >= 2 */
    int32_t order;       /* temporal interpolation order p: 1, 2, 3 or 5 */
    int32_t ring_depth;  /* stored levels, >= order + 1 */
    int32_t k_max;       /* cap of k, 0..PIC_K_MAX_LIMIT (the weight table holds
                            (4^(k_max+1) - 1) / 3 entries of 2 (order + 1)
                            doubles: 1.4 GB at k_max = 12, order 3) */
    int32_t precision;   /* pic_precision */
    int32_t binning;     /* pic_binning */
    double x_origin;     /* x of B node 0 */
    double dx;           /* cell size, > 0 */
    double dt;           /* time step, > 0 */
    double qm;           /* charge / mass, nonzero */
    double psi_max;      /* maximum rotation per sub-step, > 0 (Sec. IV) */
} pic_params;

typedef struct {
    uint64_t steps;       /* N: particle-steps of size dt taken */
    uint64_t sub_steps;   /* Boris sub-steps performed (sum of 4^k) */
    uint64_t n_star;      /* N*: sub-steps with dt* < dt (Sec. VII) */
    uint64_t clamps;      /* decisions that hit k_max unmet */
    uint64_t lost;        /* particles flagged lost */
    uint64_t steps_by_k[PIC_KHIST];
    uint64_t sub_steps_by_k[PIC_KHIST];
    uint64_t rebins;      /* group re-orderings made by an attached predictor
                             (pic_predictor_set), whole context.  There is no
                             count of mispredicted steps: the predictor ranks
                             groups by their expected load over the coming
                             launch instead of guessing each next step's k, so
                             no per-step prediction exists to be wrong; a poor
                             ranking shows as time only */
} pic_counters;

typedef struct pic_ctx pic_ctx;

/* Create a context for np particles with parameters *prm; all work goes
 * to hip_stream (a hipStream_t, NULL for the default stream) on the
 * current device.  Validates the parameters (PIC_E_ARG), allocates the
 * particle store, the field ring of prm->ring_depth levels and the table
 * of Lagrange weights for every (k, j) (Eqs. (lagrange2-2),
 * (lagrange2-3)).  On success *out owns the device memory. */
pic_status pic_create(const pic_params *prm, int64_t np, void *hip_stream,
                      pic_ctx **out);

/* Release everything a context owns (synchronises its stream). */
pic_status pic_destroy(pic_ctx *ctx);

/* Message for the last failure on ctx ("" if none); valid until the next
 * call on ctx. */
const char *pic_last_error(const pic_ctx *ctx);

/* Load the particle state: x, px, py, pz (np doubles each; may be NULL when
 * np == 0) and k_old (np int8; NULL means -1 for all), in the time
 * convention of Algorithm 1 (Sec. IV): x at t = n dt and p half the previous
 * sub-step behind, at n dt - dt*_old / 2 with dt*_old = dt / 4^k_old (the
 * leapfrog stagger of the Boris scheme, Sec. III).  Resets the status flags
 * and the counters.  Particles are reordered internally by position (cell
 * index); every per-particle output is returned in the caller's original
 * order.  A particle whose x or p is not finite is flagged
 * PIC_PARTICLE_LOST at its first step and never moved; in strict mode the
 * call returns PIC_E_NUMERIC instead and loads nothing. */
pic_status pic_particles_set(pic_ctx *ctx, pic_mem mem, const double *x,
                             const double *px, const double *py,
                             const double *pz, const int8_t *k_old);

/* Store field level n (Sec. III staggering): Ey[i] = E_y(x_origin +
 * (i + 1/2) dx, n dt), Bz[i] = B_z(x_origin + i dx, (n + 1/2) dt), ncells
 * doubles each, into ring slot n mod ring_depth. */
pic_status pic_fields_load(pic_ctx *ctx, int64_t n, pic_mem mem,
                           const double *Ey, const double *Bz);

/* Fill levels n_first .. n_first + count - 1 on the device from a phase
 * table: Ey[i] = table[(aE m + bE i + cE) mod M], Bz[i] = table[(aB m +
 * bB i + cB) mod M] for level m.  table is a device array of M doubles.
 * This samples prescribed fields ("perfectly propagating PIC", Sec. III)
 * without host traffic.  count <= ring_depth. */
pic_status pic_fields_load_lattice(pic_ctx *ctx, int64_t n_first,
                                   int32_t count, const double *table,
                                   int64_t M, int64_t aE, int64_t bE,
                                   int64_t cE, int64_t aB, int64_t bB,
                                   int64_t cB);

/* Standard PIC fields (Sec. III, Eqs. (Ey) and (Bz)): compute levels
 * n_first .. n_first + count - 1 with the 1D Yee scheme from level
 * n_first - 1, which must be in the ring (PIC_E_LEVEL otherwise), and
 * store each in its ring slot.  nu = dt / dx.  Boundaries (not given by
 * the paper; chosen here): the laser enters at node 0, where B_z of level
 * m is the incident wave table[(aB m + cB) mod M] (a hard source; table is
 * a device array of M doubles, as for pic_fields_load_lattice); the last E
 * node obeys the first-order Mur one-way condition with kappa =
 * (dt - dx) / (dt + dx).  IEEE arithmetic in the order of the equations:
 * the levels are bit-identical to a CPU loop.  count <= ring_depth - 1.
 * Asynchronous on the context's stream.  A typical run loads the levels
 * n0 - order .. n0 with pic_fields_load_lattice (or pic_fields_load) and
 * lets the solver make every later level. */
pic_status pic_fields_yee(pic_ctx *ctx, int64_t n_first, int32_t count,
                          const double *table, int64_t M, int64_t aB,
                          int64_t cB);

/* Copy ring level n of a run out (Ey, Bz: ncells doubles each, either may
 * be NULL; host or device memory; PIC_E_LEVEL if the ring does not hold
 * level n, and for runs in device-driven mode, whose ring is filled on the
 * device).  With PIC_MEM_HOST the call synchronises the stream. */
pic_status pic_fields_read(pic_ctx *ctx, int64_t n, pic_mem mem, double *Ey,
                           double *Bz);

/* Advance every live particle from x at n dt to (n + S) dt: S steps of
 * Algorithm 1 (Sec. IV) with order-p interpolation (Sec. VI).  Requires
 * levels n - order .. n + S - 1 in the ring (PIC_E_LEVEL otherwise, and
 * nothing is enqueued).  Asynchronous on the context's stream. */
pic_status pic_push_subcycled(pic_ctx *ctx, int64_t n, int32_t S);

/* Record the sub-cycling exponent k chosen at steps n_first ..
 * n_first + steps - 1 for the particles with caller index in
 * [first, first + count) into buf[(n - n_first) * count + (index - first)]
 * (device int8 array of steps * count entries owned by the caller; -1
 * where the particle was not live).  buf == NULL switches recording off.
 * Used to compare decisions and to collect training labels. */
pic_status pic_ktrace_set(pic_ctx *ctx, int8_t *buf, int64_t n_first,
                          int32_t steps, int64_t first, int64_t count);

/* Read the state: the Lorentz factor gamma = sqrt(1 + |p|^2) of the stored
 * momentum (Sec. III, Eq. (gamma); with p_x it gives the dephasing
 * invariant R = gamma - p_x of Sec. V, Eq. (R error)), p, x, the last k, the
 * status flags (np entries each, caller order; any pointer may be NULL) and
 * the counters (may be NULL): N and N* of Sec. VII (delta_steps), the steps
 * and sub-steps of each k, clamps and lost particles.  With PIC_MEM_HOST the
 * call synchronises the stream. */
pic_status pic_diag(pic_ctx *ctx, pic_mem mem, double *gamma, double *px,
                    double *py, double *pz, double *x, int8_t *k_last,
                    uint8_t *status, pic_counters *cnt);

/* pic_diag for one run of a batch: np[run] entries per output, in the
 * caller order of that run's particles, and the counters of that run. */
pic_status pic_diag_r(pic_ctx *ctx, int32_t run, pic_mem mem, double *gamma,
                      double *px, double *py, double *pz, double *x,
                      int8_t *k_last, uint8_t *status, pic_counters *cnt);

/* Strict mode (on != 0): pic_particles_set, pic_fields_load*,
 * pic_fields_yee* and pic_source_set check their particle arrays, levels or
 * phase table and return PIC_E_NUMERIC, loading nothing, if a value is not
 * finite (each check reads the whole input: a synchronising pass).  Off (the
 * default): non-finite particles are frozen and flagged as above. */
pic_status pic_strict_set(pic_ctx *ctx, int32_t on);

/* pic_diag with host outputs that allocates nothing, for callers that
 * cannot allocate device memory (serving loops, code that must not call
 * hipMalloc).  The same values as pic_diag(ctx, PIC_MEM_HOST, ...) (host
 * arrays, any pointer may be NULL), staged through a fixed array of the
 * library's own in each GPU's memory (about 64 MiB, held from the load of the
 * library until the process ends) instead of a per-call allocation.
 * PIC_E_ARG if the context holds more than PIC_DIAG_NOALLOC_MAX_NP
 * particles.  Synchronises the stream.  All calls on one GPU share that
 * array: calls that overlap on one GPU (other threads, other streams) race,
 * and callers must serialise them. */
#define PIC_DIAG_NOALLOC_MAX_NP 1572864
pic_status pic_diag_noalloc(pic_ctx *ctx, double *gamma, double *px, double *py, double *pz,
                            double *x, int8_t *k_last, uint8_t *status, pic_counters *cnt);

/* Move the grid of one run by `cells` nodes (positive: towards +x), for
 * particles that travel farther than a grid can hold (an electron riding a
 * pulse crosses ~10^6 cells, Sec. II): the run's x_origin becomes
 * x_origin0 + shift * dx in FP64, x_origin0 being the origin at creation and
 * shift the sum of all moves (written to *x_origin if not NULL).  Particle
 * positions are absolute and do not change; every ring level of the run is
 * dropped (load the levels the next push needs for the new nodes, e.g.
 * with lattice coefficients c + b * shift).  Not for runs in device-driven
 * mode (PIC_E_STATE).  Synchronises the stream. */
pic_status pic_grid_shift(pic_ctx *ctx, int32_t run, int64_t cells, double *x_origin);

/* Reset the counters to zero (asynchronous). */
pic_status pic_counters_reset(pic_ctx *ctx);

/* ------------------------------------------------------------------ */
/* Batches of independent runs.                                        */
/* ------------------------------------------------------------------ */

/* A context holding nruns independent runs, each with its own grid,
 * dt, psi_max, field ring (per_run[r]) and np[r] particles.  The runs
 * share order, precision and binning.  Caller particle arrays list the
 * runs' particles one run after the other (run 0 first).  pic_create is
 * the one-run case.  Calls without a run index act on every run (field
 * loads without an index act on run 0). */
pic_status pic_batch_create(const pic_params *per_run, const int64_t *np,
                            int32_t nruns, void *hip_stream, pic_ctx **out);

/* Field loads of one run (see pic_fields_load, pic_fields_load_lattice). */
pic_status pic_fields_load_r(pic_ctx *ctx, int32_t run, int64_t n, pic_mem mem,
                             const double *Ey, const double *Bz);
pic_status pic_fields_load_lattice_r(pic_ctx *ctx, int32_t run,
                                     int64_t n_first, int32_t count,
                                     const double *table, int64_t M,
                                     int64_t aE, int64_t bE, int64_t cE,
                                     int64_t aB, int64_t bB, int64_t cB);

/* Yee levels and level read-out for one run (see pic_fields_yee,
 * pic_fields_read). */
pic_status pic_fields_yee_r(pic_ctx *ctx, int32_t run, int64_t n_first,
                            int32_t count, const double *table, int64_t M,
                            int64_t aB, int64_t cB);
pic_status pic_fields_read_r(pic_ctx *ctx, int32_t run, int64_t n, pic_mem mem,
                             double *Ey, double *Bz);

/* Device-driven mode.  Attach a phase table (device array of M doubles,
 * coefficients as in pic_fields_load_lattice, kept valid by the caller)
 * to a run whose particles sit at level n_start and which stops at level
 * n_stop (INT64_MAX: never); the levels n_start - order .. n_start - 1
 * are sampled now.  From then on pic_advance moves every run on by S of
 * its own steps (fewer once it reaches n_stop): it samples the new levels
 * of each run on the device, pushes (Algorithm 1, Sec. IV) and moves the
 * run's level counter, all without host state, so windows can be captured
 * into a graph.  Requires a source on every run and S + order <=
 * ring_depth of every run. */
pic_status pic_source_set(pic_ctx *ctx, int32_t run, int64_t n_start,
                          int64_t n_stop, const double *table, int64_t M,
                          int64_t aE, int64_t bE, int64_t cE, int64_t aB,
                          int64_t bB, int64_t cB);
pic_status pic_advance(pic_ctx *ctx, int32_t S);

/* Level the run will have reached when the queued work is done. */
pic_status pic_run_level(const pic_ctx *ctx, int32_t run, int64_t *n);

/* Capture `windows` consecutive pic_advance(S) calls into a HIP graph
 * (replacing a previous one); pic_graph_launch replays it on the
 * context's stream, advancing every run by windows * S steps per launch.
 * The graph holds kernels only (no memset or copy nodes). */
pic_status pic_graph_capture(pic_ctx *ctx, int32_t S, int32_t windows);
pic_status pic_graph_launch(pic_ctx *ctx);
pic_status pic_graph_release(pic_ctx *ctx);

/* Counters of one run (synchronises the stream). */
pic_status pic_run_counters(pic_ctx *ctx, int32_t run, pic_counters *cnt);

/* ------------------------------------------------------------------
 * Trajectory diagnostics: the paper's two error measures, kept per
 * particle by every push kernel while switched on.
 *
 * Dephasing (Sec. V, Eq. (R error)): R = gamma - p_x of the stored
 * momentum is 1 for an electron that starts at rest in a plane wave in
 * vacuum and stays at its initial value R0 for any start (App. A), so the
 * running maximum of |R - R0| / R0 measures the integrator's error (the
 * paper's epsilon_dephasing when R0 = 1).
 *
 * Energy (App. B): the work of E over each sub-step, q dt_p / 2 E .
 * (v_before + v_after), summed from the start, and the largest
 * |(gamma_end - gamma_start) - work| over a single completed step (kinetic
 * energy in m c^2; the paper normalises it by |q| E0 dt).
 *
 * Peak energy (Sec. IV, Eq. (theoretical gamma)): the running maximum of
 * gamma after each completed step, to set against the analytic peak
 * 1 + a0^2 / 2 of an electron starting at rest.
 * ------------------------------------------------------------------ */

/* on = 1: (re)start: R0 := R of every particle now, the gamma maximum :=
 * gamma now, the other maxima and the work := 0;
 * from then on every push kernel updates them after each completed step
 * of a live particle (a few square roots and divisions per sub-step, IEEE
 * in the PIC_FP64 kernels, bit-identical to a CPU loop).  on = 0: stop
 * updating (the values are kept).  Loading particles restarts them (on or
 * off); re-binning (pic_prebin) carries them with the particles; the
 * autotuner's trials do not touch them; a captured graph keeps the setting
 * it was captured with; checkpoints do not include them.  The kernels
 * compile them in only while on. */
pic_status pic_diag_track(pic_ctx *ctx, int32_t on);

/* R0 and the running maximum of |R - R0| / R0 of every particle in caller
 * order (np doubles each, either may be NULL; host or device memory).
 * PIC_E_STATE if the diagnostics were never switched on.  With
 * PIC_MEM_HOST the call synchronises the stream. */
pic_status pic_dephasing_read(pic_ctx *ctx, pic_mem mem, double *R0,
                              double *rmax);

/* The work of E since the start and the largest single-step energy
 * mismatch of every particle, as pic_dephasing_read. */
pic_status pic_energy_read(pic_ctx *ctx, pic_mem mem, double *work,
                           double *err_max);

/* Order score from a k trace (a persistence control for the predictor;
 * ours): ktrace is a device int8 [steps][count] array as pic_ktrace_set
 * records it (k per step, -1 where a particle was not live); score (device,
 * count floats) gets, per column, log2 of the mean of 4^k over the live
 * steps, NaN for a column with none (the lightest for pic_prebin).
 * Asynchronous on hip_stream; PIC_E_ARG for null pointers or empty sizes. */
pic_status pic_ktrace_load(const int8_t *ktrace, int32_t steps, int64_t count, float *score,
                           void *hip_stream);

/* Measurement aid, not part of the method: the attainable FP64 vector FMA
 * rate.  Launches `blocks` workgroups of 256 lanes on hip_stream; each lane
 * runs 16 independent FMA chains of `iters` rounds (2 * 16 * iters flop per
 * lane) and writes one double to out (device, blocks * 256 doubles, owned
 * by the caller).  Asynchronous; PIC_E_ARG for a null out or non-positive
 * sizes. */
pic_status pic_fma_probe(double *out, int32_t blocks, int64_t iters, void *hip_stream);

/* The largest gamma of every particle since the diagnostics were (re)started
 * (np doubles, caller order), as pic_dephasing_read. */
pic_status pic_gamma_max_read(pic_ctx *ctx, pic_mem mem, double *gmax);

/* The energy error of Sec. IV, Eq. (gamma error): the running maximum over
 * completed steps of |gamma - gamma_th| / gamma_th, gamma_th = 1 + (a - a_i)^2 / 2
 * (Eq. (theoretical gamma): the plane-wave solution of an electron that started
 * at rest where the vector potential was a_i).  a is taken at the phase of the
 * momentum, which lags x by half of the step's last sub-step: time
 * (n + 1) dt - dt* / 2 and position x - v_x dt* / 2, with u = (x - x_origin)/dx - 1/2
 * its E-node coordinate; a is linear between the points of a potential table
 * on a phase lattice like the field table's: entry (A tau + B u + C) mod M at
 * time tau dt.  Computed by every push while the trajectory diagnostics are on.
 *
 * pic_gamma_error_lattice: the potential table of a run (atab: device, M
 * doubles, owned by the caller, kept alive while attached; strict mode checks
 * it is finite) and its lattice; a grid shift moves C by B per cell, so a
 * moving-grid caller sets the lattice again with its fields.  No reset of the
 * maxima.  A null atab detaches (that run's maxima stay as they are).
 * PIC_E_ARG for a bad run or M <= 0.
 *
 * pic_gamma_error_start: a_i of every particle (np doubles, caller order,
 * host or device, copied) and the maxima set to 0; needs particles loaded
 * and the diagnostics on (PIC_E_STATE otherwise).  New particles
 * (pic_particles_set) or pic_diag_track(ctx, 1) stop it until the next start.
 *
 * pic_gamma_error_read: the maxima (np doubles, caller order), as
 * pic_dephasing_read; PIC_E_ARG ("no such diagnostic") when not started. */
pic_status pic_gamma_error_lattice(pic_ctx *ctx, int32_t run, const double *atab, int64_t M,
                                   int64_t A, int64_t B, int64_t C);
pic_status pic_gamma_error_start(pic_ctx *ctx, pic_mem mem, const double *ai);
pic_status pic_gamma_error_read(pic_ctx *ctx, pic_mem mem, double *emax);

/* ------------------------------------------------------------------ */
/* Launch shape.  None of these knobs changes a result: every kernel    */
/* gives each particle the same arithmetic whichever lane runs it.      */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t waves_per_group; /* wavefront kernels: 1, 2 or 4 wavefronts
                                (64-particle groups) per workgroup */
    int32_t tile;            /* compaction kernel: particles per tile,
                                128, 256 or 512 */
    int32_t binning;         /* PIC_BIN_NONE (wavefront kernels) or
                                PIC_BIN_BALLOT (compaction kernel, FP64) */
    int32_t sort_sub;        /* position bins per cell of the load-time
                                sort, 1..256 (next pic_particles_set) */
    int32_t occupancy;       /* PIC_FP64_FAST at orders 1 to 3 with one
                                wavefront per workgroup: 0 = the compiler's
                                register budget, 5, 6 or 7 = a budget for
                                that many wavefronts per SIMD (at 6 and 7 a
                                few registers spill, reloaded on sub-cycled
                                steps); the same bits under every budget;
                                which is faster depends on the workload,
                                pic_autotune times them all */
} pic_tune;

pic_status pic_tune_set(pic_ctx *ctx, const pic_tune *t);
pic_status pic_tune_get(const pic_ctx *ctx, pic_tune *t);

/* Time `reps` device-driven windows of `steps` steps for each candidate
 * launch shape (1, 2, 4 wavefronts per workgroup; the 5-, 6- and 7-wavefront
 * register budgets with PIC_FP64_FAST at orders 1 to 3; compaction tiles of 128,
 * 256, 512 with PIC_FP64), restoring the state after every trial, and keep
 * the fastest.  Requires sources on all runs.  The winner is remembered
 * for the process under the configuration's signature (device, precision,
 * order, k_max, steps, sort_sub and every run's particle count, grid, ring
 * depth, dx, dt, psi_max, q/m and source coefficients; not the field
 * values): a later call with the same signature applies it without trials
 * (*ms_best is then the time measured when it was tuned).
 * pic_autotune_forget clears that memory. */
pic_status pic_autotune(pic_ctx *ctx, int32_t steps, int32_t reps,
                        pic_tune *best, double *ms_best);
pic_status pic_autotune_forget(void);

/* Number of 64-slot particle groups and the order in which the wavefront
 * kernels start them: order[i] is the group started i-th (a permutation;
 * NULL restores slot order).  Groups are runs' slots in position order,
 * 64 at a time; a predictor of the sub-cycling load can put heavy groups
 * first. */
int32_t pic_group_count(const pic_ctx *ctx);
pic_status pic_order_set(pic_ctx *ctx, const int32_t *order, pic_mem mem);

/* ------------------------------------------------------------------
 * Checkpoint (not part of the paper): the state the library owns and the
 * caller cannot rebuild — every particle's x, p, k_last and status (caller
 * order), the counters of every run and each run's device-driven level —
 * in one host buffer.  Field levels are not included: after an import the
 * caller loads the levels the next push needs (pic_fields_load*, or
 * pic_source_set with n_start = the returned level).
 * ------------------------------------------------------------------ */

/* buf == NULL: *bytes = the size needed.  Otherwise writes the checkpoint
 * into buf (host memory, *bytes at least that size; any alignment) and
 * sets *bytes to the size written.  Synchronises the stream. */
pic_status pic_state_export(pic_ctx *ctx, void *buf, size_t *bytes);

/* Restore a checkpoint written by pic_state_export from a context with
 * the same runs (particle counts, ncells, order; PIC_E_ARG otherwise):
 * particles (re-sorted by position), status flags and counters.  levels
 * (host array of nruns, may be NULL) receives each run's recorded
 * device-driven level.  The group order and priorities are reset.
 * Synchronises the stream. */
pic_status pic_state_import(pic_ctx *ctx, const void *buf, size_t bytes, int64_t *levels);

/* ------------------------------------------------------------------
 * Learned load predictor.
 *
 * Not part of the paper's method: the paper decides k from Psi alone
 * (Sec. III) and that decision is kept unchanged.  The predictor only
 * estimates, one step ahead, how many sub-steps each particle will take,
 * so that particles of similar load share a wavefront and the heaviest
 * wavefronts start first and issue at raised priority.  No result of the
 * push depends on it: a wrong prediction costs time, never accuracy.
 *
 * Network: 8 features -> 64 -> 64 -> 1, GELU (erf form) after the two
 * hidden layers, output = predicted log2 of the sub-steps taken over the
 * next steps.  Parameter vector (PIC_MLP_NPARAM floats or BF16 words), in
 * this order: W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3.
 * Features are standardised as (f - mean) * inv_std with norm =
 * {mean[8], inv_std[8]}.  Inference reads BF16 weights (round-to-nearest-even of the FP32
 * masters) and accumulates in FP32; training keeps FP32 masters and
 * computes gradients of the BF16-rounded forward (straight-through).
 * ------------------------------------------------------------------ */
#define PIC_MLP_FEATURES 8
#define PIC_MLP_HIDDEN 64
#define PIC_MLP_NPARAM 4801

/* Features of every particle at level n (n = -2^63: each run's level of
 * the device-driven mode, pic_run_level), written to feat[caller index *
 * 8] (device, FP32):
 *   |E_y| and |B_z| at the particle from level n-1, their backward
 *   differences with level n-2 divided by dt, gamma, p_x, |p_perp|, and
 *   log(a0) of the particle's run (run_a0: host array, one per run).
 * Spatial interpolation is linear, as in the gather.  Particles that are
 * lost get zeros.  Levels n-1 and n-2 must be in every run's ring
 * (PIC_E_LEVEL otherwise).  Synchronous. */
pic_status pic_features(pic_ctx *ctx, int64_t n, const float *run_a0, float *feat);

/* Forward pass over n feature rows (all device pointers, FP32 except the
 * BF16 weights); out[i] = network(feat[i]).  Enqueued on hip_stream
 * (NULL: the null stream); returns without synchronising. */
pic_status pic_mlp_forward(const uint16_t *w_bf16, const float *norm, const float *feat,
                           float *out, int64_t n, void *hip_stream);

/* Gradient of the mean squared error inv_total * sum_i (out_i - target_i)^2
 * with respect to the FP32 parameter vector w, accumulated (atomically)
 * into grad, and the loss into *loss; the caller zeroes both.  The forward
 * pass inside uses w rounded to BF16.  Several calls over slices of a
 * data set with the same inv_total = 1/total sum to the full gradient.
 * Device pointers; enqueued on hip_stream. */
pic_status pic_mlp_grad(const float *w, const float *norm, const float *feat, const float *target,
                        int64_t n, float inv_total, float *grad, float *loss, void *hip_stream);

/* One Adam update (Kingma and Ba, bias-corrected, step t >= 1) of n FP32
 * parameters in place; m and v are the moment buffers (start at zero).
 * Device pointers; enqueued on hip_stream. */
pic_status pic_mlp_adam(float *w, float *m, float *v, const float *grad, int32_t n, float lr,
                        float beta1, float beta2, float eps, int32_t t, void *hip_stream);

/* Re-bin the particles of every run by predicted load: score[caller
 * index] (device, FP32, larger = more sub-steps; NaN = lightest) is cut
 * into nbuckets buckets of the given width below the largest score, and
 * each run's slots are re-filled bucket by bucket (heaviest first), in
 * position order inside a bucket (the bins of the load-time sort).  Then the groups are started heaviest
 * first by the largest score of their lanes, cut into steps of the same
 * width (groups within one step keep their slot order, which keeps
 * co-running groups close in space), and the prio_groups heaviest issue
 * at raised priority.  Particles stay in their run;
 * results are unchanged.  Allowed while a graph is captured: the particle
 * arrays, the group order and the priorities are rewritten in place, so
 * the graph's next replay runs in the new order.  Synchronous. */
pic_status pic_prebin(pic_ctx *ctx, const float *score, int32_t nbuckets, float width,
                      int32_t prio_groups);

/* Attach the predictor to the context, so that the pushes order the work
 * themselves: before every every_M-th call of pic_push_subcycled (level n)
 * or pic_advance (each run's level), every particle is scored with the
 * network (pic_features, pic_mlp_forward) and the groups are re-ordered as
 * pic_prebin(score, 1 bucket, width) does; the counters' rebins field
 * counts these.  w_bf16: PIC_MLP_NPARAM BF16 words; norm: 2 *
 * PIC_MLP_FEATURES floats; run_a0: one a0 > 0 per run (host arrays,
 * copied).  The features need level n - 2 in the ring (always there for
 * order >= 2).  Each turn synchronises the stream; windows captured into a
 * graph run without it (they keep whatever order is current when they
 * run), and no turns are taken while a captured graph is held.
 * w_bf16 == NULL detaches.  Results never depend on it. */
pic_status pic_predictor_set(pic_ctx *ctx, const uint16_t *w_bf16, const float *norm,
                             const float *run_a0, float width, int32_t every_M);

#ifdef __cplusplus
}
#endif

#endif
