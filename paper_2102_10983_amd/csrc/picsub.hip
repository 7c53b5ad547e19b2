// picsub.hip -- MI355X (gfx950) implementation of the C ABI in picsub.h.
//
// Sub-cycled relativistic Boris push with order-p temporal Lagrange
// interpolation of E_y and B_z gathered from a 1D Yee grid
// (arXiv:2102.10983, Sec. III, Sec. IV with Algorithm 1, Sec. VI).
//
// Layout in HBM
//   particles: structure of arrays x, px, py, pz (double), k_old (int8),
//              status (uint8), user index (int32); slot order is sorted
//              by cell at load time;
//   fields:    ring of ring_depth levels, E[slot][ncells], B[slot][ncells];
//   weights:   table of L^E_j and L^B_j (Eqs. (lagrange2-2), (lagrange2-3))
//              for every (k, j), entry e = (4^k - 1)/3 + (j - 1), stride
//              2 (p + 1) doubles: L^E_0..L^E_p, L^B_0..L^B_p;
//   counters:  one slot of NCNT uint64 per workgroup of the persistent grid,
//              updated without atomics (a workgroup owns its slot and
//              launches are ordered on the stream).
//
// Floating point: built with -ffp-contract=off so that every product and
// sum is rounded on its own; divisions and square roots are the IEEE
// correctly rounded ones.  The FP64 path therefore evaluates the same
// expressions, in the same order, as a plain scalar implementation of the
// paper's equations.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "picsub.h"

namespace {

constexpr int NCNT = PIC_KHIST + 2;   // steps_by_k[16], clamps, lost
constexpr int CNT_CLAMPS = PIC_KHIST;
constexpr int CNT_LOST = PIC_KHIST + 1;

constexpr int64_t wtab_entries(int kmax)
{
    // sum_{k=0}^{kmax} 4^k
    return ((int64_t(1) << (2 * (kmax + 1))) - 1) / 3;
}

__host__ __device__ inline int64_t wtab_offset(int k)
{
    return ((int64_t(1) << (2 * k)) - 1) / 3;
}

__host__ __device__ inline int64_t mod_floor(int64_t a, int64_t m)
{
    int64_t r = a % m;
    return r < 0 ? r + m : r;
}

// ---------------------------------------------------------------------
// Weights table.  For sub-step j of a step with exponent k the fields are
// wanted at s = 1/2 + (j-1)/4^k (units of dt after (n - 1/2) dt).  The
// numerator product runs over k' ascending and is divided once by the
// integer denominator (exact for the dyadic s of k <= 7 at p = 3).
// ---------------------------------------------------------------------
__global__ void weights_kernel(double *__restrict__ w, int p, int kmax)
{
    const int64_t total = wtab_entries(kmax);
    const int stride = 2 * (p + 1);
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
         e += int64_t(gridDim.x) * blockDim.x) {
        int k = 0;
        while (k < kmax && e >= wtab_offset(k + 1)) ++k;
        const int64_t j = e - wtab_offset(k) + 1;
        const double s = 0.5 + double(j - 1) * ldexp(1.0, -2 * k);
        for (int a = 0; a <= p; ++a) {
            double numE = 1.0, numB = 1.0, den = 1.0;
            for (int b = 0; b <= p; ++b) {
                if (b == a) continue;
                numE = numE * ((double(p - b) - 0.5) + s);
                numB = numB * (double(p - b - 1) + s);
                den = den * double(a - b);
            }
            w[e * stride + a] = numE / den;
            w[e * stride + (p + 1) + a] = numB / den;
        }
    }
}

// ---------------------------------------------------------------------
// Field levels from a phase table (prescribed plane wave sampled on the
// Yee lattice).
// ---------------------------------------------------------------------
__global__ void lattice_kernel(double *__restrict__ ringE, double *__restrict__ ringB,
                               int D, int ncells, int64_t n_first, int count,
                               const double *__restrict__ table, int64_t M,
                               int64_t aE, int64_t bE, int64_t cE, int64_t aB,
                               int64_t bB, int64_t cB)
{
    const int64_t total = int64_t(count) * ncells;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int64_t m = n_first + t / ncells;
        const int64_t i = t % ncells;
        const int64_t slot = mod_floor(m, D);
        ringE[slot * ncells + i] = table[mod_floor(aE * m + bE * i + cE, M)];
        ringB[slot * ncells + i] = table[mod_floor(aB * m + bB * i + cB, M)];
    }
}

// ---------------------------------------------------------------------
// Particle load: scatter the caller's arrays into slot order.
// ---------------------------------------------------------------------
// Bucket = position in units of dx / SORT_SUB: particles with nearly the
// same position (for a cold beam, nearly the same phase history and hence
// the same sub-cycling history) end up in neighbouring lanes.
constexpr int SORT_SUB = 64;

__global__ void cell_key_kernel(const double *__restrict__ x, int64_t np, double x_origin,
                                double dx, int ncells, int32_t *__restrict__ key,
                                int32_t *__restrict__ hist)
{
    const int32_t nfine = ncells * SORT_SUB;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < np;
         i += int64_t(gridDim.x) * blockDim.x) {
        const double u = (x[i] - x_origin) / dx * double(SORT_SUB);
        int32_t c = nfine;   // bucket for anything outside the grid or NaN
        if (u >= 0.0 && u < double(nfine)) c = int32_t(u);
        key[i] = c;
        atomicAdd(&hist[c], 1);
    }
}

// Exclusive scan of nb counts by one workgroup of 1024 threads.
__global__ void scan_kernel(int32_t *__restrict__ hist, int nb)
{
    __shared__ int32_t part[1024];
    const int t = threadIdx.x;
    const int per = (nb + 1023) / 1024;
    const int lo = t * per, hi = min(nb, lo + per);
    int32_t s = 0;
    for (int i = lo; i < hi; ++i) s += hist[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int32_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int32_t run = part[t] - s;
    for (int i = lo; i < hi; ++i) {
        int32_t c = hist[i];
        hist[i] = run;
        run += c;
    }
}

// Scatter into cell order.  The order inside a cell is whatever the atomic
// cursors give; it changes no particle's arithmetic, only its lane.
__global__ void scatter_kernel(const int32_t *__restrict__ key, int64_t np,
                               int32_t *__restrict__ cursor, int32_t *__restrict__ perm)
{
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < np;
         i += int64_t(gridDim.x) * blockDim.x)
        perm[atomicAdd(&cursor[key[i]], 1)] = int32_t(i);
}

__global__ void gather_state_kernel(const int32_t *__restrict__ perm, int64_t np,
                                    const double *__restrict__ x, const double *__restrict__ px,
                                    const double *__restrict__ py, const double *__restrict__ pz,
                                    const int8_t *__restrict__ kold, double *__restrict__ sx,
                                    double *__restrict__ spx, double *__restrict__ spy,
                                    double *__restrict__ spz, int8_t *__restrict__ skold,
                                    uint8_t *__restrict__ sstatus)
{
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < np;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int32_t u = perm[i];
        sx[i] = x[u];
        spx[i] = px[u];
        spy[i] = py[u];
        spz[i] = pz[u];
        skold[i] = kold ? kold[u] : int8_t(-1);
        sstatus[i] = PIC_PARTICLE_LIVE;
    }
}

__global__ void diag_kernel(const int32_t *__restrict__ perm, int64_t np,
                            const double *__restrict__ sx, const double *__restrict__ spx,
                            const double *__restrict__ spy, const double *__restrict__ spz,
                            const int8_t *__restrict__ skold, const uint8_t *__restrict__ sst,
                            double *__restrict__ gamma, double *__restrict__ px,
                            double *__restrict__ py, double *__restrict__ pz,
                            double *__restrict__ x, int8_t *__restrict__ klast,
                            uint8_t *__restrict__ status)
{
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < np;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int32_t u = perm[i];
        const double a = spx[i], b = spy[i], c = spz[i];
        if (gamma) gamma[u] = sqrt(1.0 + ((a * a + b * b) + c * c));
        if (px) px[u] = a;
        if (py) py[u] = b;
        if (pz) pz[u] = c;
        if (x) x[u] = sx[i];
        if (klast) klast[u] = skold[i];
        if (status) status[u] = sst[i];
    }
}

// ---------------------------------------------------------------------
// The push.
// ---------------------------------------------------------------------
struct PushArgs {
    double *x, *px, *py, *pz;
    int8_t *kold;
    uint8_t *status;
    const int32_t *perm;
    const double *ringE, *ringB;
    const double *wtab;
    int8_t *ktrace;
    uint64_t *cnt;          // [gridDim.x][NCNT]
    int64_t np;
    int64_t n0;
    int64_t kt_n0;
    int64_t kt_first, kt_count;
    double x_origin, dx, dt, qm, psi_max;
    int32_t D, ncells, kmax, S, kt_steps;
};

// Temporal interpolation at node i (Eqs. (lagrange1-2), (lagrange1-3)),
// levels ascending, then the tent weights (Eqs. (Enp), (Bnp)).
template <int P>
__device__ __forceinline__ double tent_gather(const double *__restrict__ ring,
                                              const int64_t (&base)[P + 1], int i0, double w,
                                              const double *__restrict__ L)
{
    double f0 = L[0] * ring[base[0] + i0];
    double f1 = L[0] * ring[base[0] + i0 + 1];
#pragma unroll
    for (int j = 1; j <= P; ++j) {
        f0 = f0 + L[j] * ring[base[j] + i0];
        f1 = f1 + L[j] * ring[base[j] + i0 + 1];
    }
    return (1.0 - w) * f0 + w * f1;
}

// Boris momentum update (Sec. III, Eqs. (p)..(gamman)) for E along y and
// B along z.
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

template <int P>
__global__ void __launch_bounds__(256) push_fp64_kernel(PushArgs a)
{
    constexpr int STRIDE = 2 * (P + 1);
    uint32_t c_steps[PIC_K_MAX_LIMIT + 1];
#pragma unroll
    for (int k = 0; k <= PIC_K_MAX_LIMIT; ++k) c_steps[k] = 0;
    uint32_t c_clamps = 0, c_lost = 0;

    const double ncm1 = double(a.ncells - 1);
    const double c0 = 0.5 * a.qm * a.dt;

    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < a.np;
         i += int64_t(gridDim.x) * blockDim.x) {
        if (a.status[i] != PIC_PARTICLE_LIVE) {
            if (a.ktrace) {
                const int64_t u = a.perm[i] - a.kt_first;
                if (u >= 0 && u < a.kt_count)
                    for (int st = 0; st < a.S; ++st) {
                        const int64_t r = a.n0 + st - a.kt_n0;
                        if (r >= 0 && r < a.kt_steps) a.ktrace[r * a.kt_count + u] = -1;
                    }
            }
            continue;
        }
        double x = a.x[i], px = a.px[i], py = a.py[i], pz = a.pz[i];
        int kold = a.kold[i];
        int64_t kt_u = -1;   // column of this particle in the k trace
        if (a.ktrace) {
            const int64_t u = a.perm[i] - a.kt_first;
            if (u >= 0 && u < a.kt_count) kt_u = u;
        }
        uint8_t status = PIC_PARTICLE_LIVE;
        int st = 0;
        for (; st < a.S; ++st) {
            const int64_t n = a.n0 + st;
            int64_t baseE[P + 1], baseB[P + 1];
#pragma unroll
            for (int j = 0; j <= P; ++j) {
                const int64_t slot = mod_floor(n - P + j, a.D);
                baseE[j] = slot * a.ncells;
                baseB[j] = slot * a.ncells;
            }
            int8_t ktr = -1;
            double xi = (x - a.x_origin) / a.dx;
            if (!(xi >= 0.5 && xi < ncm1)) {
                status = PIC_PARTICLE_LOST;
                ++c_lost;
            } else {
                // decision: B at (x_n, s = 1/2), gamma of the stored p
                const double *W1 = a.wtab;   // entry (k = 0, j = 1): s = 1/2
                const double flB = floor(xi);
                const double Bd = tent_gather<P>(a.ringB, baseB, int(flB), xi - flB, W1 + P + 1);
                const double g0 = sqrt(1.0 + ((px * px + py * py) + pz * pz));
                const double psi0 = fabs(c0 * Bd) / g0;
                int k = 0;
                double lim = a.psi_max;
                while (psi0 > lim && k < a.kmax) {
                    ++k;
                    lim = lim * 4.0;
                }
                c_clamps += psi0 > lim;
                ktr = int8_t(k);
                const int ko = kold < 0 ? k : kold;
                kold = k;
                const double dt_new = ldexp(a.dt, -2 * k);
                const double dt_old = ldexp(a.dt, -2 * ko);
                const int nsub = 1 << (2 * k);
                const double *W = a.wtab + wtab_offset(k) * STRIDE;
                bool done = true;
                for (int j = 1; j <= nsub; ++j, W += STRIDE) {
                    double B;
                    if (j == 1) {
                        B = Bd;
                    } else {
                        xi = (x - a.x_origin) / a.dx;
                        if (!(xi >= 0.5 && xi < ncm1)) {
                            done = false;
                            break;
                        }
                        const double fl = floor(xi);
                        B = tent_gather<P>(a.ringB, baseB, int(fl), xi - fl, W + P + 1);
                    }
                    const double uE = xi - 0.5;
                    const double flE = floor(uE);
                    const double E = tent_gather<P>(a.ringE, baseE, int(flE), uE - flE, W);
                    const double dtp = j == 1 ? 0.5 * (dt_old + dt_new) : dt_new;
                    boris(a.qm, dtp, E, B, px, py, pz);
                    const double g2 = sqrt(1.0 + ((px * px + py * py) + pz * pz));
                    x = x + dt_new * (px / g2);
                }
                if (done) {
#pragma unroll
                    for (int kk = 0; kk <= PIC_K_MAX_LIMIT; ++kk) c_steps[kk] += (k == kk);
                } else {
                    status = PIC_PARTICLE_LOST;
                    ++c_lost;
                }
            }
            if (kt_u >= 0) {
                const int64_t r = n - a.kt_n0;
                if (r >= 0 && r < a.kt_steps) a.ktrace[r * a.kt_count + kt_u] = ktr;
            }
            if (status != PIC_PARTICLE_LIVE) {
                ++st;
                break;
            }
        }
        if (kt_u >= 0)
            for (; st < a.S; ++st) {
                const int64_t r = a.n0 + st - a.kt_n0;
                if (r >= 0 && r < a.kt_steps) a.ktrace[r * a.kt_count + kt_u] = -1;
            }
        a.x[i] = x;
        a.px[i] = px;
        a.py[i] = py;
        a.pz[i] = pz;
        a.kold[i] = int8_t(kold);
        a.status[i] = status;
    }

    // workgroup reduction of the counters into this workgroup's slot
    __shared__ uint32_t red[NCNT];
    for (int c = threadIdx.x; c < NCNT; c += blockDim.x) red[c] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k <= PIC_K_MAX_LIMIT; ++k)
        if (c_steps[k]) atomicAdd(&red[k], c_steps[k]);
    if (c_clamps) atomicAdd(&red[CNT_CLAMPS], c_clamps);
    if (c_lost) atomicAdd(&red[CNT_LOST], c_lost);
    __syncthreads();
    for (int c = threadIdx.x; c < NCNT; c += blockDim.x)
        a.cnt[int64_t(blockIdx.x) * NCNT + c] += red[c];
}

// ---------------------------------------------------------------------
// Tiled push with per-step compaction by k (PIC_BIN_BALLOT).
//
// A workgroup of TILE threads owns TILE consecutive particle slots (one
// per thread) for all S steps of a launch.  Per step:
//   1. the node window [lo, hi] its particles can touch during the step
//      (a particle moves less than one cell per dt) is reduced over the
//      workgroup and the P+1 levels of E and B on it are staged in LDS,
//      together with B interpolated to s = 1/2 (the decision's field and
//      the field of every k = 0 step);
//   2. every thread takes the decision for its particle; k = 0 particles
//      do their single sub-step in place;
//   3. sub-cycled particles leave their state in LDS and are appended to a
//      per-k queue with a ballot and a lane rank (mbcnt), so that each
//      queue is a dense list; full 64-lane chunks of one k are then run by
//      the workgroup's wavefronts, heaviest k first, with wave-uniform
//      weights;
//   4. owners pick their updated state back up.
// Every particle sees exactly the arithmetic of the one-lane-per-particle
// kernel; only which lane does it changes.
// ---------------------------------------------------------------------
constexpr int TILE = 256;
constexpr int WMAX = 256;        // staged nodes per field level

struct TileArgs {
    double *x, *px, *py, *pz;
    int8_t *kold;
    uint8_t *status;
    const int32_t *perm;
    const double *ringE, *ringB;
    const double *wtab;
    int8_t *ktrace;
    uint64_t *cnt;
    int64_t np;
    int64_t n0;
    int64_t kt_n0, kt_first, kt_count;
    double x_origin, dx, dt, qm, psi_max;
    int32_t D, ncells, kmax, S, kt_steps;
    int32_t slot0;               // ring slot of level n0 - P
    int32_t margin;              // cells a particle can cross in one dt, + 2
};

template <int P>
struct Levels {
    // element offsets of the P+1 levels needed at one step, in the ring
    int32_t off[P + 1];
    __device__ __forceinline__ void at(const TileArgs &a, int st)
    {
#pragma unroll
        for (int j = 0; j <= P; ++j) {
            int s = a.slot0 + st + j;
            s = s >= a.D ? s - a.D : s;
            s = s >= a.D ? s - a.D : s;
            off[j] = s * a.ncells;
        }
    }
};

// node value sum_j L_j F_j[i] from a view with level stride `ls`
template <int P, typename T>
__device__ __forceinline__ double node_comb(const T *__restrict__ f, const int32_t (&lo)[P + 1],
                                            int i, const double *__restrict__ L)
{
    double v = L[0] * f[lo[0] + i];
#pragma unroll
    for (int j = 1; j <= P; ++j) v = v + L[j] * f[lo[j] + i];
    return v;
}

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

__device__ __forceinline__ void flush_counts(Counts &c, uint64_t *__restrict__ slot)
{
    __shared__ uint32_t red[NCNT];
    for (int i = threadIdx.x; i < NCNT; i += blockDim.x) red[i] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k <= PIC_K_MAX_LIMIT; ++k)
        if (c.steps[k]) atomicAdd(&red[k], c.steps[k]);
    if (c.clamps) atomicAdd(&red[CNT_CLAMPS], c.clamps);
    if (c.lost) atomicAdd(&red[CNT_LOST], c.lost);
    __syncthreads();
    for (int i = threadIdx.x; i < NCNT; i += blockDim.x) slot[i] += red[i];
}

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

template <int P>
__global__ void __launch_bounds__(TILE) push_tile_kernel(TileArgs a)
{
    constexpr int STRIDE = 2 * (P + 1);
    __shared__ double sE[(P + 1) * WMAX];    // raw E levels on the window
    __shared__ double sB[(P + 1) * WMAX];    // raw B levels on the window
    __shared__ double sBh[WMAX];             // B at s = 1/2 on the window
    __shared__ double sx[TILE], spx[TILE], spy[TILE], spz[TILE];
    __shared__ uint8_t sst[TILE];
    __shared__ uint16_t sq[PIC_K_MAX_LIMIT + 1][TILE];
    __shared__ int sqn[PIC_K_MAX_LIMIT + 1];
    __shared__ int slo[2], shi[2];   // window bounds, double-buffered by step parity

    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    constexpr int NWAVE = TILE / 64;
    const double ncm1 = double(a.ncells - 1);
    const double c0 = 0.5 * a.qm * a.dt;
    const double *W1 = a.wtab;                 // (k = 0, j = 1): s = 1/2
    Counts cnt;
    cnt.zero();

    if (t <= PIC_K_MAX_LIMIT) sqn[t] = 0;
    if (t < 2) {
        slo[t] = INT_MAX;
        shi[t] = INT_MIN;
    }

    for (int64_t tile0 = int64_t(blockIdx.x) * TILE; tile0 < a.np;
         tile0 += int64_t(gridDim.x) * TILE) {
        const int64_t i = tile0 + t;
        const bool mine = i < a.np;
        double x = 0, px = 0, py = 0, pz = 0;
        int kold = 0;
        uint8_t status = PIC_PARTICLE_LOST;
        int64_t kt_u = -1;
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
        __syncthreads();     // previous tile's LDS use is over

        for (int st = 0; st < a.S; ++st) {
            Levels<P> lv;
            lv.at(a, st);
            // -- 1. window of nodes this tile may touch during the step
            double xi = (x - a.x_origin) / a.dx;
            bool live = status == PIC_PARTICLE_LIVE && xi >= 0.5 && xi < ncm1;
            if (status == PIC_PARTICLE_LIVE && !live) {
                status = PIC_PARTICLE_LOST;
                ++cnt.lost;
                if (kt_u >= 0) {
                    const int64_t r = a.n0 + st - a.kt_n0;
                    if (r >= 0 && r < a.kt_steps) a.ktrace[r * a.kt_count + kt_u] = -1;
                }
            } else if (!live && kt_u >= 0) {
                const int64_t r = a.n0 + st - a.kt_n0;
                if (r >= 0 && r < a.kt_steps) a.ktrace[r * a.kt_count + kt_u] = -1;
            }
            const int par = st & 1;
            const int cell = live ? int(floor(xi)) : 0;
            int wlo = wave_min(live ? cell - a.margin : INT_MAX);
            int whi = wave_max(live ? cell + a.margin : INT_MIN);
            if (lane == 0 && wlo <= whi) {
                atomicMin(&slo[par], wlo);
                atomicMax(&shi[par], whi);
            }
            __syncthreads();
            const int lo = max(slo[par], 0);
            const int hi = min(shi[par], a.ncells - 1);
            const bool any = slo[par] <= shi[par];
            const bool use_lds = any && hi - lo + 1 <= WMAX;
            // -- stage the window
            if (use_lds) {
                for (int q = t; q <= hi - lo; q += TILE) {
                    double bh = 0;
#pragma unroll
                    for (int j = 0; j <= P; ++j) {
                        const double e = a.ringE[lv.off[j] + lo + q];
                        const double b = a.ringB[lv.off[j] + lo + q];
                        sE[j * WMAX + q] = e;
                        sB[j * WMAX + q] = b;
                        bh = j == 0 ? W1[P + 1] * b : bh + W1[P + 1 + j] * b;
                    }
                    sBh[q] = bh;
                }
            }
            __syncthreads();
            // this parity's bounds are read by everyone; the next writes to
            // them come two steps on, after the next step's first barrier
            if (t == 0) {
                slo[par] = INT_MAX;
                shi[par] = INT_MIN;
            }
            if (!any) continue;     // uniform: nothing live in this tile

            int32_t vo[P + 1];       // LDS level offsets shifted by the window base
#pragma unroll
            for (int j = 0; j <= P; ++j) vo[j] = j * WMAX - lo;

            // -- 2. decision, k = 0 steps in place
            bool heavy = false;
            int k = 0;
            if (live) {
                const double flB = floor(xi);
                const int iB = int(flB);
                const double wB = xi - flB;
                double f0, f1;
                if (use_lds) {
                    f0 = sBh[iB - lo];
                    f1 = sBh[iB + 1 - lo];
                } else {
                    f0 = node_comb<P>(a.ringB, lv.off, iB, W1 + P + 1);
                    f1 = node_comb<P>(a.ringB, lv.off, iB + 1, W1 + P + 1);
                }
                const double Bd = (1.0 - wB) * f0 + wB * f1;
                const double g0 = sqrt(1.0 + ((px * px + py * py) + pz * pz));
                const double psi0 = fabs(c0 * Bd) / g0;
                double lim = a.psi_max;
                while (psi0 > lim && k < a.kmax) {
                    ++k;
                    lim = lim * 4.0;
                }
                cnt.clamps += psi0 > lim;
                if (kt_u >= 0) {
                    const int64_t r = a.n0 + st - a.kt_n0;
                    if (r >= 0 && r < a.kt_steps) a.ktrace[r * a.kt_count + kt_u] = int8_t(k);
                }
                const int ko = kold < 0 ? k : kold;
                kold = k;
                if (k == 0) {
                    const double uE = xi - 0.5;
                    const double flE = floor(uE);
                    const int iE = int(flE);
                    const double wE = uE - flE;
                    // s = 1/2 is the time of level n: E's weights are
                    // (0, .., 0, 1), so the node values are level n's
                    double e0, e1;
                    if (use_lds) {
                        e0 = sE[vo[P] + iE];
                        e1 = sE[vo[P] + iE + 1];
                    } else {
                        e0 = a.ringE[lv.off[P] + iE];
                        e1 = a.ringE[lv.off[P] + iE + 1];
                    }
                    const double E = (1.0 - wE) * e0 + wE * e1;
                    const double dto = ldexp(a.dt, -2 * ko);
                    boris(a.qm, 0.5 * (dto + a.dt), E, Bd, px, py, pz);
                    const double g2 = sqrt(1.0 + ((px * px + py * py) + pz * pz));
                    x = x + a.dt * (px / g2);
                    cnt.step_done(0);
                } else {
                    heavy = true;
                    // remember dt*_old through the LDS state: pack it in kold
                    sx[t] = x;
                    spx[t] = px;
                    spy[t] = py;
                    spz[t] = pz;
                    sst[t] = uint8_t(ko);
                }
            }
            // -- 3. per-k queues: ballot + lane rank
            if (__syncthreads_or(heavy)) {
                for (int kk = 1; kk <= a.kmax; ++kk) {
                    const uint64_t m = __ballot(heavy && k == kk);
                    if (m) {
                        int base = 0;
                        if (lane == 0) base = atomicAdd(&sqn[kk], __popcll(m));
                        base = __shfl(base, 0);
                        if (heavy && k == kk) {
                            const uint32_t below =
                                __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32),
                                                          __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
                            sq[kk][base + below] = uint16_t(t);
                        }
                    }
                }
                __syncthreads();
                // chunks ordered by k descending; wave w takes every NWAVE-th
                int total = 0;
                for (int kk = a.kmax; kk >= 1; --kk) total += (sqn[kk] + 63) >> 6;
                for (int g = wave; g < total; g += NWAVE) {
                    int kk = a.kmax, c = g;
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
                    const double dt_new = ldexp(a.dt, -2 * kk);
                    const double dt_old = ldexp(a.dt, -2 * ko);
                    const int nsub = 1 << (2 * kk);
                    const double *Wk = a.wtab + wtab_offset(kk) * STRIDE;
                    uint8_t hst = PIC_PARTICLE_LIVE;
                    for (int j = 1; j <= nsub; ++j, Wk += STRIDE) {
                        const double hxi = (hx - a.x_origin) / a.dx;
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
                            b0 = node_comb<P>(a.ringB, lv.off, iB, Wk + P + 1);
                            b1 = node_comb<P>(a.ringB, lv.off, iB + 1, Wk + P + 1);
                            e0 = node_comb<P>(a.ringE, lv.off, iE, Wk);
                            e1 = node_comb<P>(a.ringE, lv.off, iE + 1, Wk);
                        }
                        const double B = (1.0 - wB) * b0 + wB * b1;
                        const double E = (1.0 - wE) * e0 + wE * e1;
                        const double dtp = j == 1 ? 0.5 * (dt_old + dt_new) : dt_new;
                        boris(a.qm, dtp, E, B, hpx, hpy, hpz);
                        const double g2 = sqrt(1.0 + ((hpx * hpx + hpy * hpy) + hpz * hpz));
                        hx = hx + dt_new * (hpx / g2);
                    }
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
                    } else {
                        status = PIC_PARTICLE_LOST;
                        ++cnt.lost;
                    }
                }
                if (t <= PIC_K_MAX_LIMIT) sqn[t] = 0;
                // the next step's first barrier orders these resets before
                // any new enqueue
            }
        }
        if (mine) {
            a.x[i] = x;
            a.px[i] = px;
            a.py[i] = py;
            a.pz[i] = pz;
            a.kold[i] = int8_t(kold);
            a.status[i] = status;
        }
    }
    flush_counts(cnt, a.cnt + int64_t(blockIdx.x) * NCNT);
}

// ---------------------------------------------------------------------
// Asynchronous wavefront push.
//
// One wavefront per workgroup and one workgroup per group of 64
// consecutive particle slots, carried through all S steps of the launch;
// the dispatcher starts a new workgroup wherever one retires, so no
// particle ever waits for another wavefront: a particle that sub-cycles
// deeply holds up only its own group while every other wavefront keeps
// advancing (the steps' field levels are all resident in the ring).
// Slots are sorted by position at load, so the 64 lanes of a group hold
// electrons with nearly the same phase history and mostly choose the same
// k.  Per step the group's node window is staged in the wavefront's own
// LDS (raw levels plus B at s = 1/2).  The arithmetic of every particle
// is that of the other push kernels.
// ---------------------------------------------------------------------

__device__ __forceinline__ void flush_counts_atomic(Counts &c, uint64_t *__restrict__ slot)
{
    __shared__ uint32_t red[NCNT];
    for (int i = threadIdx.x; i < NCNT; i += blockDim.x) red[i] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k <= PIC_K_MAX_LIMIT; ++k)
        if (c.steps[k]) atomicAdd(&red[k], c.steps[k]);
    if (c.clamps) atomicAdd(&red[CNT_CLAMPS], c.clamps);
    if (c.lost) atomicAdd(&red[CNT_LOST], c.lost);
    __syncthreads();
    for (int i = threadIdx.x; i < NCNT; i += blockDim.x)
        if (red[i]) atomicAdd(reinterpret_cast<unsigned long long *>(slot + i),
                              static_cast<unsigned long long>(red[i]));
}

constexpr int WWIN = 64;         // staged nodes per level in a wavefront window

struct WaveArgs {
    double *x, *px, *py, *pz;
    int8_t *kold;
    uint8_t *status;
    const int32_t *perm;
    const double *ringE, *ringB;
    const double *wtab;
    int8_t *ktrace;
    uint64_t *cnt;               // nslot counter slots, shared through atomics
    int32_t nslot;
    int64_t np;
    int64_t n0;
    int64_t kt_n0, kt_first, kt_count;
    double x_origin, dx, dt, qm, psi_max;
    int32_t D, ncells, kmax, S, kt_steps;
    int32_t slot0;
    int32_t margin;
};

template <int P>
struct WaveLevels {
    int32_t off[P + 1];
    __device__ __forceinline__ void at(const WaveArgs &a, int st)
    {
#pragma unroll
        for (int j = 0; j <= P; ++j) {
            int s = a.slot0 + st + j;
            s = s >= a.D ? s - a.D : s;
            s = s >= a.D ? s - a.D : s;
            off[j] = s * a.ncells;
        }
    }
};

template <int P>
__global__ void __launch_bounds__(64) push_wave_kernel(WaveArgs a)
{
    constexpr int STRIDE = 2 * (P + 1);
    __shared__ double sE[(P + 1) * WWIN];
    __shared__ double sB[(P + 1) * WWIN];
    __shared__ double sBh[WWIN];
    const int lane = threadIdx.x;
    const double ncm1 = double(a.ncells - 1);
    const double c0 = 0.5 * a.qm * a.dt;
    const double *W1 = a.wtab;
    Counts cnt;
    cnt.zero();
    {
        const int64_t i = int64_t(blockIdx.x) * 64 + lane;
        const bool mine = i < a.np;
        double x = 0, px = 0, py = 0, pz = 0;
        int kold = 0;
        uint8_t status = PIC_PARTICLE_LOST;
        int64_t kt_u = -1;
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
        for (int st = 0; st < a.S; ++st) {
            WaveLevels<P> lv;
            lv.at(a, st);
            double xi = (x - a.x_origin) / a.dx;
            const bool live = status == PIC_PARTICLE_LIVE && xi >= 0.5 && xi < ncm1;
            if (status == PIC_PARTICLE_LIVE && !live) {
                status = PIC_PARTICLE_LOST;
                ++cnt.lost;
            }
            if (!live && kt_u >= 0) {
                const int64_t r = a.n0 + st - a.kt_n0;
                if (r >= 0 && r < a.kt_steps) a.ktrace[r * a.kt_count + kt_u] = -1;
            }
            if (!__any(live)) {          // wave-uniform: the group is done
                if (kt_u >= 0)
                    for (int s2 = st + 1; s2 < a.S; ++s2) {
                        const int64_t r = a.n0 + s2 - a.kt_n0;
                        if (r >= 0 && r < a.kt_steps) a.ktrace[r * a.kt_count + kt_u] = -1;
                    }
                break;
            }
            const int cell = live ? int(floor(xi)) : 0;
            const int lo = max(wave_min(live ? cell - a.margin : INT_MAX), 0);
            const int hi = min(wave_max(live ? cell + a.margin : INT_MIN), a.ncells - 1);
            const bool use_lds = hi - lo + 1 <= WWIN;
            if (use_lds) {
                __syncthreads();          // one wavefront: orders the previous step's reads
                for (int q = lane; q <= hi - lo; q += 64) {
                    double bh = 0;
#pragma unroll
                    for (int j = 0; j <= P; ++j) {
                        const double e = a.ringE[lv.off[j] + lo + q];
                        const double b = a.ringB[lv.off[j] + lo + q];
                        sE[j * WWIN + q] = e;
                        sB[j * WWIN + q] = b;
                        bh = j == 0 ? W1[P + 1] * b : bh + W1[P + 1 + j] * b;
                    }
                    sBh[q] = bh;
                }
                __syncthreads();
            }
            int32_t vo[P + 1];
#pragma unroll
            for (int j = 0; j <= P; ++j) vo[j] = j * WWIN - lo;
            if (!live) continue;

            // decision: B at (x_n, s = 1/2), gamma of the stored momentum
            const double flB = floor(xi);
            const int iB = int(flB);
            const double wB = xi - flB;
            double f0, f1;
            if (use_lds) {
                f0 = sBh[iB - lo];
                f1 = sBh[iB + 1 - lo];
            } else {
                f0 = node_comb<P>(a.ringB, lv.off, iB, W1 + P + 1);
                f1 = node_comb<P>(a.ringB, lv.off, iB + 1, W1 + P + 1);
            }
            const double Bd = (1.0 - wB) * f0 + wB * f1;
            const double g0 = sqrt(1.0 + ((px * px + py * py) + pz * pz));
            const double psi0 = fabs(c0 * Bd) / g0;
            int k = 0;
            double lim = a.psi_max;
            while (psi0 > lim && k < a.kmax) {
                ++k;
                lim = lim * 4.0;
            }
            cnt.clamps += psi0 > lim;
            if (kt_u >= 0) {
                const int64_t r = a.n0 + st - a.kt_n0;
                if (r >= 0 && r < a.kt_steps) a.ktrace[r * a.kt_count + kt_u] = int8_t(k);
            }
            const int ko = kold < 0 ? k : kold;
            kold = k;
            const double dt_new = ldexp(a.dt, -2 * k);
            const double dt_old = ldexp(a.dt, -2 * ko);
            const int nsub = 1 << (2 * k);
            const double *Wk = a.wtab + wtab_offset(k) * STRIDE;
            bool done = true;
            for (int j = 1; j <= nsub; ++j, Wk += STRIDE) {
                double B, E;
                if (j == 1) {
                    // s = 1/2: B is the decision's, E's weights pick level n
                    B = Bd;
                    const double uE = xi - 0.5;
                    const double flE = floor(uE);
                    const int iE = int(flE);
                    const double wE = uE - flE;
                    double e0, e1;
                    if (use_lds) {
                        e0 = sE[vo[P] + iE];
                        e1 = sE[vo[P] + iE + 1];
                    } else {
                        e0 = a.ringE[lv.off[P] + iE];
                        e1 = a.ringE[lv.off[P] + iE + 1];
                    }
                    E = (1.0 - wE) * e0 + wE * e1;
                } else {
                    xi = (x - a.x_origin) / a.dx;
                    if (!(xi >= 0.5 && xi < ncm1)) {
                        done = false;
                        break;
                    }
                    const double fl = floor(xi);
                    const int ib = int(fl);
                    const double wb = xi - fl;
                    const double uE = xi - 0.5;
                    const double flE = floor(uE);
                    const int iE = int(flE);
                    const double wE = uE - flE;
                    double b0, b1, e0, e1;
                    if (use_lds) {
                        b0 = node_comb<P>(sB, vo, ib, Wk + P + 1);
                        b1 = node_comb<P>(sB, vo, ib + 1, Wk + P + 1);
                        e0 = node_comb<P>(sE, vo, iE, Wk);
                        e1 = node_comb<P>(sE, vo, iE + 1, Wk);
                    } else {
                        b0 = node_comb<P>(a.ringB, lv.off, ib, Wk + P + 1);
                        b1 = node_comb<P>(a.ringB, lv.off, ib + 1, Wk + P + 1);
                        e0 = node_comb<P>(a.ringE, lv.off, iE, Wk);
                        e1 = node_comb<P>(a.ringE, lv.off, iE + 1, Wk);
                    }
                    B = (1.0 - wb) * b0 + wb * b1;
                    E = (1.0 - wE) * e0 + wE * e1;
                }
                const double dtp = j == 1 ? 0.5 * (dt_old + dt_new) : dt_new;
                boris(a.qm, dtp, E, B, px, py, pz);
                const double g2 = sqrt(1.0 + ((px * px + py * py) + pz * pz));
                x = x + dt_new * (px / g2);
            }
            if (done) {
                cnt.step_done(k);
            } else {
                status = PIC_PARTICLE_LOST;
                ++cnt.lost;
            }
        }
        if (mine) {
            a.x[i] = x;
            a.px[i] = px;
            a.py[i] = py;
            a.pz[i] = pz;
            a.kold[i] = int8_t(kold);
            a.status[i] = status;
        }
    }
    flush_counts_atomic(cnt, a.cnt + int64_t(blockIdx.x % a.nslot) * NCNT);
}

// ---------------------------------------------------------------------
// FP32 bulk push with compensated state, FP64 sub-cycled steps
// (pic_precision PIC_FP32_COMP).
//
// Registers hold x as an int32 node index `cell`, an FP32 fraction `fr`
// of a cell and its FP32 carry, and each momentum component as an FP32
// pair (hi, lo).  A step with k = 0 runs in FP32: the fields come from
// the FP64 temporal combination rounded once to FP32, the Boris update is
// formed as increments of p that are added to (hi, lo) with TwoSum, and
// the position increment uses 1 - v = (1 + p_y^2 + p_z^2) / (gamma
// (gamma + |p_x|)), free of cancellation for ultra-relativistic
// electrons.  A step with k >= 1 (the stopping points, where gamma is near
// 1) is done entirely in FP64 with the FP64 weights, in node units, then
// split back.  The state in HBM stays FP64: a launch converts on entry
// and on exit.
// ---------------------------------------------------------------------
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

// 1 / b: hardware estimate and two Newton steps
__device__ __forceinline__ double rcp_nr(double b)
{
    double r = __builtin_amdgcn_rcp(b);
    double e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    e = fma(-b, r, 1.0);
    return fma(r, e, r);
}

// 1 / sqrt(a), a >= 1: hardware estimate and two Newton steps
__device__ __forceinline__ double rsq_nr(double a)
{
    double y = __builtin_amdgcn_rsq(a);
    double h = 0.5 * a;
    double r = fma(-h * y, y, 0.5);
    y = fma(y, r, y);
    r = fma(-h * y, y, 0.5);
    return fma(y, r, y);
}

__device__ __forceinline__ void boris_fast(double qm, double dtp, double E, double B, double &px,
                                           double &py, double &pz)
{
    const double c = 0.5 * qm * dtp;
    const double h = c * E;
    const double mx = px, my = py + h, mz = pz;
    const double ig = rsq_nr(1.0 + ((mx * mx + my * my) + mz * mz));
    const double t = (c * B) * ig;
    const double sz = (2.0 * t) * rcp_nr(1.0 + t * t);
    const double ax = mx + my * t;
    const double ay = my - mx * t;
    px = mx + ay * sz;
    py = (my - ax * sz) + h;
    pz = mz;
}

struct MixArgs {
    WaveArgs w;
    float dtdx_hi, dtdx_lo;      // dt / dx as an FP32 pair
    double dtdx;                 // dt / dx
};

template <int P>
__global__ void __launch_bounds__(64) push_wave_mixed_kernel(MixArgs ma)
{
    const WaveArgs &a = ma.w;
    constexpr int STRIDE = 2 * (P + 1);
    __shared__ double sE[(P + 1) * WWIN];
    __shared__ double sB[(P + 1) * WWIN];
    __shared__ float sBh[WWIN];          // B at s = 1/2, FP64 combination rounded
    __shared__ float sEn[WWIN];          // E at level n
    const int lane = threadIdx.x;
    const int ncm2 = a.ncells - 2;
    const double *W1 = a.wtab;
    const float c0f = float(0.5 * a.qm * a.dt);
    const float psif = float(a.psi_max);
    Counts cnt;
    cnt.zero();

    const int64_t i = int64_t(blockIdx.x) * 64 + lane;
    const bool mine = i < a.np;
    int cell = 0;
    float fr = 0.f, frc = 0.f, pxh = 0.f, pxl = 0.f, pyh = 0.f, pyl = 0.f, pzh = 0.f, pzl = 0.f;
    int kold = 0;
    uint8_t status = PIC_PARTICLE_LOST;
    int64_t kt_u = -1;
    if (mine) {
        const double xi = (a.x[i] - a.x_origin) / a.dx;
        status = a.status[i];
        if (status == PIC_PARTICLE_LIVE && xi >= 0.0 && xi < double(a.ncells)) {
            const double fl = floor(xi);
            cell = int(fl);
            split(xi - fl, fr, frc);
        } else if (status == PIC_PARTICLE_LIVE) {
            cell = -1;     // outside: flagged at the first step
        }
        split(a.px[i], pxh, pxl);
        split(a.py[i], pyh, pyl);
        split(a.pz[i], pzh, pzl);
        kold = a.kold[i];
        if (a.ktrace) {
            const int64_t u = a.perm[i] - a.kt_first;
            if (u >= 0 && u < a.kt_count) kt_u = u;
        }
    }
    bool moved = false;      // the FP64 state must be rewritten

    for (int st = 0; st < a.S; ++st) {
        WaveLevels<P> lv;
        lv.at(a, st);
        const bool live = status == PIC_PARTICLE_LIVE && cell >= 0 && cell <= ncm2 &&
                          (cell > 0 || fr >= 0.5f);
        if (status == PIC_PARTICLE_LIVE && !live) {
            status = PIC_PARTICLE_LOST;
            ++cnt.lost;
        }
        if (!live && kt_u >= 0) {
            const int64_t r = a.n0 + st - a.kt_n0;
            if (r >= 0 && r < a.kt_steps) a.ktrace[r * a.kt_count + kt_u] = -1;
        }
        if (!__any(live)) {
            if (kt_u >= 0)
                for (int s2 = st + 1; s2 < a.S; ++s2) {
                    const int64_t r = a.n0 + s2 - a.kt_n0;
                    if (r >= 0 && r < a.kt_steps) a.ktrace[r * a.kt_count + kt_u] = -1;
                }
            break;
        }
        const int lo = max(wave_min(live ? cell - a.margin : INT_MAX), 0);
        const int hi = min(wave_max(live ? cell + a.margin : INT_MIN), a.ncells - 1);
        const bool use_lds = hi - lo + 1 <= WWIN;
        if (use_lds) {
            __syncthreads();
            for (int q = lane; q <= hi - lo; q += 64) {
                const double b = node_comb<P>(a.ringB, lv.off, lo + q, W1 + P + 1);
                sBh[q] = float(b);
                sEn[q] = float(a.ringE[lv.off[P] + lo + q]);
            }
            __syncthreads();
        }

        // decision in FP32: B at (x_n, s = 1/2), gamma of the stored p
        int k = 0;
        float Bd = 0.f;
        float wB = fr, wE;
        int iE;
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
                b0 = float(node_comb<P>(a.ringB, lv.off, cell, W1 + P + 1));
                b1 = float(node_comb<P>(a.ringB, lv.off, cell + 1, W1 + P + 1));
            }
            Bd = (1.f - wB) * b0 + wB * b1;
            const float p2 = (pxh * pxh + pyh * pyh) + pzh * pzh;
            const float psi0 = fabsf(c0f * Bd) * __builtin_amdgcn_rsqf(1.f + p2);
            float lim = psif;
            while (psi0 > lim && k < a.kmax) {
                ++k;
                lim = lim * 4.f;
            }
            cnt.clamps += psi0 > lim;
            if (kt_u >= 0) {
                const int64_t r = a.n0 + st - a.kt_n0;
                if (r >= 0 && r < a.kt_steps) a.ktrace[r * a.kt_count + kt_u] = int8_t(k);
            }
        }
        const bool heavy = live && k > 0;
        // raw FP64 levels for the sub-cycled steps
        const bool any_heavy = __any(heavy);
        if (any_heavy && use_lds) {
            __syncthreads();
            for (int q = lane; q <= hi - lo; q += 64) {
#pragma unroll
                for (int j = 0; j <= P; ++j) {
                    sE[j * WWIN + q] = a.ringE[lv.off[j] + lo + q];
                    sB[j * WWIN + q] = a.ringB[lv.off[j] + lo + q];
                }
            }
            __syncthreads();
        }
        if (!live) continue;
        moved = true;
        const int ko = kold < 0 ? k : kold;
        kold = k;
        if (!heavy) {
            // ---- k = 0 in FP32 with compensated accumulation
            float e0, e1;
            if (use_lds) {
                e0 = sEn[iE - lo];
                e1 = sEn[iE + 1 - lo];
            } else {
                e0 = float(a.ringE[lv.off[P] + iE]);
                e1 = float(a.ringE[lv.off[P] + iE + 1]);
            }
            const float E = (1.f - wE) * e0 + wE * e1;
            const float cf = float(0.5 * a.qm * (0.5 * (ldexp(a.dt, -2 * ko) + a.dt)));
            const float h = cf * E;
            const float mx = pxh, my = pyh + h, mz = pzh;
            const float ig = __builtin_amdgcn_rsqf(1.f + ((mx * mx + my * my) + mz * mz));
            const float t = cf * Bd * ig;
            const float sz = 2.f * t * __builtin_amdgcn_rcpf(1.f + t * t);
            const float ax = mx + my * t;
            const float ay = my - mx * t;
            comp_add(pxh, pxl, ay * sz);
            comp_add(pyh, pyl, (h + h) - ax * sz);
            // position: v = p_x / gamma, with 1 - |v| formed without cancellation
            const float q2 = (pyh * pyh + pzh * pzh);
            const float g2 = __builtin_amdgcn_sqrtf(1.f + (pxh * pxh + q2));
            const float apx = fabsf(pxh);
            const float omv = (1.f + q2) * __builtin_amdgcn_rcpf(g2 * (g2 + apx));   // 1 - |v|
            // dfr = (dt/dx) v = sign(p_x) ((dt/dx) - (dt/dx)(1 - |v|))
            const float sgn = pxh < 0.f ? -1.f : 1.f;
            const float small = ma.dtdx_hi * omv;
            float y = sgn * ((ma.dtdx_lo - small) + 0.f);
            // fr + sgn*dtdx_hi is the large part; add the small part to the carry
            float s, e;
            two_sum(fr, sgn * ma.dtdx_hi, s, e);
            y = y + e + frc;
            float s2, e2;
            two_sum(s, y, s2, e2);
            // back into [0, 1)
            const float adj = s2 >= 1.f ? -1.f : (s2 < 0.f ? 1.f : 0.f);
            cell -= int(adj);
            two_sum(s2, adj, fr, e);
            frc = e2 + e;
            cnt.step_done(0);
        } else {
            // ---- sub-cycled step in FP64, node units
            double xi = double(cell) + (double(fr) + double(frc));
            double px = double(pxh) + double(pxl);
            double py = double(pyh) + double(pyl);
            double pz = double(pzh) + double(pzl);
            const double dt_new = ldexp(a.dt, -2 * k);
            const double dt_old = ldexp(a.dt, -2 * ko);
            const double rdx = ldexp(ma.dtdx, -2 * k);
            const int nsub = 1 << (2 * k);
            const double *Wk = a.wtab + wtab_offset(k) * STRIDE;
            int32_t vo[P + 1];
#pragma unroll
            for (int j = 0; j <= P; ++j) vo[j] = j * WWIN - lo;
            const double ncm1 = double(a.ncells - 1);
            bool done = true;
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
                double b0, b1, e0, e1;
                if (use_lds) {
                    b0 = node_comb<P>(sB, vo, ib, Wk + P + 1);
                    b1 = node_comb<P>(sB, vo, ib + 1, Wk + P + 1);
                    e0 = node_comb<P>(sE, vo, ie, Wk);
                    e1 = node_comb<P>(sE, vo, ie + 1, Wk);
                } else {
                    b0 = node_comb<P>(a.ringB, lv.off, ib, Wk + P + 1);
                    b1 = node_comb<P>(a.ringB, lv.off, ib + 1, Wk + P + 1);
                    e0 = node_comb<P>(a.ringE, lv.off, ie, Wk);
                    e1 = node_comb<P>(a.ringE, lv.off, ie + 1, Wk);
                }
                const double B = (1.0 - wb) * b0 + wb * b1;
                const double E = (1.0 - we) * e0 + we * e1;
                const double dtp = j == 1 ? 0.5 * (dt_old + dt_new) : dt_new;
                boris(a.qm, dtp, E, B, px, py, pz);
                const double g2 = sqrt(1.0 + ((px * px + py * py) + pz * pz));
                xi = xi + rdx * (px / g2);
            }
            if (done) {
                cnt.step_done(k);
            } else {
                status = PIC_PARTICLE_LOST;
                ++cnt.lost;
            }
            const double fl = floor(xi);
            cell = (xi >= 0.0 && xi < double(a.ncells)) ? int(fl) : -1;
            split(xi - fl, fr, frc);
            split(px, pxh, pxl);
            split(py, pyh, pyl);
            split(pz, pzh, pzl);
        }
    }
    if (mine) {
        if (moved) {
            const double xi = double(cell) + (double(fr) + double(frc));
            a.x[i] = a.x_origin + xi * a.dx;
            a.px[i] = double(pxh) + double(pxl);
            a.py[i] = double(pyh) + double(pyl);
            a.pz[i] = double(pzh) + double(pzl);
        }
        a.kold[i] = int8_t(kold);
        a.status[i] = status;
    }
    flush_counts_atomic(cnt, a.cnt + int64_t(blockIdx.x % a.nslot) * NCNT);
}

// ---------------------------------------------------------------------
// Fast FP64 push (pic_precision PIC_FP64_FAST).
//
// The same method in FP64 throughout, with three changes of evaluation
// that move results by rounding only: the reciprocal and the reciprocal
// square root use the hardware estimates refined by two Newton steps
// (faithfully rounded) in place of the IEEE division and square-root
// sequences; the position is carried in node units xi = (x - x_origin) / dx,
// so a step needs no division by dx; and 1 / gamma of the stored momentum,
// computed by the previous step's position update, is reused by the next
// step's decision.
// ---------------------------------------------------------------------
template <int P>
__global__ void __launch_bounds__(64) push_wave_fast_kernel(MixArgs ma)
{
    const WaveArgs &a = ma.w;
    constexpr int STRIDE = 2 * (P + 1);
    __shared__ double sE[(P + 1) * WWIN];
    __shared__ double sB[(P + 1) * WWIN];
    const int lane = threadIdx.x;
    const double ncm1 = double(a.ncells - 1);
    const double c0 = 0.5 * a.qm * a.dt;
    const double *W1 = a.wtab;
    double LB1[P + 1];                 // B weights at s = 1/2
#pragma unroll
    for (int j = 0; j <= P; ++j) LB1[j] = W1[P + 1 + j];
    Counts cnt;
    cnt.zero();

    const int64_t i = int64_t(blockIdx.x) * 64 + lane;
    const bool mine = i < a.np;
    double xi = 0, px = 0, py = 0, pz = 0, ig = 1;
    int kold = 0;
    uint8_t status = PIC_PARTICLE_LOST;
    int64_t kt_u = -1;
    if (mine) {
        xi = (a.x[i] - a.x_origin) / a.dx;
        px = a.px[i];
        py = a.py[i];
        pz = a.pz[i];
        ig = rsq_nr(1.0 + ((px * px + py * py) + pz * pz));
        kold = a.kold[i];
        status = a.status[i];
        if (a.ktrace) {
            const int64_t u = a.perm[i] - a.kt_first;
            if (u >= 0 && u < a.kt_count) kt_u = u;
        }
    }
    bool moved = false;

    for (int st = 0; st < a.S; ++st) {
        WaveLevels<P> lv;
        lv.at(a, st);
        const bool live = status == PIC_PARTICLE_LIVE && xi >= 0.5 && xi < ncm1;
        if (status == PIC_PARTICLE_LIVE && !live) {
            status = PIC_PARTICLE_LOST;
            ++cnt.lost;
        }
        if (!live && kt_u >= 0) {
            const int64_t r = a.n0 + st - a.kt_n0;
            if (r >= 0 && r < a.kt_steps) a.ktrace[r * a.kt_count + kt_u] = -1;
        }
        if (!__any(live)) {
            if (kt_u >= 0)
                for (int s2 = st + 1; s2 < a.S; ++s2) {
                    const int64_t r = a.n0 + s2 - a.kt_n0;
                    if (r >= 0 && r < a.kt_steps) a.ktrace[r * a.kt_count + kt_u] = -1;
                }
            break;
        }
        // decision from B at (x_n, s = 1/2), gathered straight from the ring
        int k = 0;
        int cell = 0;
        double Bd = 0.0;
        if (live) {
            const double flB = floor(xi);
            cell = int(flB);
            const double wB = xi - flB;
            const double b0 = node_comb<P>(a.ringB, lv.off, cell, LB1);
            const double b1 = node_comb<P>(a.ringB, lv.off, cell + 1, LB1);
            Bd = (1.0 - wB) * b0 + wB * b1;
            const double psi0 = fabs(c0 * Bd) * ig;
            double lim = a.psi_max;
            while (psi0 > lim && k < a.kmax) {
                ++k;
                lim = lim * 4.0;
            }
            cnt.clamps += psi0 > lim;
            if (kt_u >= 0) {
                const int64_t r = a.n0 + st - a.kt_n0;
                if (r >= 0 && r < a.kt_steps) a.ktrace[r * a.kt_count + kt_u] = int8_t(k);
            }
        }
        const bool heavy = live && k > 0;
        // sub-cycled lanes: stage their node window once for all sub-steps
        bool use_lds = false;
        int lo = 0;
        if (__any(heavy)) {
            lo = max(wave_min(heavy ? cell - a.margin : INT_MAX), 0);
            const int hi = min(wave_max(heavy ? cell + a.margin : INT_MIN), a.ncells - 1);
            use_lds = hi - lo + 1 <= WWIN;
            if (use_lds) {
                __syncthreads();
                for (int q = lane; q <= hi - lo; q += 64) {
#pragma unroll
                    for (int j = 0; j <= P; ++j) {
                        sE[j * WWIN + q] = a.ringE[lv.off[j] + lo + q];
                        sB[j * WWIN + q] = a.ringB[lv.off[j] + lo + q];
                    }
                }
                __syncthreads();
            }
        }
        if (!live) continue;
        moved = true;
        const int ko = kold < 0 ? k : kold;
        kold = k;
        const double dt_new = ldexp(a.dt, -2 * k);
        const double dt_old = ldexp(a.dt, -2 * ko);
        const double rdx = ldexp(ma.dtdx, -2 * k);
        if (k == 0) {
            const double uE = xi - 0.5;
            const double flE = floor(uE);
            const int iE = int(flE);
            const double wE = uE - flE;
            const double e0 = a.ringE[lv.off[P] + iE];
            const double e1 = a.ringE[lv.off[P] + iE + 1];
            const double E = (1.0 - wE) * e0 + wE * e1;
            boris_fast(a.qm, 0.5 * (dt_old + dt_new), E, Bd, px, py, pz);
            ig = rsq_nr(1.0 + ((px * px + py * py) + pz * pz));
            xi = xi + rdx * (px * ig);
            cnt.step_done(0);
        } else {
            // the longest dependency chains of the launch: let this
            // wavefront issue ahead of those doing single steps
            __builtin_amdgcn_s_setprio(2);
            int32_t vo[P + 1];
#pragma unroll
            for (int j = 0; j <= P; ++j) vo[j] = j * WWIN - lo;
            const int nsub = 1 << (2 * k);
            const double *Wk = a.wtab + wtab_offset(k) * STRIDE;
            bool done = true;
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
                double bb0, bb1, e0, e1;
                if (use_lds) {
                    bb0 = node_comb<P>(sB, vo, ib, Wk + P + 1);
                    bb1 = node_comb<P>(sB, vo, ib + 1, Wk + P + 1);
                    e0 = node_comb<P>(sE, vo, ie, Wk);
                    e1 = node_comb<P>(sE, vo, ie + 1, Wk);
                } else {
                    bb0 = node_comb<P>(a.ringB, lv.off, ib, Wk + P + 1);
                    bb1 = node_comb<P>(a.ringB, lv.off, ib + 1, Wk + P + 1);
                    e0 = node_comb<P>(a.ringE, lv.off, ie, Wk);
                    e1 = node_comb<P>(a.ringE, lv.off, ie + 1, Wk);
                }
                const double B = (1.0 - wb) * bb0 + wb * bb1;
                const double E = (1.0 - we) * e0 + we * e1;
                const double dtp = j == 1 ? 0.5 * (dt_old + dt_new) : dt_new;
                boris_fast(a.qm, dtp, E, B, px, py, pz);
                ig = rsq_nr(1.0 + ((px * px + py * py) + pz * pz));
                xi = xi + rdx * (px * ig);
            }
            __builtin_amdgcn_s_setprio(0);
            if (done) {
                cnt.step_done(k);
            } else {
                status = PIC_PARTICLE_LOST;
                ++cnt.lost;
            }
        }
    }
    if (mine) {
        if (moved) {
            a.x[i] = a.x_origin + xi * a.dx;
            a.px[i] = px;
            a.py[i] = py;
            a.pz[i] = pz;
        }
        a.kold[i] = int8_t(kold);
        a.status[i] = status;
    }
    flush_counts_atomic(cnt, a.cnt + int64_t(blockIdx.x % a.nslot) * NCNT);
}

}  // namespace

// ---------------------------------------------------------------------
// Host side.
// ---------------------------------------------------------------------
struct pic_ctx {
    pic_params prm;
    int64_t np = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    int ncu = 0;
    int grid = 0;        // persistent workgroups of the one-lane-per-particle push
    int tile_grid = 0;   // workgroups of the tiled push
    int block = 256;
    int tile = 256;
    bool have_particles = false;
    // particle store
    double *x = nullptr, *px = nullptr, *py = nullptr, *pz = nullptr;
    int8_t *kold = nullptr;
    uint8_t *status = nullptr;
    int32_t *perm = nullptr;
    int32_t *key = nullptr;
    // field ring
    double *ringE = nullptr, *ringB = nullptr;
    std::vector<int64_t> tags;
    // weights table
    double *wtab = nullptr;
    // counters
    uint64_t *cnt = nullptr;
    // k trace
    int8_t *ktrace = nullptr;
    int64_t kt_n0 = 0;
    int32_t kt_steps = 0;
    int64_t kt_first = 0, kt_count = 0;
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

int grid_for(int64_t work, int block, int cap)
{
    int64_t g = (work + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return int(g);
}

void free_all(pic_ctx *c)
{
    void *ptrs[] = {c->x, c->px, c->py, c->pz, c->kold, c->status, c->perm, c->key,
                    c->ringE, c->ringB, c->wtab, c->cnt};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
}

pic_status check_params(pic_ctx *ctx, const pic_params *p, int64_t np)
{
    if (!p) return fail(ctx, PIC_E_ARG, "params is NULL");
    if (np < 0 || np > INT32_MAX) return fail(ctx, PIC_E_ARG, "np out of range: %lld", (long long)np);
    if (p->ncells < 2) return fail(ctx, PIC_E_ARG, "ncells must be >= 2");
    if (p->order != 1 && p->order != 3 && p->order != 5)
        return fail(ctx, PIC_E_ARG, "order must be 1, 3 or 5 (got %d)", p->order);
    if (p->ring_depth < p->order + 1 || p->ring_depth > 1 << 20)
        return fail(ctx, PIC_E_ARG, "ring_depth must be in [order+1, 2^20]");
    if (p->k_max < 0 || p->k_max > PIC_K_MAX_LIMIT)
        return fail(ctx, PIC_E_ARG, "k_max must be in [0, %d]", PIC_K_MAX_LIMIT);
    if (!(p->dx > 0) || !(p->dt > 0)) return fail(ctx, PIC_E_ARG, "dx and dt must be > 0");
    if (!(p->dt <= 64.0 * p->dx)) return fail(ctx, PIC_E_ARG, "dt / dx must be <= 64");
    if (!(p->psi_max > 0)) return fail(ctx, PIC_E_ARG, "psi_max must be > 0");
    if (!(p->qm != 0) || p->qm != p->qm) return fail(ctx, PIC_E_ARG, "qm must be nonzero");
    if (p->x_origin != p->x_origin) return fail(ctx, PIC_E_ARG, "x_origin is NaN");
    if (p->precision != PIC_FP64 && p->precision != PIC_FP32_COMP &&
        p->precision != PIC_FP64_FAST)
        return fail(ctx, PIC_E_ARG, "unknown precision %d", p->precision);
    if (p->binning < PIC_BIN_NONE || p->binning > PIC_BIN_LEARNED)
        return fail(ctx, PIC_E_ARG, "unknown binning %d", p->binning);
    if (p->precision != PIC_FP64 && p->binning == PIC_BIN_BALLOT)
        return fail(ctx, PIC_E_ARG, "the tiled ballot push runs with PIC_FP64 only");
    if (int64_t(p->ring_depth) * p->ncells >= (int64_t(1) << 31))
        return fail(ctx, PIC_E_ARG, "ring_depth * ncells must stay below 2^31");
    if (int64_t(p->ncells) * SORT_SUB >= (int64_t(1) << 30))
        return fail(ctx, PIC_E_ARG, "ncells too large");
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

}  // namespace

extern "C" {

pic_status pic_create(const pic_params *prm, int64_t np, void *hip_stream, pic_ctx **out)
{
    if (!out) return PIC_E_ARG;
    *out = nullptr;
    pic_ctx *ctx = new (std::nothrow) pic_ctx;
    if (!ctx) return PIC_E_NOMEM;
    pic_status st = check_params(ctx, prm, np);
    if (st != PIC_OK) {
        // keep the message reachable through a context that owns nothing
        *out = ctx;
        return st;
    }
    ctx->prm = *prm;
    ctx->np = np;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    hipError_t e = hipGetDevice(&ctx->device);
    if (e != hipSuccess) {
        *out = ctx;
        return fail(ctx, PIC_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    }
    int ncu = 256;
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, ctx->device);
    const size_t n = size_t(np);
    const size_t ring = size_t(prm->ring_depth) * prm->ncells;
    const int64_t went = wtab_entries(prm->k_max);
    ctx->ncu = ncu;
    ctx->grid = grid_for(np, ctx->block, ncu * 8);
    ctx->tile_grid = grid_for(np, TILE, ncu * 16);
    if ((st = dev_alloc(ctx, &ctx->x, n)) || (st = dev_alloc(ctx, &ctx->px, n)) ||
        (st = dev_alloc(ctx, &ctx->py, n)) || (st = dev_alloc(ctx, &ctx->pz, n)) ||
        (st = dev_alloc(ctx, &ctx->kold, n)) || (st = dev_alloc(ctx, &ctx->status, n)) ||
        (st = dev_alloc(ctx, &ctx->perm, n)) || (st = dev_alloc(ctx, &ctx->key, n)) ||
        (st = dev_alloc(ctx, &ctx->ringE, ring)) || (st = dev_alloc(ctx, &ctx->ringB, ring)) ||
        (st = dev_alloc(ctx, &ctx->wtab, size_t(went) * 2 * (prm->order + 1))) ||
        (st = dev_alloc(ctx, &ctx->cnt, size_t(ncu) * 16 * NCNT))) {
        free_all(ctx);
        ctx->x = ctx->px = ctx->py = ctx->pz = ctx->ringE = ctx->ringB = ctx->wtab = nullptr;
        ctx->kold = nullptr;
        ctx->status = nullptr;
        ctx->perm = ctx->key = nullptr;
        ctx->cnt = nullptr;
        *out = ctx;
        return st;
    }
    ctx->tags.assign(size_t(prm->ring_depth), INT64_MIN);
    *out = ctx;
    weights_kernel<<<grid_for(went, 256, 4096), 256, 0, ctx->stream>>>(ctx->wtab, prm->order,
                                                                        prm->k_max);
    LAUNCH_CHECK(ctx);
    HIP_TRY(ctx, hipMemsetAsync(ctx->cnt, 0, size_t(ncu) * 16 * NCNT * sizeof(uint64_t),
                                ctx->stream));
    HIP_TRY(ctx, hipMemsetAsync(ctx->status, PIC_PARTICLE_LOST, n ? n : 1, ctx->stream));
    return PIC_OK;
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

pic_status pic_particles_set(pic_ctx *ctx, pic_mem mem, const double *x, const double *px,
                             const double *py, const double *pz, const int8_t *k_old)
{
    if (!ctx || !ctx->x) return ctx ? fail(ctx, PIC_E_STATE, "context not created") : PIC_E_ARG;
    const int64_t np = ctx->np;
    if (np > 0 && (!x || !px || !py || !pz)) return fail(ctx, PIC_E_ARG, "null particle array");
    if (mem != PIC_MEM_HOST && mem != PIC_MEM_DEVICE) return fail(ctx, PIC_E_ARG, "bad pic_mem");
    const size_t n = size_t(np);
    const double *dx_ = x, *dpx = px, *dpy = py, *dpz = pz;
    const int8_t *dk = k_old;
    double *tmp = nullptr;
    int8_t *tmpk = nullptr;
    if (mem == PIC_MEM_HOST && np > 0) {
        pic_status st = dev_alloc(ctx, &tmp, 4 * n);
        if (st) return st;
        if (k_old && (st = dev_alloc(ctx, &tmpk, n))) {
            (void)hipFree(tmp);
            return st;
        }
        const double *src[4] = {x, px, py, pz};
        for (int a = 0; a < 4; ++a) {
            hipError_t e = hipMemcpyAsync(tmp + a * n, src[a], n * sizeof(double),
                                          hipMemcpyHostToDevice, ctx->stream);
            if (e != hipSuccess) {
                (void)hipFree(tmp);
                if (tmpk) (void)hipFree(tmpk);
                return fail(ctx, PIC_E_DEVICE, "hipMemcpyAsync: %s", hipGetErrorString(e));
            }
        }
        if (k_old) HIP_TRY(ctx, hipMemcpyAsync(tmpk, k_old, n, hipMemcpyHostToDevice, ctx->stream));
        dx_ = tmp;
        dpx = tmp + n;
        dpy = tmp + 2 * n;
        dpz = tmp + 3 * n;
        dk = tmpk;
    }
    pic_status result = PIC_OK;
    if (np > 0) {
        const int nb = ctx->prm.ncells * SORT_SUB + 1;
        int32_t *hist = nullptr;
        if ((result = dev_alloc(ctx, &hist, size_t(nb)))) goto done;
        if (hipMemsetAsync(hist, 0, size_t(nb) * sizeof(int32_t), ctx->stream) != hipSuccess) {
            (void)hipFree(hist);
            result = fail(ctx, PIC_E_DEVICE, "hipMemsetAsync failed");
            goto done;
        }
        cell_key_kernel<<<grid_for(np, 256, 8192), 256, 0, ctx->stream>>>(
            dx_, np, ctx->prm.x_origin, ctx->prm.dx, ctx->prm.ncells, ctx->key, hist);
        scan_kernel<<<1, 1024, 0, ctx->stream>>>(hist, nb);
        scatter_kernel<<<grid_for(np, 256, 8192), 256, 0, ctx->stream>>>(ctx->key, np, hist,
                                                                        ctx->perm);
        gather_state_kernel<<<grid_for(np, 256, 8192), 256, 0, ctx->stream>>>(
            ctx->perm, np, dx_, dpx, dpy, dpz, dk, ctx->x, ctx->px, ctx->py, ctx->pz, ctx->kold,
            ctx->status);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(ctx->stream);
            (void)hipFree(hist);
            result = fail(ctx, PIC_E_DEVICE, "load kernels: %s", hipGetErrorString(e));
            goto done;
        }
        // hist and the staging copy are released after the stream passes them
        e = hipStreamSynchronize(ctx->stream);
        (void)hipFree(hist);
        if (e != hipSuccess) {
            result = fail(ctx, PIC_E_DEVICE, "particle load: %s", hipGetErrorString(e));
            goto done;
        }
    }
    {
        hipError_t e = hipMemsetAsync(ctx->cnt, 0, size_t(ctx->ncu) * 16 * NCNT * sizeof(uint64_t),
                                      ctx->stream);
        if (e != hipSuccess) result = fail(ctx, PIC_E_DEVICE, "hipMemsetAsync: %s", hipGetErrorString(e));
    }
    ctx->have_particles = true;
done:
    if (tmp) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipFree(tmp);
        if (tmpk) (void)hipFree(tmpk);
    }
    return result;
}

pic_status pic_fields_load(pic_ctx *ctx, int64_t n, pic_mem mem, const double *Ey,
                           const double *Bz)
{
    if (!ctx || !ctx->x) return ctx ? fail(ctx, PIC_E_STATE, "context not created") : PIC_E_ARG;
    if (!Ey || !Bz) return fail(ctx, PIC_E_ARG, "null field array");
    if (mem != PIC_MEM_HOST && mem != PIC_MEM_DEVICE) return fail(ctx, PIC_E_ARG, "bad pic_mem");
    const int D = ctx->prm.ring_depth;
    const int64_t slot = mod_floor(n, D);
    const size_t bytes = size_t(ctx->prm.ncells) * sizeof(double);
    const hipMemcpyKind kind = mem == PIC_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->ringE + slot * ctx->prm.ncells, Ey, bytes, kind, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(ctx->ringB + slot * ctx->prm.ncells, Bz, bytes, kind, ctx->stream));
    if (mem == PIC_MEM_HOST) HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    ctx->tags[size_t(slot)] = n;
    return PIC_OK;
}

pic_status pic_fields_load_lattice(pic_ctx *ctx, int64_t n_first, int32_t count,
                                   const double *table, int64_t M, int64_t aE, int64_t bE,
                                   int64_t cE, int64_t aB, int64_t bB, int64_t cB)
{
    if (!ctx || !ctx->x) return ctx ? fail(ctx, PIC_E_STATE, "context not created") : PIC_E_ARG;
    if (!table || M <= 0) return fail(ctx, PIC_E_ARG, "bad table");
    const int D = ctx->prm.ring_depth;
    if (count < 0 || count > D) return fail(ctx, PIC_E_ARG, "count must be in [0, ring_depth]");
    if (count == 0) return PIC_OK;
    const int64_t work = int64_t(count) * ctx->prm.ncells;
    lattice_kernel<<<grid_for(work, 256, 16384), 256, 0, ctx->stream>>>(
        ctx->ringE, ctx->ringB, D, ctx->prm.ncells, n_first, count, table, M, aE, bE, cE, aB, bB,
        cB);
    LAUNCH_CHECK(ctx);
    for (int32_t c = 0; c < count; ++c) ctx->tags[size_t(mod_floor(n_first + c, D))] = n_first + c;
    return PIC_OK;
}

pic_status pic_ktrace_set(pic_ctx *ctx, int8_t *buf, int64_t n_first, int32_t steps,
                          int64_t first, int64_t count)
{
    if (!ctx || !ctx->x) return ctx ? fail(ctx, PIC_E_STATE, "context not created") : PIC_E_ARG;
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
    if (!ctx || !ctx->x) return ctx ? fail(ctx, PIC_E_STATE, "context not created") : PIC_E_ARG;
    if (!ctx->have_particles) return fail(ctx, PIC_E_STATE, "particles not loaded");
    if (S < 1) return fail(ctx, PIC_E_ARG, "S must be >= 1");
    const pic_params &p = ctx->prm;
    if (int64_t(S) + p.order > p.ring_depth)
        return fail(ctx, PIC_E_LEVEL, "S + order = %d exceeds ring_depth %d", S + p.order,
                    p.ring_depth);
    for (int64_t m = n - p.order; m <= n + S - 1; ++m)
        if (ctx->tags[size_t(mod_floor(m, p.ring_depth))] != m)
            return fail(ctx, PIC_E_LEVEL, "field level %lld is not in the ring", (long long)m);
    if (ctx->np == 0) return PIC_OK;
    PushArgs a;
    a.x = ctx->x;
    a.px = ctx->px;
    a.py = ctx->py;
    a.pz = ctx->pz;
    a.kold = ctx->kold;
    a.status = ctx->status;
    a.perm = ctx->perm;
    a.ringE = ctx->ringE;
    a.ringB = ctx->ringB;
    a.wtab = ctx->wtab;
    a.ktrace = ctx->ktrace;
    a.cnt = ctx->cnt;
    a.np = ctx->np;
    a.n0 = n;
    a.kt_n0 = ctx->kt_n0;
    a.kt_steps = ctx->kt_steps;
    a.kt_first = ctx->kt_first;
    a.kt_count = ctx->kt_count;
    a.x_origin = p.x_origin;
    a.dx = p.dx;
    a.dt = p.dt;
    a.qm = p.qm;
    a.psi_max = p.psi_max;
    a.D = p.ring_depth;
    a.ncells = p.ncells;
    a.kmax = p.k_max;
    a.S = S;
    const int32_t slot0 = int32_t(mod_floor(n - p.order, p.ring_depth));
    // |v| < c, so a particle crosses fewer than dt / dx cells per step
    const int32_t margin = int32_t(std::ceil(p.dt / p.dx)) + 2;
    if (p.binning == PIC_BIN_NONE) {
        WaveArgs wa;
        wa.x = ctx->x;
        wa.px = ctx->px;
        wa.py = ctx->py;
        wa.pz = ctx->pz;
        wa.kold = ctx->kold;
        wa.status = ctx->status;
        wa.perm = ctx->perm;
        wa.ringE = ctx->ringE;
        wa.ringB = ctx->ringB;
        wa.wtab = ctx->wtab;
        wa.ktrace = ctx->ktrace;
        wa.cnt = ctx->cnt;
        wa.nslot = ctx->ncu * 16;
        wa.np = ctx->np;
        wa.n0 = n;
        wa.kt_n0 = ctx->kt_n0;
        wa.kt_first = ctx->kt_first;
        wa.kt_count = ctx->kt_count;
        wa.x_origin = p.x_origin;
        wa.dx = p.dx;
        wa.dt = p.dt;
        wa.qm = p.qm;
        wa.psi_max = p.psi_max;
        wa.D = p.ring_depth;
        wa.ncells = p.ncells;
        wa.kmax = p.k_max;
        wa.S = S;
        wa.kt_steps = ctx->kt_steps;
        wa.slot0 = slot0;
        wa.margin = margin;
        const dim3 grid(unsigned((ctx->np + 63) / 64)), block(64);
        MixArgs ma;
        ma.w = wa;
        ma.dtdx = p.dt / p.dx;
        ma.dtdx_hi = float(ma.dtdx);
        ma.dtdx_lo = float(ma.dtdx - double(ma.dtdx_hi));
        if (p.precision == PIC_FP32_COMP) {
            switch (p.order) {
            case 1: push_wave_mixed_kernel<1><<<grid, block, 0, ctx->stream>>>(ma); break;
            case 3: push_wave_mixed_kernel<3><<<grid, block, 0, ctx->stream>>>(ma); break;
            default: push_wave_mixed_kernel<5><<<grid, block, 0, ctx->stream>>>(ma); break;
            }
        } else if (p.precision == PIC_FP64_FAST) {
            switch (p.order) {
            case 1: push_wave_fast_kernel<1><<<grid, block, 0, ctx->stream>>>(ma); break;
            case 3: push_wave_fast_kernel<3><<<grid, block, 0, ctx->stream>>>(ma); break;
            default: push_wave_fast_kernel<5><<<grid, block, 0, ctx->stream>>>(ma); break;
            }
        } else {
            switch (p.order) {
            case 1: push_wave_kernel<1><<<grid, block, 0, ctx->stream>>>(wa); break;
            case 3: push_wave_kernel<3><<<grid, block, 0, ctx->stream>>>(wa); break;
            default: push_wave_kernel<5><<<grid, block, 0, ctx->stream>>>(wa); break;
            }
        }
        LAUNCH_CHECK(ctx);
        return PIC_OK;
    }
    TileArgs ta;
    ta.x = ctx->x;
    ta.px = ctx->px;
    ta.py = ctx->py;
    ta.pz = ctx->pz;
    ta.kold = ctx->kold;
    ta.status = ctx->status;
    ta.perm = ctx->perm;
    ta.ringE = ctx->ringE;
    ta.ringB = ctx->ringB;
    ta.wtab = ctx->wtab;
    ta.ktrace = ctx->ktrace;
    ta.cnt = ctx->cnt;
    ta.np = ctx->np;
    ta.n0 = n;
    ta.kt_n0 = ctx->kt_n0;
    ta.kt_first = ctx->kt_first;
    ta.kt_count = ctx->kt_count;
    ta.x_origin = p.x_origin;
    ta.dx = p.dx;
    ta.dt = p.dt;
    ta.qm = p.qm;
    ta.psi_max = p.psi_max;
    ta.D = p.ring_depth;
    ta.ncells = p.ncells;
    ta.kmax = p.k_max;
    ta.S = S;
    ta.kt_steps = ctx->kt_steps;
    ta.slot0 = slot0;
    ta.margin = margin;
    const dim3 tgrid(ctx->tile_grid), tblock(TILE);
    switch (p.order) {
    case 1: push_tile_kernel<1><<<tgrid, tblock, 0, ctx->stream>>>(ta); break;
    case 3: push_tile_kernel<3><<<tgrid, tblock, 0, ctx->stream>>>(ta); break;
    default: push_tile_kernel<5><<<tgrid, tblock, 0, ctx->stream>>>(ta); break;
    }
    LAUNCH_CHECK(ctx);
    return PIC_OK;
}

pic_status pic_counters_reset(pic_ctx *ctx)
{
    if (!ctx || !ctx->x) return ctx ? fail(ctx, PIC_E_STATE, "context not created") : PIC_E_ARG;
    HIP_TRY(ctx, hipMemsetAsync(ctx->cnt, 0, size_t(ctx->ncu) * 16 * NCNT * sizeof(uint64_t),
                                ctx->stream));
    return PIC_OK;
}

pic_status pic_diag(pic_ctx *ctx, pic_mem mem, double *gamma, double *px, double *py,
                    double *pz, double *x, int8_t *k_last, uint8_t *status, pic_counters *cnt)
{
    if (!ctx || !ctx->x) return ctx ? fail(ctx, PIC_E_STATE, "context not created") : PIC_E_ARG;
    if (mem != PIC_MEM_HOST && mem != PIC_MEM_DEVICE) return fail(ctx, PIC_E_ARG, "bad pic_mem");
    const int64_t np = ctx->np;
    const size_t n = size_t(np);
    const bool any = gamma || px || py || pz || x || k_last || status;
    if (any && np > 0) {
        if (!ctx->have_particles) return fail(ctx, PIC_E_STATE, "particles not loaded");
        if (mem == PIC_MEM_DEVICE) {
            diag_kernel<<<grid_for(np, 256, 8192), 256, 0, ctx->stream>>>(
                ctx->perm, np, ctx->x, ctx->px, ctx->py, ctx->pz, ctx->kold, ctx->status, gamma,
                px, py, pz, x, k_last, status);
            LAUNCH_CHECK(ctx);
        } else {
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
            diag_kernel<<<grid_for(np, 256, 8192), 256, 0, ctx->stream>>>(
                ctx->perm, np, ctx->x, ctx->px, ctx->py, ctx->pz, ctx->kold, ctx->status, d,
                d + n, d + 2 * n, d + 3 * n, d + 4 * n, dk, ds);
            hipError_t e = hipGetLastError();
            double *outs[5] = {gamma, px, py, pz, x};
            for (int a = 0; a < 5 && e == hipSuccess; ++a)
                if (outs[a])
                    e = hipMemcpyAsync(outs[a], d + a * n, n * sizeof(double),
                                       hipMemcpyDeviceToHost, ctx->stream);
            if (e == hipSuccess && k_last)
                e = hipMemcpyAsync(k_last, dk, n, hipMemcpyDeviceToHost, ctx->stream);
            if (e == hipSuccess && status)
                e = hipMemcpyAsync(status, ds, n, hipMemcpyDeviceToHost, ctx->stream);
            hipError_t e2 = hipStreamSynchronize(ctx->stream);
            (void)hipFree(d);
            (void)hipFree(dk);
            (void)hipFree(ds);
            if (e != hipSuccess || e2 != hipSuccess)
                return fail(ctx, PIC_E_DEVICE, "diag copy: %s",
                            hipGetErrorString(e != hipSuccess ? e : e2));
        }
    }
    if (cnt) {
        std::vector<uint64_t> h(size_t(ctx->ncu) * 16 * NCNT);
        HIP_TRY(ctx, hipMemcpyAsync(h.data(), ctx->cnt, h.size() * sizeof(uint64_t),
                                    hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        std::memset(cnt, 0, sizeof *cnt);
        for (size_t b = 0; b < h.size() / NCNT; ++b) {
            const uint64_t *r = h.data() + b * NCNT;
            for (int k = 0; k < PIC_KHIST; ++k) cnt->steps_by_k[k] += r[k];
            cnt->clamps += r[CNT_CLAMPS];
            cnt->lost += r[CNT_LOST];
        }
        for (int k = 0; k < PIC_KHIST; ++k) {
            const uint64_t sub = cnt->steps_by_k[k] << (2 * k);
            cnt->sub_steps_by_k[k] = sub;
            cnt->steps += cnt->steps_by_k[k];
            cnt->sub_steps += sub;
            if (k > 0) cnt->n_star += sub;
        }
    }
    return PIC_OK;
}

pic_status pic_tune_set(pic_ctx *ctx, int32_t block, int32_t tile)
{
    if (!ctx || !ctx->x) return ctx ? fail(ctx, PIC_E_STATE, "context not created") : PIC_E_ARG;
    if (block && (block < 64 || block > 1024 || block % 64))
        return fail(ctx, PIC_E_ARG, "block must be a multiple of 64 in [64, 1024]");
    if (tile && (tile < 64 || (block ? tile % block : tile % ctx->block)))
        return fail(ctx, PIC_E_ARG, "tile must be a multiple of block");
    if (block) ctx->block = block;
    if (tile) ctx->tile = tile;
    return PIC_OK;
}

}  // extern "C"
