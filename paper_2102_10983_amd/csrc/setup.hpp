// setup.hpp -- kernels around the push: weight table, field sampling,
// particle load (sort by position) and read-back.
#pragma once

#include "common.hpp"

namespace picsub {

// ---------------------------------------------------------------------
// Weights table: L^E_j and L^B_j (Eqs. (lagrange2-2), (lagrange2-3)) for
// sub-step j of a step with exponent k, at s = 1/2 + (j-1)/4^k (units of
// dt after (n - 1/2) dt).  Entry e = (4^k - 1)/3 + (j - 1), stride
// 2 (p + 1): L^E_0..L^E_p, L^B_0..L^B_p.  The numerator product runs over
// the other nodes in ascending order and is divided once by the integer
// denominator (exact for the dyadic s of k <= 7 at p = 3).
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
// Field levels from a phase table: E_y(level m, node i) =
// table[(aE m + bE i + cE) mod M], likewise B_z.  This samples prescribed
// fields on the Yee lattice ("perfectly propagating PIC", Sec. III).
// ---------------------------------------------------------------------
__global__ void lattice_kernel(double *__restrict__ ringE, double *__restrict__ ringB, int D,
                               int ncells, int64_t n_first, int count,
                               const double *__restrict__ table, int64_t M, int64_t aE, int64_t bE,
                               int64_t cE, int64_t aB, int64_t bB, int64_t cB)
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

// Device-driven form for a batch: run blockIdx.y fills its levels
// n_cur .. n_cur + count - 1 from its own table.
__global__ void batch_lattice_kernel(const RunDesc *__restrict__ runs, int count)
{
    const RunDesc &R = runs[blockIdx.y];
    double *ringE = const_cast<double *>(R.ringE);
    double *ringB = const_cast<double *>(R.ringB);
    const int64_t left = R.n_stop - R.n_cur;
    const int64_t levels = left <= 0 ? 0 : (left < count ? left : count);
    const int64_t total = levels * R.ncells;
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
         t += int64_t(gridDim.x) * blockDim.x) {
        const int64_t m = R.n_cur + t / R.ncells;
        const int64_t i = t % R.ncells;
        const int64_t slot = mod_floor(m, R.D);
        ringE[slot * R.ncells + i] = R.table[mod_floor(R.aE * m + R.bE * i + R.cE, R.M)];
        ringB[slot * R.ncells + i] = R.table[mod_floor(R.aB * m + R.bB * i + R.cB, R.M)];
    }
}

// Device-driven form: every run's current level moves on by S, up to its
// stop level.
__global__ void tick_kernel(RunDesc *__restrict__ runs, int nruns, int S)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nruns) {
        const int64_t left = runs[r].n_stop - runs[r].n_cur;
        runs[r].n_cur += left <= 0 ? 0 : (left < S ? left : S);
    }
}

// ---------------------------------------------------------------------
// Particle load.  Key = run's bin base + position in units of
// dx / sort_sub: particles with nearly the same position (for a cold beam,
// nearly the same phase history and so the same sub-cycling history) land
// in neighbouring lanes.  Bin nb_r of a run collects particles outside its
// grid or with a NaN position.
// ---------------------------------------------------------------------
struct LoadRun {
    int64_t caller_off, np, p_off, bin_off;
    double x_origin, dx;
    int32_t ncells, pad;
};

__device__ __forceinline__ int find_run(const LoadRun *__restrict__ lr, int nruns, int64_t i)
{
    int lo = 0, hi = nruns - 1;      // last run with caller_off <= i
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (lr[mid].caller_off <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void key_kernel(const double *__restrict__ x, int64_t np, const LoadRun *__restrict__ lr,
                           int nruns, int sort_sub, int32_t *__restrict__ key,
                           int32_t *__restrict__ hist)
{
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < np;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int r = find_run(lr, nruns, i);
        const int32_t nfine = lr[r].ncells * sort_sub;
        const double u = (x[i] - lr[r].x_origin) / lr[r].dx * double(sort_sub);
        int32_t c = nfine;
        if (u >= 0.0 && u < double(nfine)) c = int32_t(u);
        const int32_t k = int32_t(lr[r].bin_off) + c;
        key[i] = k;
        atomicAdd(&hist[k], 1);
    }
}

// Exclusive scan of nb counts: per-chunk sums, a scan of the sums, then
// each chunk rescanned from its base.
constexpr int SCAN_CHUNK = 4096;

__global__ void scan_sums_kernel(const int32_t *__restrict__ v, int64_t nb, int32_t *__restrict__ sums)
{
    __shared__ int32_t part[256];
    const int64_t base = int64_t(blockIdx.x) * SCAN_CHUNK;
    int32_t s = 0;
    for (int q = threadIdx.x; q < SCAN_CHUNK; q += 256)
        if (base + q < nb) s += v[base + q];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if (int(threadIdx.x) < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[blockIdx.x] = part[0];
}

__global__ void scan_top_kernel(int32_t *__restrict__ sums, int n)
{
    // one workgroup of 1024 threads, sequential runs of n / 1024
    __shared__ int32_t part[1024];
    const int t = threadIdx.x;
    const int per = (n + 1023) / 1024;
    const int lo = t * per, hi = min(n, lo + per);
    int32_t s = 0;
    for (int i = lo; i < hi; ++i) s += sums[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int32_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int32_t run = part[t] - s;
    for (int i = lo; i < hi; ++i) {
        const int32_t c = sums[i];
        sums[i] = run;
        run += c;
    }
}

__global__ void scan_chunk_kernel(int32_t *__restrict__ v, int64_t nb, const int32_t *__restrict__ sums)
{
    // 256 threads, 16 consecutive entries each
    __shared__ int32_t part[256];
    const int64_t base = int64_t(blockIdx.x) * SCAN_CHUNK + int64_t(threadIdx.x) * 16;
    int32_t loc[16];
    int32_t s = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        loc[q] = base + q < nb ? v[base + q] : 0;
        s += loc[q];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int32_t w = int(threadIdx.x) >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += w;
        __syncthreads();
    }
    int32_t run = sums[blockIdx.x] + part[threadIdx.x] - s;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        if (base + q < nb) v[base + q] = run;
        run += loc[q];
    }
}

// Scatter into slots: position within the run from an atomic cursor on the
// particle's bin (order inside a bin is arbitrary: it changes no
// particle's arithmetic, only its lane).
__global__ void scatter_kernel(const int32_t *__restrict__ key, int64_t np,
                               const LoadRun *__restrict__ lr, int nruns,
                               int32_t *__restrict__ cursor, int32_t *__restrict__ perm)
{
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < np;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int r = find_run(lr, nruns, i);
        const int64_t pos = atomicAdd(&cursor[key[i]], 1);
        perm[pos - lr[r].caller_off + lr[r].p_off] = int32_t(i);
    }
}

__global__ void gather_state_kernel(const int32_t *__restrict__ perm, int64_t slots,
                                    const double *__restrict__ x, const double *__restrict__ px,
                                    const double *__restrict__ py, const double *__restrict__ pz,
                                    const int8_t *__restrict__ kold, double *__restrict__ sx,
                                    double *__restrict__ spx, double *__restrict__ spy,
                                    double *__restrict__ spz, int8_t *__restrict__ skold,
                                    uint8_t *__restrict__ sstatus,
                                    const uint8_t *__restrict__ status)
{
    for (int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < slots;
         s += int64_t(gridDim.x) * blockDim.x) {
        const int32_t u = perm[s];
        if (u >= 0) {
            sx[s] = x[u];
            spx[s] = px[u];
            spy[s] = py[u];
            spz[s] = pz[u];
            skold[s] = kold ? kold[u] : int8_t(-1);
            sstatus[s] = status ? status[u] : uint8_t(PIC_PARTICLE_LIVE);
        } else {
            sx[s] = spx[s] = spy[s] = spz[s] = 0.0;
            skold[s] = -1;
            sstatus[s] = PIC_PARTICLE_LOST;
        }
    }
}

// Per-particle outputs of pic_diag in caller order, for the caller indices
// u_lo .. u_lo + u_n - 1 (written at u - u_lo); null outputs are skipped.
__global__ void diag_kernel(const int32_t *__restrict__ perm, int64_t slots,
                            const double *__restrict__ sx, const double *__restrict__ spx,
                            const double *__restrict__ spy, const double *__restrict__ spz,
                            const int8_t *__restrict__ skold, const uint8_t *__restrict__ sst,
                            int64_t u_lo, int64_t u_n,
                            double *__restrict__ gamma, double *__restrict__ px,
                            double *__restrict__ py, double *__restrict__ pz,
                            double *__restrict__ x, int8_t *__restrict__ klast,
                            uint8_t *__restrict__ status)
{
    for (int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < slots;
         s += int64_t(gridDim.x) * blockDim.x) {
        const int64_t u = int64_t(perm[s]) - u_lo;
        if (u < 0 || u >= u_n) continue;
        const double a = spx[s], b = spy[s], c = spz[s];
        if (gamma) gamma[u] = sqrt(1.0 + ((a * a + b * b) + c * c));
        if (px) px[u] = a;
        if (py) py[u] = b;
        if (pz) pz[u] = c;
        if (x) x[u] = sx[s];
        if (klast) klast[u] = skold[s];
        if (status) status[u] = sst[s];
    }
}

// Strict mode: flag[0] := 1 if any of a[0 .. n) is not finite (flag is
// cleared by the caller).
__global__ void nonfinite_kernel(const double *__restrict__ a, int64_t n, int32_t *__restrict__ flag)
{
    bool bad = false;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        bad |= !__builtin_isfinite(a[i]);
    if (bad) flag[0] = 1;
}

// Sum of the counter words over `rows` slots (all runs): out[j] = sum_r
// cnt[r][j], one workgroup of 256 threads.  Every word of out is written.
__global__ void __launch_bounds__(256) counter_sum_kernel(const uint64_t *__restrict__ cnt,
                                                          int64_t rows, uint64_t *__restrict__ out)
{
    __shared__ uint64_t part[256][NCNT];
    uint64_t acc[NCNT];
#pragma unroll
    for (int j = 0; j < NCNT; ++j) acc[j] = 0;
    for (int64_t r = threadIdx.x; r < rows; r += 256)
#pragma unroll
        for (int j = 0; j < NCNT; ++j) acc[j] += cnt[r * NCNT + j];
#pragma unroll
    for (int j = 0; j < NCNT; ++j) part[threadIdx.x][j] = acc[j];
    __syncthreads();
    if (threadIdx.x < NCNT) {
        uint64_t s = 0;
        for (int t = 0; t < 256; ++t) s += part[t][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// Trajectory diagnostics: R0 = gamma - p_x of the stored momentum of every
// slot; running maximum, work and largest step energy error reset to zero.
__global__ void diag_init_kernel(int64_t slots, const double *__restrict__ px,
                                 const double *__restrict__ py, const double *__restrict__ pz,
                                 double *__restrict__ r0, double *__restrict__ rmax,
                                 double *__restrict__ work, double *__restrict__ werr,
                                 double *__restrict__ gmax)
{
    for (int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < slots;
         s += int64_t(gridDim.x) * blockDim.x) {
        const double a = px[s], b = py[s], c = pz[s];
        const double g = sqrt(1.0 + ((a * a + b * b) + c * c));
        r0[s] = g - a;
        gmax[s] = g;
        rmax[s] = 0.0;
        work[s] = 0.0;
        werr[s] = 0.0;
    }
}

// Energy error start: a_i from caller order into slots, running maxima 0.
__global__ void gerr_init_kernel(const int32_t *__restrict__ perm, int64_t slots,
                                 const double *__restrict__ ai_caller, double *__restrict__ ai,
                                 double *__restrict__ emax)
{
    for (int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < slots;
         s += int64_t(gridDim.x) * blockDim.x) {
        const int32_t u = perm[s];
        ai[s] = u >= 0 ? ai_caller[u] : 0.0;
        emax[s] = 0.0;
    }
}

// Two per-slot arrays in caller order (an output, or the array it would
// come from, may be null: that output is skipped).
__global__ void slots_to_caller_kernel(const int32_t *__restrict__ perm, int64_t slots,
                                       const double *__restrict__ a,
                                       const double *__restrict__ b, double *__restrict__ oa,
                                       double *__restrict__ ob)
{
    for (int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < slots;
         s += int64_t(gridDim.x) * blockDim.x) {
        const int32_t u = perm[s];
        if (u < 0) continue;
        if (oa && a) oa[u] = a[s];
        if (ob && b) ob[u] = b[s];
    }
}

// Order score from a k trace (persistence): per particle (column), log2 of
// the mean of 4^k over the steps where it was live (k >= 0); NaN when it was
// never live.  Columns are consecutive in memory across threads.
__global__ void ktrace_load_kernel(const int8_t *__restrict__ kt, int32_t steps, int64_t count,
                                   float *__restrict__ score)
{
    for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < count;
         c += int64_t(gridDim.x) * blockDim.x) {
        uint64_t tot = 0;
        int32_t live = 0;
        for (int32_t s = 0; s < steps; ++s) {
            const int k = kt[int64_t(s) * count + c];
            if (k >= 0) {
                tot += uint64_t(1) << (2 * k);
                ++live;
            }
        }
        score[c] = live ? float(log2(double(tot) / double(live))) : __builtin_nanf("");
    }
}

// Attainable FP64 vector rate on this device (a measurement aid, not part of
// the method): every lane runs 16 independent chains of fused multiply-adds,
// enough to cover the FMA latency, `iters` rounds each; the sums are stored
// so that none of the work can be dropped.
__global__ void __launch_bounds__(256) fma_probe_kernel(double *__restrict__ out, int64_t iters,
                                                        double a, double b)
{
    double v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = double(threadIdx.x + i);
    for (int64_t it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = fma(v[i], a, b);
    }
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) s += v[i];
    out[int64_t(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

}  // namespace picsub
