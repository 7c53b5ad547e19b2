// mlp.hpp -- the sub-cycling load predictor: features, forward, gradients,
// Adam.
//
// Network: 8 -> 64 -> 64 -> 1, GELU (erf form, erf to 1.5e-7) after both hidden layers,
// weights used in BF16 (rounded to nearest even from FP32 master weights),
// activations and accumulation in FP32.  Parameter vector (FP32, 4801
// entries): W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3.
// Inputs are standardised: u_j = (f_j - mean_j) * inv_std_j.
#pragma once

#include "common.hpp"

namespace picsub {

constexpr int NF = 8, NH = 64;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NH * NF, OFF_W2 = OFF_B1 + NH,
              OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH,
              NPARAM = OFF_B3 + 1;   // 4801

// FP32 -> BF16 bits, round to nearest even (finite inputs)
__host__ __device__ inline uint16_t bf16_bits(float f)
{
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

__host__ __device__ inline float bf16_value(uint16_t b)
{
    const uint32_t u = uint32_t(b) << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
}

// erf by Abramowitz & Stegun's rational approximation 7.1.26 (Handbook of
// Mathematical Functions, 1964): erf(x) = 1 - t (a1 + t (a2 + t (a3 +
// t (a4 + t a5)))) exp(-x^2), t = 1 / (1 + p x) for x >= 0, odd in x;
// absolute error at most 1.5e-7 (one or two FP32 ulps of values near 1).
// Branch-free: hardware reciprocal and exponential estimates.
__device__ __forceinline__ float erf_as(float x)
{
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
    float q = fmaf(1.061405429f, t, -1.453152027f);
    q = fmaf(q, t, 1.421413741f);
    q = fmaf(q, t, -0.284496736f);
    q = fmaf(q, t, 0.254829592f);
    const float e = __builtin_amdgcn_exp2f(-(ax * ax) * 1.44269504088896341f);
    return copysignf(fmaf(-(q * t), e, 1.0f), x);
}

__device__ __forceinline__ float gelu(float z)
{
    return 0.5f * z * (1.0f + erf_as(z * 0.70710678118654752f));
}

__device__ __forceinline__ float gelu_grad(float z)
{
    return 0.5f * (1.0f + erf_as(z * 0.70710678118654752f)) +
           z * 0.39894228040143268f * __builtin_amdgcn_exp2f(-0.5f * z * z * 1.44269504088896341f);
}

// Stage the BF16-valued weights in LDS as FP32; from FP32 masters (w32)
// rounded here, or from BF16 bits (w16).
__device__ __forceinline__ void stage_weights(float *sw, const float *w32, const uint16_t *w16)
{
    for (int q = threadIdx.x; q < NPARAM; q += blockDim.x)
        sw[q] = w32 ? bf16_value(bf16_bits(w32[q])) : bf16_value(w16[q]);
    __syncthreads();
}

typedef float floatx16 __attribute__((ext_vector_type(16)));

// Forward pass with the second layer (64 x 64 per sample, 88 % of the
// network's multiply-adds) on the matrix cores, FP32 in and out
// (v_mfma_f32_32x32x2_f32: D[32 x 32] += A[32 x 2] B[2 x 32]), so the
// arithmetic is the network's own: BF16-valued weights, FP32 activations
// and sums (summed in the matrix unit's order).  A wavefront takes 64
// samples at a time and computes Z2^T = W2 H1^T as 2 x 2 tiles of 32 x 32
// over 32 steps of K = 2.  In step kk lane l (c = l mod 32, h = l / 32)
// supplies
//   A: W2[32 mt + c][2 kk + h] (from LDS),
//   B: H1[32 nt + c][2 kk + h], the first layer of samples c and 32 + c at
//      hidden neuron 2 kk + h, which it computes just before,
// and it ends holding D: Z2[sample 32 nt + c][output 32 mt + 8 (r / 4) +
// 4 h + r mod 4], so a sample's output sum is the lane's own 32 terms plus
// those of lane l ^ 32.
__global__ void __launch_bounds__(256) mlp_forward_kernel(const uint16_t *__restrict__ w16,
                                                          const float *__restrict__ norm,
                                                          const float *__restrict__ feat,
                                                          float *__restrict__ out, int64_t n)
{
    __shared__ float sw[NPARAM];
    stage_weights(sw, nullptr, w16);
    const int lane = threadIdx.x & 63;
    const int c = lane & 31, h = lane >> 5;
    const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = (int64_t(gridDim.x) * blockDim.x) >> 6;
    for (int64_t base = wave * 64; base < n; base += nwaves * 64) {
        float u[2][NF];
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            const int64_t s = base + 32 * nt + c;
#pragma unroll
            for (int j = 0; j < NF; ++j)
                u[nt][j] = s < n ? (feat[s * NF + j] - norm[j]) * norm[NF + j] : 0.f;
        }
        floatx16 acc[2][2];
#pragma unroll
        for (int mt = 0; mt < 2; ++mt)
#pragma unroll
            for (int nt = 0; nt < 2; ++nt)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[mt][nt][r] = 0.f;
#pragma unroll 1
        for (int kk = 0; kk < NH / 2; ++kk) {
            const int i = 2 * kk + h;
            float hb[2];
#pragma unroll
            for (int nt = 0; nt < 2; ++nt) {
                float z = sw[OFF_B1 + i];
#pragma unroll
                for (int j = 0; j < NF; ++j) z = fmaf(sw[OFF_W1 + i * NF + j], u[nt][j], z);
                hb[nt] = gelu(z);
            }
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                const float a = sw[OFF_W2 + (32 * mt + c) * NH + i];
#pragma unroll
                for (int nt = 0; nt < 2; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, hb[nt], acc[mt][nt], 0, 0, 0);
            }
        }
        // bias, GELU and the output neuron
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
            float y = 0.f;
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int o = 32 * mt + 8 * (r >> 2) + 4 * h + (r & 3);
                    y = fmaf(sw[OFF_W3 + o], gelu(acc[mt][nt][r] + sw[OFF_B2 + o]), y);
                }
            y += __shfl_xor(y, 32);
            const int64_t s = base + 32 * nt + c;
            if (h == 0 && s < n) out[s] = y + sw[OFF_B3];
        }
    }
}

// Gradient of L = (1/n_total) sum_s (y_s - t_s)^2 with respect to the FP32
// master weights (straight through the BF16 rounding), accumulated into
// grad[NPARAM] and the loss into loss[0].  One wavefront per workgroup
// takes 64 samples at a time in four phases over two LDS tiles:
//   A  lane = sample: forward; h1 -> T1, z2 -> T2;
//   B  lane = neuron o: dL/dz2 of every sample of the chunk (written over
//      z2 in T2) and the rows o of dW2, db2, dW3;
//   C  lane = sample: dL/dz1 (written over h1 in T1);
//   D  lane = neuron i: the rows i of dW1 and db1.
// The per-lane row sums are added to grad once at the end.
__global__ void __launch_bounds__(64) mlp_grad_kernel(const float *__restrict__ w32,
                                                      const float *__restrict__ norm,
                                                      const float *__restrict__ feat,
                                                      const float *__restrict__ target, int64_t n,
                                                      float inv_total, float *__restrict__ grad,
                                                      float *__restrict__ loss)
{
    __shared__ float sw[NPARAM];
    __shared__ float T1[64][NH + 1];
    __shared__ float T2[64][NH + 1];
    __shared__ float su[64][NF];
    __shared__ float sd3[64];
    stage_weights(sw, w32, nullptr);
    const int lane = threadIdx.x;
    float gW2[NH], gW1[NF];
#pragma unroll
    for (int i = 0; i < NH; ++i) gW2[i] = 0.f;
#pragma unroll
    for (int j = 0; j < NF; ++j) gW1[j] = 0.f;
    float gb1 = 0.f, gb2 = 0.f, gW3 = 0.f, gb3 = 0.f, lsum = 0.f;

    for (int64_t base = int64_t(blockIdx.x) * 64; base < n; base += int64_t(gridDim.x) * 64) {
        const int64_t s = base + lane;
        const bool valid = s < n;
        // A: forward of this lane's sample
        float u[NF];
#pragma unroll
        for (int j = 0; j < NF; ++j) u[j] = valid ? (feat[s * NF + j] - norm[j]) * norm[NF + j] : 0.f;
#pragma unroll 4
        for (int o = 0; o < NH; ++o) {
            float z = sw[OFF_B1 + o];
#pragma unroll
            for (int j = 0; j < NF; ++j) z = fmaf(sw[OFF_W1 + o * NF + j], u[j], z);
            T1[lane][o] = gelu(z);
        }
        float y = sw[OFF_B3];
#pragma unroll 1
        for (int o = 0; o < NH; ++o) {
            float z = sw[OFF_B2 + o];
#pragma unroll
            for (int i = 0; i < NH; ++i) z = fmaf(sw[OFF_W2 + o * NH + i], T1[lane][i], z);
            T2[lane][o] = z;
            y = fmaf(sw[OFF_W3 + o], gelu(z), y);
        }
        const float r = valid ? y - target[s] : 0.f;
        lsum = fmaf(r, r, lsum);
        sd3[lane] = valid ? 2.f * r * inv_total : 0.f;      // dL/dy
#pragma unroll
        for (int j = 0; j < NF; ++j) su[lane][j] = u[j];
        __syncthreads();
        // B: lane = neuron o
        {
            const int o = lane;
            const float w3 = sw[OFF_W3 + o];
            for (int b = 0; b < 64; ++b) {
                const float z2 = T2[b][o];
                const float d3 = sd3[b];
                gW3 = fmaf(d3, gelu(z2), gW3);
                const float d2 = d3 * w3 * gelu_grad(z2);
                T2[b][o] = d2;
                gb2 += d2;
#pragma unroll
                for (int i = 0; i < NH; ++i) gW2[i] = fmaf(d2, T1[b][i], gW2[i]);
            }
            if (o == 0)
                for (int b = 0; b < 64; ++b) gb3 += sd3[b];
        }
        __syncthreads();
        // C: lane = sample, dL/dz1 (z1 recomputed from the inputs)
#pragma unroll 1
        for (int i = 0; i < NH; ++i) {
            float z = sw[OFF_B1 + i];
#pragma unroll
            for (int j = 0; j < NF; ++j) z = fmaf(sw[OFF_W1 + i * NF + j], u[j], z);
            float d = 0.f;
#pragma unroll 8
            for (int o = 0; o < NH; ++o) d = fmaf(sw[OFF_W2 + o * NH + i], T2[lane][o], d);
            T1[lane][i] = d * gelu_grad(z);
        }
        __syncthreads();
        // D: lane = neuron i
        {
            const int i = lane;
            for (int b = 0; b < 64; ++b) {
                const float d1 = T1[b][i];
                gb1 += d1;
#pragma unroll
                for (int j = 0; j < NF; ++j) gW1[j] = fmaf(d1, su[b][j], gW1[j]);
            }
        }
        __syncthreads();
    }
    const int o = lane;
#pragma unroll
    for (int i = 0; i < NH; ++i) atomicAdd(&grad[OFF_W2 + o * NH + i], gW2[i]);
#pragma unroll
    for (int j = 0; j < NF; ++j) atomicAdd(&grad[OFF_W1 + o * NF + j], gW1[j]);
    atomicAdd(&grad[OFF_B1 + o], gb1);
    atomicAdd(&grad[OFF_B2 + o], gb2);
    atomicAdd(&grad[OFF_W3 + o], gW3);
    if (o == 0) atomicAdd(&grad[OFF_B3], gb3);
    float ls = lsum;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) ls += __shfl_xor(ls, off);
    if (lane == 0) atomicAdd(loss, ls * inv_total);
}

__global__ void adam_kernel(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                            const float *__restrict__ g, int n, float lr, float b1, float b2,
                            float eps, float c1, float c2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// Features of every particle at level n (caller order): |E|, |B| at the
// particle from levels n-1 (E at (n-1) dt, B at (n-1/2) dt), their
// backward differences with level n-2 divided by dt, gamma, p_x,
// |p_perp|, log a0 of the run.  Particles not live get zeros.
struct FeatArgs {
    const RunDesc *runs;
    const int32_t *group_run;
    const double *x, *px, *py, *pz;
    const uint8_t *status;
    const int32_t *perm;
    const float *run_a0;
    float *feat;
    int64_t n;          // NO_LEVEL: each run's n_cur
    int64_t slots;
};

__global__ void features_kernel(FeatArgs f)
{
    for (int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < f.slots;
         s += int64_t(gridDim.x) * blockDim.x) {
        const int32_t u = f.perm[s];
        if (u < 0) continue;
        const int run = f.group_run[s / 64];
        const RunDesc &R = f.runs[run];
        float *o = f.feat + int64_t(u) * NF;
        const double xi = (f.x[s] - R.x_origin) / R.dx;
        if (f.status[s] != PIC_PARTICLE_LIVE || !(xi >= 0.5 && xi < double(R.ncells - 1))) {
#pragma unroll
            for (int j = 0; j < NF; ++j) o[j] = 0.f;
            continue;
        }
        const int64_t n = f.n != NO_LEVEL ? f.n : R.n_cur;
        const int64_t s1 = mod_floor(n - 1, R.D) * R.ncells, s2 = mod_floor(n - 2, R.D) * R.ncells;
        const double flB = floor(xi), wB = xi - flB;
        const double uE = xi - 0.5, flE = floor(uE), wE = uE - flE;
        const int iB = int(flB), iE = int(flE);
        const double E1 = (1.0 - wE) * R.ringE[s1 + iE] + wE * R.ringE[s1 + iE + 1];
        const double E2 = (1.0 - wE) * R.ringE[s2 + iE] + wE * R.ringE[s2 + iE + 1];
        const double B1 = (1.0 - wB) * R.ringB[s1 + iB] + wB * R.ringB[s1 + iB + 1];
        const double B2 = (1.0 - wB) * R.ringB[s2 + iB] + wB * R.ringB[s2 + iB + 1];
        const double a = f.px[s], b = f.py[s], c = f.pz[s];
        o[0] = float(fabs(E1));
        o[1] = float(fabs(B1));
        o[2] = float((E1 - E2) / R.dt);
        o[3] = float((B1 - B2) / R.dt);
        o[4] = float(sqrt(1.0 + ((a * a + b * b) + c * c)));
        o[5] = float(a);
        o[6] = float(sqrt(b * b + c * c));
        o[7] = logf(f.run_a0[run]);
    }
}

// Largest non-NaN score (-1e30 if none): each block reduces a grid-stride
// share into out[blockIdx.x]; a second one-block launch over those
// partial results leaves the maximum in out[0].
constexpr int SCORE_MAX_BLOCKS = 256;

__global__ void __launch_bounds__(256) score_max_kernel(const float *in, int64_t n, float *out)
{
    __shared__ float part[4];
    float m = -1e30f;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        const float v = in[i];
        if (v == v) m = fmaxf(m, v);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)
        out[blockIdx.x] = fmaxf(fmaxf(part[0], part[1]), fmaxf(part[2], part[3]));
}

// Re-binning key: (run, predicted-cost bucket with heavy first, position).
__global__ void prebin_key_kernel(const RunDesc *__restrict__ runs,
                                  const int32_t *__restrict__ group_run, const double *__restrict__ x,
                                  const int32_t *__restrict__ perm, const float *__restrict__ score,
                                  const int64_t *__restrict__ bin_off, int nbuckets, float width,
                                  const float *__restrict__ topp, int sort_sub, int64_t slots,
                                  int32_t *__restrict__ key, int32_t *__restrict__ hist)
{
    const float top = *topp;
    for (int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < slots;
         s += int64_t(gridDim.x) * blockDim.x) {
        const int32_t u = perm[s];
        if (u < 0) continue;
        const int run = group_run[s / 64];
        const RunDesc &R = runs[run];
        const float sc = score[u];
        int b = int((top - sc) / width);                  // 0: heaviest
        b = b < 0 ? 0 : (b >= nbuckets ? nbuckets - 1 : b);
        if (!(sc == sc)) b = nbuckets - 1;
        const int32_t nfine = R.ncells * sort_sub;
        const double q = (x[s] - R.x_origin) / R.dx * double(sort_sub);
        int32_t c = nfine;
        if (q >= 0.0 && q < double(nfine)) c = int32_t(q);
        const int32_t k = int32_t(bin_off[run] + int64_t(b) * (nfine + 1) + c);
        key[s] = k;
        atomicAdd(&hist[k], 1);
    }
}

// New slot of every particle from its key; cursor holds the scanned
// counts, slot_base[run] - caller base folds run offsets back in.
__global__ void prebin_scatter_kernel(const int32_t *__restrict__ key, const int32_t *__restrict__ perm,
                                      const int32_t *__restrict__ group_run,
                                      const int64_t *__restrict__ shift, int64_t slots,
                                      int32_t *__restrict__ cursor, int32_t *__restrict__ dest)
{
    for (int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < slots;
         s += int64_t(gridDim.x) * blockDim.x) {
        if (perm[s] < 0) continue;
        const int run = group_run[s / 64];
        dest[s] = int32_t(atomicAdd(&cursor[key[s]], 1) + shift[run]);
    }
}

__global__ void permute_state_kernel(const int32_t *__restrict__ dest, int64_t slots,
                                     const double *__restrict__ x, const double *__restrict__ px,
                                     const double *__restrict__ py, const double *__restrict__ pz,
                                     const int8_t *__restrict__ kold, const uint8_t *__restrict__ st,
                                     const int32_t *__restrict__ perm, double *__restrict__ nx,
                                     double *__restrict__ npx, double *__restrict__ npy,
                                     double *__restrict__ npz, int8_t *__restrict__ nkold,
                                     uint8_t *__restrict__ nst, int32_t *__restrict__ nperm)
{
    for (int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < slots;
         s += int64_t(gridDim.x) * blockDim.x) {
        if (perm[s] < 0) continue;
        const int32_t d = dest[s];
        nx[d] = x[s];
        npx[d] = px[s];
        npy[d] = py[s];
        npz[d] = pz[s];
        nkold[d] = kold[s];
        nst[d] = st[s];
        nperm[d] = perm[s];
    }
}

// Two per-slot FP64 arrays moved to the slots permute_state_kernel gives.
__global__ void permute_pair_kernel(const int32_t *__restrict__ dest, int64_t slots,
                                    const int32_t *__restrict__ perm,
                                    const double *__restrict__ a, const double *__restrict__ b,
                                    double *__restrict__ na, double *__restrict__ nb)
{
    for (int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < slots;
         s += int64_t(gridDim.x) * blockDim.x) {
        if (perm[s] < 0) continue;
        const int32_t d = dest[s];
        na[d] = a[s];
        nb[d] = b[s];
    }
}

// One per-slot FP64 array moved the same way.
__global__ void permute_one_kernel(const int32_t *__restrict__ dest, int64_t slots,
                                   const int32_t *__restrict__ perm, const double *__restrict__ a,
                                   double *__restrict__ na)
{
    for (int64_t s = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; s < slots;
         s += int64_t(gridDim.x) * blockDim.x) {
        if (perm[s] < 0) continue;
        na[dest[s]] = a[s];
    }
}

// Predicted cost of each group: largest score of its lanes (LPT key).
__global__ void group_cost_kernel(const float *__restrict__ score, const int32_t *__restrict__ perm,
                                  int32_t ngroups, float *__restrict__ gcost)
{
    const int g = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    if (g >= ngroups) return;
    const int lane = threadIdx.x & 63;
    const int32_t u = perm[int64_t(g) * 64 + lane];
    float v = u >= 0 ? score[u] : -1e30f;
    if (!(v == v)) v = -1e30f;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    if (lane == 0) gcost[g] = v;
}

}  // namespace picsub
