// fields_yee.hpp -- the 1D Yee field solver of the "standard PIC" (Sec. III,
// Eqs. (Ey) and (Bz)), writing the levels the push reads into a run's ring.
//
// Level n = (E_y at n dt on the nodes (i + 1/2) dx, B_z at (n + 1/2) dt on
// the nodes i dx) follows from level n - 1 alone:
//     E^n[i]       = E^{n-1}[i] - nu (B^{n-1/2}[i+1] - B^{n-1/2}[i])
//     B^{n+1/2}[i] = B^{n-1/2}[i] - nu (E^n[i] - E^n[i-1]),   nu = dt / dx,
// with the laser entering at node 0 (B_z there is the incident wave, read
// from a phase table) and the first-order Mur one-way condition on the last
// E node,
//     E^n[N-1] = E^{n-1}[N-2] + kappa (E^n[N-2] - E^{n-1}[N-1]),
//     kappa = (dt - dx) / (dt + dx).
// Plain IEEE subtract / multiply / add in this order (the library is built
// without contraction), so the levels are bit-identical to a CPU loop.
//
// Levels depend on each other in sequence, and one level of a 16k-node grid
// is far too little work for the GPU, so a launch advances T levels at once
// with overlapping tiles: one wavefront holds 64 R consecutive nodes in
// registers (R per lane), advances them T levels with neighbour values
// passed between lanes by shuffles, and stores only its middle 64 R - 2 H
// nodes, H = T + 2.  Values near a tile's ends go stale one node per level
// (they miss neighbours outside the tile), which the halo H absorbs.  No
// LDS, no barrier, no inter-wavefront communication.
#pragma once

#include "common.hpp"

namespace picsub {

constexpr int YEE_R = 2;     // nodes per lane
constexpr int YEE_T = 40;    // levels per launch (at most)

template <int R, int T>
__global__ void __launch_bounds__(64) yee_kernel(double *__restrict__ ringE,
                                                 double *__restrict__ ringB, int D, int ncells,
                                                 int64_t n_first, int count, double nu,
                                                 double kappa, const double *__restrict__ table,
                                                 int64_t M, int64_t aB, int64_t cB)
{
    constexpr int H = T + 2;
    constexpr int WT = 64 * R - 2 * H;     // nodes a wavefront stores
    static_assert(WT > 0, "tile too small for the halo");
    const int lane = threadIdx.x;
    const int t0 = blockIdx.x * WT;        // first stored node
    const int base = t0 - H + lane * R;    // this lane's first node (may be off the grid)
    const int64_t prev = mod_floor(n_first - 1, D) * ncells;
    double e[R], b[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = base + r;
        const bool in = i >= 0 && i < ncells;
        e[r] = in ? ringE[prev + i] : 0.0;
        b[r] = in ? ringB[prev + i] : 0.0;
    }
    // ring slot and source-table index of the level being made, moved on
    // by one level per pass (no division in the loop)
    int32_t slot = int32_t(mod_floor(n_first, D));
    int64_t q = mod_floor(aB * n_first + cB, M);
    const int64_t dq = mod_floor(aB, M);
    for (int c = 0; c < count; ++c) {
        // E: B of the node to the right (the next lane's first node)
        const double bnext = __shfl_down(b[0], 1);
        double en[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double br = r + 1 < R ? b[r + 1] : bnext;
            en[r] = e[r] - nu * (br - b[r]);
        }
        // new and old E of the node to the left of this lane's first node
        const double enprev = __shfl_up(en[R - 1], 1);
        const double eoprev = __shfl_up(e[R - 1], 1);
        // right end: Mur on node ncells - 1
        if (base <= ncells - 1 && ncells - 1 < base + R) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (base + r == ncells - 1) {
                    const double eo2 = r > 0 ? e[r - 1] : eoprev;
                    const double en2 = r > 0 ? en[r - 1] : enprev;
                    en[r] = eo2 + kappa * (en2 - e[r]);
                }
            }
        }
        double bn[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double el = r > 0 ? en[r - 1] : enprev;
            bn[r] = b[r] - nu * (en[r] - el);
        }
        // left end: the incident wave at node 0
        if (base <= 0 && 0 < base + R) {
            const double src = table[q];
#pragma unroll
            for (int r = 0; r < R; ++r)
                if (base + r == 0) bn[r] = src;
        }
        const int64_t off = int64_t(slot) * ncells;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = base + r;
            if (i >= t0 && i < t0 + WT && i < ncells) {
                ringE[off + i] = en[r];
                ringB[off + i] = bn[r];
            }
            e[r] = en[r];
            b[r] = bn[r];
        }
        slot = slot + 1 == D ? 0 : slot + 1;
        q += dq;
        if (q >= M) q -= M;
    }
}

}  // namespace picsub
