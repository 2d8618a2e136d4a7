// Orientation choice by local Fourier analysis (Sec. 3, strategy on
// macro-elements).  For every vertex permutation of a macro-tetrahedron: the
// constant stencil A_d of the permuted tetrahedron for a unit coefficient, the
// asymptotic ILU stencil (L^inf_d, D^inf_c) as the Gauss-Seidel fixed point of
// the stencil equations, and the smoothing factor
//     mu = max over theta in Theta_osc of |(L D conj(L) - A)(theta) / (L D conj(L))(theta)|
// with the symbols L(theta) = 1 + sum_{d in D_l} L_d e^{i d.theta},
// D(theta) = D^inf_c, A(theta) = sum_{d in D} A_d e^{i d.theta}, sampled on a
// uniform grid of cell centres theta_j = -pi + (2j+1) pi / samples per
// direction and kept where some |theta_i| >= pi/2.
#include <hip/hip_runtime.h>

#include <math.h>

#include "kernels_common.h"
#include "lfa_kernels.h"
#include "stencil_device.h"

namespace ilu {

namespace {

// Index in D_l of the lattice offset (dx, dy, dz); -1 if it is not a lower direction.
__device__ inline int lower_index(int dx, int dy, int dz) {
    for (int s = 0; s < NLOW; ++s)
        if (low_dx(s) == dx && low_dy(s) == dy && low_dz(s) == dz) return s;
    return -1;
}

// k-th permutation of (0, 1, 2, 3) in lexicographic order.
__device__ inline void perm_of(int k, int seq[4]) {
    int avail[4] = {0, 1, 2, 3};
    const int fact[4] = {6, 2, 1, 1};
    for (int i = 0; i < 4; ++i) {
        const int q = k / fact[i];
        k %= fact[i];
        seq[i] = avail[q];
        for (int j = q; j < 3 - i; ++j) avail[j] = avail[j + 1];
    }
}

}  // namespace

// One thread per (tetrahedron, permutation k).  Original vertex i becomes
// vertex seq[i] of the permuted tetrahedron.  The stencil is taken at the
// lattice point (4,4,4) of level 4 (every neighbour interior; with a constant
// coefficient all such points share it, and mu does not depend on the level).
// The stencil equations are swept in the order bc, s, bnw, be, w, bn, se,
// then c, from L_c = D_c = 1 and L_d = 0, until no value moves by more than
// 1e-15 (relative for D).
__global__ void __launch_bounds__(64) k_lfa_stencils(const double* __restrict__ verts, int64_t vstride, int ntets,
                               double* __restrict__ rec) {
    const int id = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (id >= ntets * LFA_PERMS) return;
    const int tet = id / LFA_PERMS, k = id % LFA_PERMS;
    int seq[4];
    perm_of(k, seq);
    double pv[4][3];
    for (int i = 0; i < 4; ++i)
        for (int r = 0; r < 3; ++r) pv[seq[i]][r] = verts[(int64_t)tet * vstride + 3 * i + r];
    double J[9], v0[3];
    for (int r = 0; r < 3; ++r) {
        v0[r] = pv[0][r];
        for (int c = 0; c < 3; ++c) J[3 * r + c] = pv[c + 1][r] - pv[0][r];
    }
    double A[15];
    stencil_row(J, v0, 1.0 / 16.0, 4, 4, 4, [](double, double, double) { return 1.0; }, A);
    constexpr int order[NLOW] = {5, 1, 3, 6, 0, 4, 2};
    double L[NLOW] = {0, 0, 0, 0, 0, 0, 0};
    double D = 1.0;
    bool conv = false;
    for (int it = 0; it < LFA_MAX_ITERS && !conv; ++it) {
        double Lold[NLOW];
        for (int s = 0; s < NLOW; ++s) Lold[s] = L[s];
        const double Dold = D;
        for (int q = 0; q < NLOW; ++q) {
            const int d = order[q];
            double acc = A[d];
            for (int dt = 0; dt < NLOW; ++dt) {
                if (dt == d) continue;
                const int e = lower_index(low_dx(dt) - low_dx(d), low_dy(dt) - low_dy(d), low_dz(dt) - low_dz(d));
                if (e >= 0) acc -= L[dt] * D * L[e];
            }
            L[d] = acc / D;
        }
        double ss = 0.0;
        for (int s = 0; s < NLOW; ++s) ss += L[s] * L[s];
        D = A[7] - D * ss;
        double dl = 0.0;
        for (int s = 0; s < NLOW; ++s) dl = fmax(dl, fabs(L[s] - Lold[s]));
        conv = dl < 1e-15 && fabs(D - Dold) < 1e-15 * fabs(D);
    }
    double* o = rec + (int64_t)id * LFA_REC;
    for (int s = 0; s < 15; ++s) o[s] = A[s];
    for (int s = 0; s < NLOW; ++s) o[15 + s] = L[s];
    o[22] = D;
    o[23] = conv && D > 0.0 && isfinite(D) ? 1.0 : 0.0;
}

// One workgroup per (tetrahedron, permutation): the frequencies are split over
// the threads, each keeps its largest ratio, and a fixed-order max reduction
// gives mu (+inf where the fixed point was not reached).
__global__ void __launch_bounds__(256) k_lfa_symbols(const double* __restrict__ rec, int samples,
                                                     double* __restrict__ mu) {
    __shared__ double red[256];
    const double* p = rec + (int64_t)blockIdx.x * LFA_REC;
    double A[15], L[NLOW];
    for (int s = 0; s < 15; ++s) A[s] = p[s];
    for (int s = 0; s < NLOW; ++s) L[s] = p[15 + s];
    const double D = p[22];
    const int total = samples * samples * samples;
    double m = 0.0;
    for (int f = (int)threadIdx.x; f < total; f += 256) {
        const int ij[3] = {f / (samples * samples), (f / samples) % samples, f % samples};
        // |theta_i| >= pi/2  <=>  2 |2 j + 1 - samples| >= samples
        bool osc = false;
        double th[3];
        for (int c = 0; c < 3; ++c) {
            osc = osc || 2 * abs(2 * ij[c] + 1 - samples) >= samples;
            th[c] = -M_PI + (2 * ij[c] + 1) * M_PI / samples;
        }
        if (!osc) continue;
        double lre = 1.0, lim = 0.0, are = A[7], aim = 0.0;
        for (int s = 0; s < NLOW; ++s) {
            double sn, cs;
            sincos(low_dx(s) * th[0] + low_dy(s) * th[1] + low_dz(s) * th[2], &sn, &cs);
            lre += L[s] * cs;
            lim += L[s] * sn;
            are += (A[s] + A[8 + s]) * cs;   // A[8+s] sits at -d_s
            aim += (A[s] - A[8 + s]) * sn;
        }
        const double C = D * (lre * lre + lim * lim);
        m = fmax(m, sqrt((C - are) * (C - are) + aim * aim) / fabs(C));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) mu[blockIdx.x] = p[23] != 0.0 ? red[0] : HUGE_VAL;
}

// One thread per tetrahedron: the first permutation with the smallest mu
// (the same comparisons, in the same order, as the host-side choice).
__global__ void k_lfa_best(const double* __restrict__ mu, int ntets, int32_t* __restrict__ best) {
    const int tet = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (tet >= ntets) return;
    const double* m = mu + (int64_t)tet * LFA_PERMS;
    int b = 0;
    for (int k = 1; k < LFA_PERMS; ++k)
        if (m[k] < m[b]) b = k;
    best[tet] = b;
}

void launch_lfa_stencils(const double* verts, int64_t vstride, int ntets, double* rec, hipStream_t st) {
    const int n = ntets * LFA_PERMS;
    k_lfa_stencils<<<(n + 63) / 64, 64, 0, st>>>(verts, vstride, ntets, rec);
}

void launch_lfa_best(const double* mu, int ntets, int32_t* best, hipStream_t st) {
    k_lfa_best<<<(ntets + 63) / 64, 64, 0, st>>>(mu, ntets, best);
}

void launch_lfa_symbols(const double* rec, int ntets, int samples, double* mu, hipStream_t st) {
    k_lfa_symbols<<<ntets * LFA_PERMS, 256, 0, st>>>(rec, samples, mu);
}

}  // namespace ilu
