// Setup kernels of libilu: stencil assembly, ILU(0) factorisation by the
// stencil recurrences, factor transposition, sampling on S_d, FP64 TSQR
// least squares and the per-row surrogate evaluation tables.
#include <hip/hip_runtime.h>
#include <math.h>

#include "kernels_common.h"
#include "setup_kernels.h"
#include "stencil_device.h"

namespace ilu {

// ---------------------------------------------------------------- assembly

__device__ double kappa_at(const TetDev& T, double X, double Y, double Z) {
    const double two_pi = 6.283185307179586476925286766559;
    const double* p = T.cp;
    switch (T.kind) {
    case 0: return p[0];
    case 1: return p[0] + p[1] * sin(two_pi * p[2] * X) * sin(two_pi * p[2] * Y) * sin(two_pi * p[2] * Z);
    case 2: return exp(p[0] * sin(two_pi * p[2] * X) * cos(two_pi * p[2] * Y));
    default: {
        int i = (int)p[2];
        return p[0] + p[1] * (pow(X, (double)i) + pow(Y, (double)i) + pow(Z, (double)i));
    }
    }
}

// One thread per (block, lane, hyperplane): the stencil row of p (sum over the
// 24 micro-tetrahedra around p, stencil_row).  Writes the centre and the
// seven lower weights (entries whose
// neighbour is on the macro boundary are stored as 0: the restricted matrix
// drops them), slot order [c, w, s, se, bnw, bn, bc, be].
__global__ void __launch_bounds__(256) k_assemble(const TetDev* __restrict__ tets, const BlockDev* __restrict__ blocks,
                           const LaneDev* __restrict__ lanes, int lpb, int groups, int nblocks, int64_t S, double* __restrict__ A8,
                           double* __restrict__ Afull /* optional [15][S] */) {
    int b, lane;
    decode_group(groups, b, lane);
    const BlockDev B = blocks[b];
    const LaneDev& Ln = lanes[(int64_t)b * lpb + lane];
    if (Ln.v == 0) return;
    const TetDev& T = tets[B.tet];
    const int n = T.n, v = Ln.v, w = Ln.w, y = v - w, z = w;
    const double invn = 1.0 / n;
    for (int t = B.tb + (int)(threadIdx.x >> 6); t <= B.te; t += (int)(blockDim.x >> 6)) {
        const int x = t - 2 * v - w;  // x = u - v, u = t - v - w
        if (x < 1 || x > n - 1 - v) continue;
        double Ad[15];
        stencil_row(T.J, T.v0, invn, x, y, z, [&](double X, double Y, double Z) { return kappa_at(T, X, Y, Z); }, Ad);
        const int64_t idx = Ln.rp[R_SELF] + (int64_t)lpb * t;
        A8[idx] = Ad[7];
        for (int s = 0; s < NLOW; ++s) {
            const bool in = interior(n, x + low_dx(s), y + low_dy(s), z + low_dz(s));
            A8[(int64_t)(1 + s) * S + idx] = in ? Ad[s] : 0.0;
        }
        if (Afull) {
            for (int s = 0; s < 15; ++s) {
                const int dx = s < 7 ? low_dx(s) : s == 7 ? 0 : -low_dx(s - 8);
                const int dy = s < 7 ? low_dy(s) : s == 7 ? 0 : -low_dy(s - 8);
                const int dz = s < 7 ? low_dz(s) : s == 7 ? 0 : -low_dz(s - 8);
                const bool in = (s == 7) || interior(n, x + dx, y + dy, z + dz);
                Afull[(int64_t)s * S + idx] = in ? Ad[s] : 0.0;
            }
        }
    }
}

// ------------------------------------------------------------ factorisation

// One launch per hyperplane t (every point of a hyperplane only depends on
// earlier hyperplanes).  For each active point p solves the stencil equations
// of Sec. 3 (eq. matrix-equations) in the order of Alg. 1 -- bc, s, bnw, be,
// w, bn, se, then the pivot c -- from the already factored lower neighbours.
// Neighbours that are not interior contribute L = 0, D = 1 (the guard values
// of Alg. 1).  k_factor_plane writes the factors to full planes Lf[7][S]
// (lower weights) and Df[S], k_factor_ring to a ring of four hyperplanes.
// A point with D <= 0 is reported through flags[0].

// The stencil equations of one point (Alg. 1): lower weights a[s] = A^p_{d_s}
// and centre Ac of the point, pivots Dn[s] of the lower neighbours (1 where
// the neighbour is not interior) and their factors Lq(s, d) = L^{p+d_s}_d (0
// where not interior).  Equations in the order bc, s, bnw, be, w, bn, se, c.
template <class LQ>
__device__ __forceinline__ void stencil_equations(const double (&a)[NLOW], double Ac, const double (&Dn)[NLOW], LQ Lq,
                                                  double (&Lp)[NLOW], double& Dp) {
    enum { W_ = 0, S_ = 1, SE = 2, BNW = 3, BN = 4, BC = 5, BE = 6 };
    const double Lbc = a[BC] / Dn[BC];
    const double Ls = (a[S_] - Lbc * Dn[BC] * Lq(S_, BN)) / Dn[S_];
    const double Lbnw = (a[BNW] - Lbc * Dn[BC] * Lq(BNW, SE)) / Dn[BNW];
    const double Lbe = (a[BE] - Lbc * Dn[BC] * Lq(BE, W_)) / Dn[BE];
    const double Lw = (a[W_] - Lbc * Dn[BC] * Lq(W_, BE) - Lbnw * Dn[BNW] * Lq(W_, BN) - Ls * Dn[S_] * Lq(W_, SE)) /
                      Dn[W_];
    const double Lbn = (a[BN] - Lbc * Dn[BC] * Lq(BN, S_) - Lbe * Dn[BE] * Lq(BN, SE) - Lbnw * Dn[BNW] * Lq(BN, W_)) /
                       Dn[BN];
    const double Lse = (a[SE] - Lbc * Dn[BC] * Lq(SE, BNW) - Lbe * Dn[BE] * Lq(SE, BN) - Ls * Dn[S_] * Lq(SE, W_)) /
                       Dn[SE];
    Dp = Ac - Lbc * Lbc * Dn[BC] - Lbe * Lbe * Dn[BE] - Lbnw * Lbnw * Dn[BNW] - Lbn * Lbn * Dn[BN] -
         Lse * Lse * Dn[SE] - Ls * Ls * Dn[S_] - Lw * Lw * Dn[W_];
    Lp[W_] = Lw;
    Lp[S_] = Ls;
    Lp[SE] = Lse;
    Lp[BNW] = Lbnw;
    Lp[BN] = Lbn;
    Lp[BC] = Lbc;
    Lp[BE] = Lbe;
}

// Alg. 1 on the hyperplane schedule into full factor planes (stored variant).
__global__ void k_factor_plane(const TetDev* __restrict__ tets, const BlockDev* __restrict__ blocks,
                               const LaneDev* __restrict__ lanes, int lpb, int groups, int t_glob, int64_t S, const double* __restrict__ A8,
                               double* __restrict__ Lf, double* __restrict__ Df, int* __restrict__ flags) {
    int b, lane;
    decode_group(groups, b, lane);
    const BlockDev& B = blocks[b];
    const int t = t_glob;
    if (t < B.tb || t > B.te) return;
    const LaneDev& Ln = lanes[(int64_t)b * lpb + lane];
    if (Ln.v == 0) return;
    const int n = tets[B.tet].n, v = Ln.v, w = Ln.w, y = v - w, z = w;
    const int x = t - 2 * v - w;
    if (x < 1 || x > n - 1 - v) return;
    const int64_t idx = Ln.rp[R_SELF] + (int64_t)lpb * t;
    int64_t q[NLOW];
    bool in[NLOW];
    double Dn[NLOW], a[NLOW];
#pragma unroll
    for (int s = 0; s < NLOW; ++s) {
        q[s] = Ln.rp[low_row(s)] + (int64_t)lpb * (t + low_dt(s));
        in[s] = interior(n, x + low_dx(s), y + low_dy(s), z + low_dz(s));
        Dn[s] = in[s] ? Df[q[s]] : 1.0;
        a[s] = A8[(int64_t)(1 + s) * S + idx];
    }
    auto Lq = [&](int s, int d) -> double { return in[s] ? Lf[(int64_t)d * S + q[s]] : 0.0; };
    double Lp[NLOW], Dp;
    stencil_equations(a, A8[idx], Dn, Lq, Lp, Dp);
#pragma unroll
    for (int s = 0; s < NLOW; ++s) Lf[(int64_t)s * S + idx] = in[s] ? Lp[s] : 0.0;
    Df[idx] = Dp;
    if (!(Dp > 0.0)) atomicOr(&flags[0], 1);
}

// Backward-sweep weights per point: Lb[0] = 1/D^p, Lb[1+s] = L^{p-d_s}_{d_s}
// (the transposed factor, read from the upper neighbour; 0 if that neighbour
// is not interior).
__global__ void k_transpose_factors(const TetDev* __restrict__ tets, const BlockDev* __restrict__ blocks,
                                    const LaneDev* __restrict__ lanes, int lpb, int groups, int64_t S, const double* __restrict__ Lf,
                                    const double* __restrict__ Df, double* __restrict__ Lb) {
    int b, lane;
    decode_group(groups, b, lane);
    const BlockDev B = blocks[b];
    const LaneDev& Ln = lanes[(int64_t)b * lpb + lane];
    if (Ln.v == 0) return;
    const int n = tets[B.tet].n, v = Ln.v, w = Ln.w, y = v - w, z = w;
    for (int t = B.tb + (int)(threadIdx.x >> 6); t <= B.te; t += (int)(blockDim.x >> 6)) {
        const int x = t - 2 * v - w;
        if (x < 1 || x > n - 1 - v) continue;
        const int64_t idx = Ln.rp[R_SELF] + (int64_t)lpb * t;
        Lb[idx] = 1.0 / Df[idx];
#pragma unroll
        for (int s = 0; s < NLOW; ++s) {
            const bool in = interior(n, x - low_dx(s), y - low_dy(s), z - low_dz(s));
            const int64_t qq = Ln.rp[up_row(s)] + (int64_t)lpb * (t + up_dt(s));
            Lb[(int64_t)(1 + s) * S + idx] = in ? Lf[(int64_t)s * S + qq] : 0.0;
        }
    }
}

// ----------------------------------------------------------------- sampling

// Sample sets (Sec. 4.1, reading of the garbled formula): p interior,
// p = shift_d (mod stride) componentwise with shift_d = 1 - min(d, 0), and
// p + d interior.  With k = (p - shift)/stride the set is the lattice simplex
// {k >= 0, k_x + k_y + k_z <= M_d}; sample k is stored at its lexicographic
// position (k_z slowest).
__device__ __forceinline__ int64_t simplex_index(int M, int kx, int ky, int kz) {
    // points with k_z' < k_z: C(M+3,3) - C(M+3-kz,3)
    const int64_t Mz = M - kz;  // layer side
    return choose3(M + 3) - choose3(M + 3 - kz) + (int64_t)ky * (Mz + 1) - (int64_t)ky * (ky - 1) / 2 + kx;
}

// Samples of one point (Sec. 4.1, reading of the garbled formula): for every
// fitted direction whose sample set S_d holds p (p = shift_d mod stride
// componentwise, shift_d = 1 - min(d, 0), and p + d interior), val[f] (the
// lower directions, then the centre) at its lexicographic position
// k = (p - shift)/stride in the lattice simplex of S_d.
__device__ __forceinline__ void put_samples(const TetDev& T, int x, int y, int z, const double (&val)[NFIT],
                                            double* __restrict__ samples) {
    const int n = T.n, st = T.stride;
    for (int f = 0; f < NFIT; ++f) {
        const int dx = f < NLOW ? low_dx(f) : 0, dy = f < NLOW ? low_dy(f) : 0, dz = f < NLOW ? low_dz(f) : 0;
        const int sx = 1 - (dx < 0 ? dx : 0), sy = 1 - (dy < 0 ? dy : 0), sz = 1 - (dz < 0 ? dz : 0);
        if ((x - sx) % st || (y - sy) % st || (z - sz) % st) continue;
        if (!interior(n, x + dx, y + dy, z + dz)) continue;
        const int kx = (x - sx) / st, ky = (y - sy) / st, kz = (z - sz) / st;
        samples[T.samp_off[f] + simplex_index(T.samp_M[f], kx, ky, kz)] = val[f];
    }
}

// Alg. 1 in O(h^-2) memory (surrogate variants): the factors of hyperplane t
// go to slot t mod 4 of a ring of four hyperplanes, ring[(k * 4 + slot) *
// nring + global lane], k = 0..6 the lower factors and 7 the pivot, nring =
// lanes + 1 (the last lane is zero and stands for rows outside the lattice);
// the stencil equations at t read t-1 .. t-3 only.  Each factored point
// leaves its samples (L^p_d, 1/D^p) and, variant V1, its boundary record
// [L_0..L_6, 1/D] right away, so no full factor array is ever held.  Without
// an assembled stencil (A8 null: the surrogate operator) the point's stencil
// row is computed here, as the assembly would, and its samples (A^p_d, A^p_c)
// go to asamples: then the whole setup holds no O(h^-3) array.
template <typename FT>
__global__ void __launch_bounds__(64) k_factor_ring(const TetDev* __restrict__ tets, const BlockDev* __restrict__ blocks,
                              const LaneDev* __restrict__ lanes, int lpb, int groups, int t_glob, int64_t S,
                              const double* __restrict__ A8, double* __restrict__ ring, int64_t nring,
                              double* __restrict__ samples, double* __restrict__ asamples, FT* __restrict__ F,
                              int* __restrict__ flags) {
    int b, lane;
    decode_group(groups, b, lane);
    const BlockDev& B = blocks[b];
    const int t = t_glob;
    if (t < B.tb || t > B.te) return;
    const LaneDev& Ln = lanes[(int64_t)b * lpb + lane];
    if (Ln.v == 0) return;
    const TetDev& T = tets[B.tet];
    const int n = T.n, v = Ln.v, w = Ln.w, y = v - w, z = w, xmax = n - 1 - v;
    const int x = t - 2 * v - w;
    if (x < 1 || x > xmax) return;
    const int64_t idx = Ln.rp[R_SELF] + (int64_t)lpb * t;
    int64_t q[NLOW];
    bool in[NLOW];
    double Dn[NLOW], a[NLOW], Ac;
    double Ad[15];
    if (!A8)
        stencil_row(T.J, T.v0, 1.0 / n, x, y, z, [&](double X, double Y, double Z) { return kappa_at(T, X, Y, Z); },
                    Ad);
#pragma unroll
    for (int s = 0; s < NLOW; ++s) {
        const int32_t g = Ln.gl[low_row(s)];
        const int slot = (t + low_dt(s)) & 3;
        q[s] = (int64_t)slot * nring + (g >= 0 ? g : nring - 1);
        in[s] = interior(n, x + low_dx(s), y + low_dy(s), z + low_dz(s));
        Dn[s] = in[s] ? ring[(int64_t)7 * 4 * nring + q[s]] : 1.0;
        a[s] = A8 ? A8[(int64_t)(1 + s) * S + idx] : (in[s] ? Ad[s] : 0.0);
    }
    Ac = A8 ? A8[idx] : Ad[7];
    auto Lq = [&](int s, int d) -> double { return in[s] ? ring[(int64_t)d * 4 * nring + q[s]] : 0.0; };
    double Lp[NLOW], Dp;
    stencil_equations(a, Ac, Dn, Lq, Lp, Dp);
#pragma unroll
    for (int s = 0; s < NLOW; ++s) Lp[s] = in[s] ? Lp[s] : 0.0;
    const int64_t me = (int64_t)(t & 3) * nring + Ln.gl[R_SELF];
#pragma unroll
    for (int s = 0; s < NLOW; ++s) ring[(int64_t)s * 4 * nring + me] = Lp[s];
    ring[(int64_t)7 * 4 * nring + me] = Dp;
    if (!(Dp > 0.0)) atomicOr(&flags[0], 1);
    if (samples) {
        double val[NFIT];
#pragma unroll
        for (int s = 0; s < NLOW; ++s) val[s] = Lp[s];
        val[NLOW] = 1.0 / Dp;
        put_samples(T, x, y, z, val, samples);
    }
    if (asamples) {
        double val[NFIT];
#pragma unroll
        for (int s = 0; s < NLOW; ++s) val[s] = a[s];
        val[NLOW] = Ac;
        put_samples(T, x, y, z, val, asamples);
    }
    if (F) {
        const int k = v1f_pos(x, xmax, y, z);
        if (k >= 0) {
            const int64_t j = (int64_t)Ln.v1f[0] + k;
#pragma unroll
            for (int s = 0; s < NLOW; ++s) F[j * 8 + s] = (FT)Lp[s];
            F[j * 8 + NLOW] = (FT)(1.0 / Dp);
        }
    }
}

// ------------------------------------------------------------ least squares

// P_a(s) of the shifted Legendre recurrence (the values legendre() tabulates).
__device__ __forceinline__ double legendre_at(double s, int a) {
    if (a == 0) return 1.0;
    double pm = 1.0, p = s;
    for (int k = 1; k < a; ++k) {
        const double pn = ((2 * k + 1) * s * p - k * pm) / (k + 1);
        pm = p;
        p = pn;
    }
    return p;
}

// Streaming Householder QR of the rows of one least-squares problem (FP64),
// as in TSQR with flat trees: a run of rows is taken QR_ROWS at a time as a
// block B under the triangular factor R of the rows before it, and [R; B] is
// reduced to the new R by m reflectors that each touch one row of R and all
// rows of B (R's structure below the diagonal is kept).  Reflector j:
// x = [R_jj; B_:j], beta = -sign(R_jj) |x|, v = [1; B_:j / (R_jj - beta)],
// tau = (beta - R_jj) / beta; every column k > j gets s = R_jk + v^T B_:k,
// R_jk -= tau s, B_:k -= tau s v.
// Thread k owns column k: its QR_ROWS entries of B in registers and its
// entries of R in the run's output slot (m x m, row-major, zeros below the
// diagonal), so R needs no synchronisation; reflector j's v is passed through
// shared memory by thread j (double-buffered: one barrier per reflector).
// Level 0 builds the rows from the samples ([basis values | sample value] at
// the sample points), later levels read the stacked R factors of the level
// before.  Each run leaves its R; stacking them and reducing again gives the
// R of the whole problem.
constexpr int QR_ROWS = 32;  // rows per block
constexpr int QR_MAXM = 512; // columns (threads per workgroup) at most

__global__ void __launch_bounds__(QR_MAXM) k_qr_stream(const TetDev* __restrict__ tets,
                                                       const QrJob* __restrict__ jobs, int njobs, int level0, int m,
                                                       const double* __restrict__ samples,
                                                       const double* __restrict__ in, double* __restrict__ out,
                                                       int nruns) {
    __shared__ double vbuf[2][QR_ROWS];
    __shared__ double taus[2];
    __shared__ double pts[QR_ROWS][4];  // level 0: rescaled sample point and value of each block row
    const int k = (int)threadIdx.x;
    const bool col = k < m;
    for (int cid = blockIdx.x; cid < nruns; cid += gridDim.x) {
        int lo = 0, hi = njobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (jobs[mid].chunk0 <= cid) lo = mid; else hi = mid - 1;
        }
        const QrJob J = jobs[lo];
        const int c = cid - J.chunk0;
        const int64_t rbeg = (int64_t)c * J.run_rows, rend = min<int64_t>(J.in_rows, rbeg + J.run_rows);
        double* R = out + (J.out_off + (int64_t)c * m) * m;
        if (col)
            for (int r = 0; r < m; ++r) R[(int64_t)r * m + k] = 0.0;
        // the basis function of column k (level 0): Legendre degrees (i, j, l)
        // with x fastest, the last column is the sample value
        const TetDev& T = tets[J.tet];
        const int nx = T.deg[0] + 1, ny = T.deg[1] + 1;
        const int bi = k % nx, bj = (k / nx) % ny, bl = k / (nx * ny);
        for (int64_t p0 = rbeg; p0 < rend; p0 += QR_ROWS) {
            const int nb = (int)min<int64_t>(QR_ROWS, rend - p0);
            double Bc[QR_ROWS];
            if (level0) {
                if (k < nb) {
                    const int M = T.samp_M[J.fit];
                    const int dx = J.fit < NLOW ? low_dx(J.fit) : 0, dy = J.fit < NLOW ? low_dy(J.fit) : 0,
                              dz = J.fit < NLOW ? low_dz(J.fit) : 0;
                    const int sx = 1 - (dx < 0 ? dx : 0), sy = 1 - (dy < 0 ? dy : 0), sz = 1 - (dz < 0 ? dz : 0);
                    // decode the lexicographic simplex index back to the lattice point
                    int64_t si = p0 + k;
                    const double val = samples[J.in_off + si];
                    int kz = 0;
                    while (choose3(M + 3) - choose3(M + 3 - (kz + 1)) <= si) ++kz;
                    si -= choose3(M + 3) - choose3(M + 3 - kz);
                    const int Mz = M - kz;
                    int ky = 0;
                    while ((int64_t)(ky + 1) * (Mz + 1) - (int64_t)(ky + 1) * ky / 2 <= si) ++ky;
                    si -= (int64_t)ky * (Mz + 1) - (int64_t)ky * (ky - 1) / 2;
                    const int kx = (int)si;
                    const double invn = 1.0 / T.n;
                    pts[k][0] = 2 * ((sx + T.stride * kx) * invn) - 1;
                    pts[k][1] = 2 * ((sy + T.stride * ky) * invn) - 1;
                    pts[k][2] = 2 * ((sz + T.stride * kz) * invn) - 1;
                    pts[k][3] = val;
                }
                __syncthreads();
#pragma unroll
                for (int i = 0; i < QR_ROWS; ++i) {
                    double v = 0.0;
                    if (col && i < nb)
                        v = k == m - 1 ? pts[i][3]
                                       : legendre_at(pts[i][0], bi) * legendre_at(pts[i][1], bj) *
                                             legendre_at(pts[i][2], bl);
                    Bc[i] = v;
                }
                __syncthreads();
            } else {
                const int kc = col ? k : 0;
#pragma unroll
                for (int i = 0; i < QR_ROWS; ++i)
                    Bc[i] = (col && i < nb) ? in[(J.in_off + p0 + i) * m + kc] : 0.0;
            }
            // R_jk for the next four reflectors, loaded ahead (row j of R
            // changes only under reflector j, and only thread k touches
            // column k); unconditional loads at a clamped row, and four
            // registers in turn, so each wait covers the load of four
            // reflectors ago only
            const int kc = col ? k : 0;
            auto rload = [&](int r) { return R[(int64_t)min(r, m - 1) * m + kc]; };
            auto reflect = [&](int j, double rjk) {
                const int buf = j & 1;
                if (k == j) {
                    // four partial sums: the chain is on the critical path of every reflector
                    double sp[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int i = 0; i < QR_ROWS; ++i) sp[i & 3] += Bc[i] * Bc[i];
                    const double sg = (sp[0] + sp[1]) + (sp[2] + sp[3]);
                    double tau = 0.0;
                    if (sg != 0.0) {  // else the column is already reduced: H = I
                        const double alpha = rjk;
                        const double nrm = sqrt(alpha * alpha + sg);
                        const double beta = alpha > 0.0 ? -nrm : nrm;
                        tau = (beta - alpha) / beta;
                        const double scl = 1.0 / (alpha - beta);
#pragma unroll
                        for (int i = 0; i < QR_ROWS; ++i) vbuf[buf][i] = Bc[i] * scl;
                        R[(int64_t)j * m + j] = beta;
                    }
                    taus[buf] = tau;
                }
                lds_barrier();  // v and tau of reflector j; R and B stay private to their threads
                const double tau = taus[buf];
                if (col && k > j && tau != 0.0) {
                    double sp[4] = {rjk, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int i = 0; i < QR_ROWS; ++i) sp[i & 3] += vbuf[buf][i] * Bc[i];
                    const double sv = ((sp[0] + sp[1]) + (sp[2] + sp[3])) * tau;
                    R[(int64_t)j * m + k] = rjk - sv;
#pragma unroll
                    for (int i = 0; i < QR_ROWS; ++i) Bc[i] -= sv * vbuf[buf][i];
                }
            };
            double ra = rload(0), rb = rload(1), rc = rload(2), rd = rload(3);
            for (int j = 0; j < m; j += 4) {
                reflect(j, ra);
                ra = rload(j + 4);
                if (j + 1 < m) reflect(j + 1, rb);
                rb = rload(j + 5);
                if (j + 2 < m) reflect(j + 2, rc);
                rc = rload(j + 6);
                if (j + 3 < m) reflect(j + 3, rd);
                rd = rload(j + 7);
            }
            __syncthreads();
        }
    }
}

// Back substitution R[:K,:K] c = R[:K,K] for every problem (one thread each),
// with a rank test on the diagonal of R.
__global__ void k_qr_solve(const QrJob* __restrict__ jobs, int njobs, int m, const double* __restrict__ Rall,
                           double* __restrict__ coef, int* __restrict__ flags) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= njobs) return;
    const QrJob J = jobs[p];
    const double* R = Rall + J.out_off * m;
    const int K = m - 1;
    double dmax = 0.0, dmin = INFINITY;
    for (int i = 0; i < K; ++i) {
        const double d = fabs(R[(int64_t)i * m + i]);
        dmax = fmax(dmax, d);
        dmin = fmin(dmin, d);
    }
    double* c = coef + ((int64_t)J.tet * NFIT + J.fit) * K;
    if (!(dmin > 1e-15 * dmax)) {
        atomicOr(&flags[1], 1);
        for (int i = 0; i < K; ++i) c[i] = 0.0;
        return;
    }
    for (int i = K - 1; i >= 0; --i) {
        double s = R[(int64_t)i * m + K];
        for (int j = i + 1; j < K; ++j) s -= R[(int64_t)i * m + j] * c[j];
        c[i] = s / R[(int64_t)i * m + i];
    }
}

// ------------------------------------------------------- evaluation tables

// Per row (y, z) and per sweep, the surrogate restricted to the row as a
// polynomial in eta = (x - xm) / hw, the row's x-range [1, n-1-y-z] mapped to
// [-1, 1]:  coefficients of eta^0..eta^dgx (Horner in the sweeps).
//   forward table  [7][NC]: L_d at (x, y, z)                 (d in D_l)
//   backward table [8][NC]: 1/D at (x, y, z), then L_d at p - d
// Row record layout: [xm, 1/hw, fwd 7*NC, bwd 8*NC].
__global__ void __launch_bounds__(128) k_row_tables(const TetDev* __restrict__ tets, const BlockDev* __restrict__ blocks,
                             const LaneDev* __restrict__ lanes, int lpb, int groups, int nslots, const double* __restrict__ coef,
                             int NC, double* __restrict__ tab, float* __restrict__ tab32) {
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= nslots) return;
    const LaneDev& Ln = lanes[slot];
    const int rec = 2 + 15 * NC;
    double* o = tab + (int64_t)slot * rec;
    if (Ln.v == 0) {
        for (int k = 0; k < rec; ++k) o[k] = 0.0;
        if (tab32)
            for (int k = 0; k < rec; ++k) tab32[(int64_t)slot * rec + k] = 0.f;
        return;
    }
    const BlockDev& B = blocks[slot / lpb];
    const TetDev& T = tets[B.tet];
    const int n = T.n, y = Ln.v - Ln.w, z = Ln.w;
    const int dgx = T.deg[0], dgy = T.deg[1], dgz = T.deg[2];
    const int K = (dgx + 1) * (dgy + 1) * (dgz + 1);
    const double xlo = 1.0, xhi = n - 1 - Ln.v;
    const double xm = 0.5 * (xlo + xhi);
    const double hw = xhi > xlo ? 0.5 * (xhi - xlo) : 1.0;
    o[0] = xm;
    o[1] = 1.0 / hw;
    for (int e = 0; e < 15; ++e) {
        // entry e < 7: forward L_e at own row; e == 7: 1/D; e > 7: L_{e-8} at p - d
        const int fit = e < 7 ? e : e == 7 ? 7 : e - 8;
        int sx = 0, sy = 0, sz = 0;
        if (e > 7) { sx = low_dx(e - 8); sy = low_dy(e - 8); sz = low_dz(e - 8); }
        const double* a = coef + ((int64_t)B.tet * NFIT + fit) * K;
        double py[9], pz[9];
        legendre(2.0 * (y - sy) / n - 1.0, dgy, py);
        legendre(2.0 * (z - sz) / n - 1.0, dgz, pz);
        double cx[9];
        for (int i = 0; i <= dgx; ++i) cx[i] = 0.0;
        for (int kk = 0; kk <= dgz; ++kk)
            for (int j = 0; j <= dgy; ++j) {
                const double wgt = py[j] * pz[kk];
                for (int i = 0; i <= dgx; ++i) cx[i] += a[(kk * (dgy + 1) + j) * (dgx + 1) + i] * wgt;
            }
        // s = 2 (x - sx)/n - 1 = alpha + beta eta
        const double alpha = 2.0 * (xm - sx) / n - 1.0, beta = 2.0 * hw / n;
        double Pm1[9], P0[9], P1[9], out[9];
        for (int i = 0; i < 9; ++i) { Pm1[i] = 0.0; P0[i] = 0.0; out[i] = 0.0; }
        P0[0] = 1.0;  // P_0
        for (int i = 0; i <= dgx; ++i) out[i] = 0.0;
        out[0] += cx[0];
        if (dgx >= 1) {
            for (int i = 0; i < 9; ++i) { Pm1[i] = P0[i]; P0[i] = 0.0; }
            P0[0] = alpha;
            P0[1] = beta;  // P_1
            for (int i = 0; i <= 1; ++i) out[i] += cx[1] * P0[i];
            for (int k = 1; k < dgx; ++k) {
                // P_{k+1} = ((2k+1) s P_k - k P_{k-1}) / (k+1)
                for (int i = 0; i < 9; ++i) P1[i] = -k * Pm1[i];
                for (int i = 0; i <= k; ++i) {
                    P1[i] += (2 * k + 1) * alpha * P0[i];
                    P1[i + 1] += (2 * k + 1) * beta * P0[i];
                }
                for (int i = 0; i < 9; ++i) { P1[i] /= (k + 1); Pm1[i] = P0[i]; P0[i] = P1[i]; }
                for (int i = 0; i <= k + 1; ++i) out[i] += cx[k + 1] * P0[i];
            }
        }
        for (int i = 0; i < NC; ++i) o[2 + e * NC + i] = i <= dgx ? out[i] : 0.0;
    }
    if (tab32)
        for (int k = 0; k < rec; ++k) tab32[(int64_t)slot * rec + k] = (float)o[k];
}

// ------------------------------------------------------- boundary variant V1

__device__ __forceinline__ double horner_d(const double* c, int NC, double eta) {
    double acc = c[NC - 1];
    for (int i = NC - 2; i >= 0; --i) acc = acc * eta + c[i];
    return acc;
}

// Backward weights of the points of set B: [1/D^p, L^{p-d}_d for d in D_l],
// each the exact factor (from F) where the point holding it is in F, else the
// surrogate evaluated from the FP64 row table (0 where p - d is not interior).
template <typename T>
__global__ void k_build_v1b(const TetDev* __restrict__ tets, const BlockDev* __restrict__ blocks,
                            const LaneDev* __restrict__ lanes, int lpb, int groups, const double* __restrict__ tab,
                            int NC, const T* __restrict__ F, T* __restrict__ Bw) {
    int b, lane;
    decode_group(groups, b, lane);
    const BlockDev B = blocks[b];
    const LaneDev& Ln = lanes[(int64_t)b * lpb + lane];
    if (Ln.v == 0) return;
    const int n = tets[B.tet].n, v = Ln.v, w = Ln.w, y = v - w, z = w, xmax = n - 1 - v;
    const double* c = tab + ((int64_t)b * lpb + lane) * (2 + 15 * NC);
    for (int t = B.tb + (int)(threadIdx.x >> 6); t <= B.te; t += (int)(blockDim.x >> 6)) {
        const int x = t - 2 * v - w;
        if (x < 1 || x > xmax) continue;
        const int k = v1b_pos(x, xmax, y, z);
        if (k < 0) continue;
        const int64_t j = (int64_t)Ln.v1b + k;
        const double eta = ((double)x - c[0]) * c[1];
        const int kf = v1f_pos(x, xmax, y, z);
        Bw[j * 8] = kf >= 0 ? F[((int64_t)Ln.v1f[0] + kf) * 8 + NLOW] : (T)horner_d(c + 2 + 7 * NC, NC, eta);
        for (int s = 0; s < NLOW; ++s) {
            const int xq = x - low_dx(s), yq = y - low_dy(s), zq = z - low_dz(s);
            T val = (T)0;
            if (interior(n, xq, yq, zq)) {
                // row of p - d_s: own (s = 0), v+1 (s, se), w+1 (bnw, bn), v+1 w+1 (bc, be)
                const int fr = s == 0 ? 0 : s <= 2 ? 1 : s <= 4 ? 2 : 3;
                const int kq = v1f_pos(xq, n - 1 - yq - zq, yq, zq);
                val = kq >= 0 ? F[((int64_t)Ln.v1f[fr] + kq) * 8 + s] : (T)horner_d(c + 2 + (8 + s) * NC, NC, eta);
            }
            Bw[j * 8 + 1 + s] = val;
        }
    }
}

// ------------------------------------------------------------ lex <-> stream

// NV vectors (1 or 2: x and b at once), lexicographic <-> stream, through an
// LDS tile of PT_T hyperplanes x the 64 rows of a workgroup (256 threads) per
// vector.  On the stream side a wave moves one hyperplane of all 64 rows per
// access (one 512-byte run); on the lexicographic side half a wave moves PT_T
// consecutive points of one row (x = t - 2v - w, so row (v, w) is contiguous
// in t).  MODE 0: stream -> lex, MODE 1: lex -> stream.
constexpr int PT_T = 32;
template <int MODE, int NV>
__global__ __launch_bounds__(256) void k_permute_tile(const TetDev* __restrict__ tets,
                                                      const BlockDev* __restrict__ blocks,
                                                      const LaneDev* __restrict__ lanes, int lpb, int groups,
                                                      const double* __restrict__ src0, double* __restrict__ dst0,
                                                      const double* __restrict__ src1, double* __restrict__ dst1,
                                                      int only_tet) {
    __shared__ double tile[NV][PT_T][WAVE + 1];
    const double* const src[2] = {src0, src1};
    double* const dst[2] = {dst0, dst1};
    __shared__ int64_t s_lrow[WAVE], s_srow[WAVE];
    __shared__ int s_lo[WAVE], s_hi[WAVE];
    int b, lane;
    decode_group(groups, b, lane);
    const BlockDev B = blocks[b];
    if (only_tet >= 0 && B.tet != only_tet) return;  // the whole workgroup
    const int l = (int)(threadIdx.x & (WAVE - 1)), wv = (int)(threadIdx.x >> 6);
    if (wv == 0) {
        // row (v, w) holds x = t - 2v - w in [1, n-1-v]: t in [lo, hi], at
        // lexicographic index lrow + t and stream index srow + lpb t
        const LaneDev& Ln = lanes[(int64_t)b * lpb + lane];
        int lo = 1, hi = 0;
        int64_t lrow = 0, srow = 0;
        if (Ln.v != 0) {
            const TetDev& T = tets[B.tet];
            const int n = T.n, v = Ln.v, w = Ln.w;
            lo = max(B.tb, 2 * v + w + 1);
            hi = min(B.te, n - 1 + v + w);
            lrow = (only_tet >= 0 ? 0 : T.lex_off) + lex_index(n, 1, v - w, w) - 1 - (2 * v + w);
            srow = Ln.rp[R_SELF];
        }
        s_lo[l] = lo;
        s_hi[l] = hi;
        s_lrow[l] = lrow;
        s_srow[l] = srow;
    }
    __syncthreads();
    // stream side: row l, hyperplanes wv + 4k of the tile
    const int slo = s_lo[l], shi = s_hi[l];
    const int64_t srow = s_srow[l];
    // lexicographic side: rows r0 + 8k, hyperplane tx of the tile
    constexpr int RK = WAVE / 8;
    const int tx = (int)(threadIdx.x & (PT_T - 1)), r0 = (int)(threadIdx.x >> 5);
    int llo[RK], lhi[RK];
    int64_t lrow[RK];
#pragma unroll
    for (int k = 0; k < RK; ++k) {
        llo[k] = s_lo[r0 + 8 * k];
        lhi[k] = s_hi[r0 + 8 * k];
        lrow[k] = s_lrow[r0 + 8 * k];
    }
    constexpr int SK = PT_T / 4;
    for (int t0 = B.tb; t0 <= B.te; t0 += PT_T) {
        static_assert(RK == 8 && SK == 8, "one register per access of either side");
        double val[NV][8];
        if (MODE == 1) {
            const int t = t0 + tx;
#pragma unroll
            for (int q = 0; q < NV; ++q)
#pragma unroll
                for (int k = 0; k < RK; ++k) val[q][k] = t >= llo[k] && t <= lhi[k] ? src[q][lrow[k] + t] : 0.0;
#pragma unroll
            for (int q = 0; q < NV; ++q)
#pragma unroll
                for (int k = 0; k < RK; ++k) tile[q][tx][r0 + 8 * k] = val[q][k];
            __syncthreads();
#pragma unroll
            for (int q = 0; q < NV; ++q)
#pragma unroll
                for (int k = 0; k < SK; ++k) {
                    const int t = t0 + wv + 4 * k;
                    if (t >= slo && t <= shi) dst[q][srow + (int64_t)lpb * t] = tile[q][wv + 4 * k][l];
                }
        } else {
#pragma unroll
            for (int q = 0; q < NV; ++q)
#pragma unroll
                for (int k = 0; k < SK; ++k) {
                    const int t = t0 + wv + 4 * k;
                    val[q][k] = t >= slo && t <= shi ? src[q][srow + (int64_t)lpb * t] : 0.0;
                }
#pragma unroll
            for (int q = 0; q < NV; ++q)
#pragma unroll
                for (int k = 0; k < SK; ++k) tile[q][wv + 4 * k][l] = val[q][k];
            __syncthreads();
            const int t = t0 + tx;
#pragma unroll
            for (int q = 0; q < NV; ++q)
#pragma unroll
                for (int k = 0; k < RK; ++k)
                    if (t >= llo[k] && t <= lhi[k]) dst[q][lrow[k] + t] = tile[q][tx][r0 + 8 * k];
        }
        __syncthreads();
    }
}

// mode 0: stream -> lex (dst[lex] = src[stream]); mode 1: lex -> stream.
// Stencil/factor exports use `count` arrays spaced `sstride` / `lstride` apart
// (one vector goes through k_permute_tile).
__global__ void k_permute(const TetDev* __restrict__ tets, const BlockDev* __restrict__ blocks,
                          const LaneDev* __restrict__ lanes, int lpb, int groups, int mode, int count, const double* __restrict__ src,
                          double* __restrict__ dst, int64_t sstride, int lmul, int only_tet) {
    int b, lane;
    decode_group(groups, b, lane);
    const BlockDev B = blocks[b];
    if (only_tet >= 0 && B.tet != only_tet) return;
    const LaneDev& Ln = lanes[(int64_t)b * lpb + lane];
    if (Ln.v == 0) return;
    const TetDev& T = tets[B.tet];
    const int n = T.n, v = Ln.v, w = Ln.w, y = v - w, z = w;
    const int64_t lexbase = only_tet >= 0 ? 0 : T.lex_off;
    for (int t = B.tb + (int)(threadIdx.x >> 6); t <= B.te; t += (int)(blockDim.x >> 6)) {
        const int x = t - 2 * v - w;
        if (x < 1 || x > n - 1 - v) continue;
        const int64_t si = Ln.rp[R_SELF] + (int64_t)lpb * t;
        const int64_t li = lexbase + lex_index(n, x, y, z);
        for (int k = 0; k < count; ++k) {
            if (mode == 0) dst[li * lmul + k] = src[k * sstride + si];
            else dst[k * sstride + si] = src[li * lmul + k];
        }
    }
}

}  // namespace ilu

namespace ilu {

void launch_assemble(const Ctx& c, double* A8, double* Afull, hipStream_t st) {
    k_assemble<<<c.nblocks * c.groups, 256, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, c.nblocks, c.S, A8, Afull);
}

void launch_factor_plane(const Ctx& c, int t, double* Lf, double* Df, int* flags, hipStream_t st) {
    k_factor_plane<<<c.nblocks * c.groups, 64, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, t, c.S, c.A8, Lf, Df, flags);
}

void launch_factor_ring(const Ctx& c, int t, double* ring, int64_t nring, double* samples, double* asamples,
                        void* F, bool f32, int* flags, hipStream_t st) {
    if (f32)
        k_factor_ring<float><<<c.nblocks * c.groups, 64, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, t, c.S,
                                                                  c.A8, ring, nring, samples, asamples, (float*)F,
                                                                  flags);
    else
        k_factor_ring<double><<<c.nblocks * c.groups, 64, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, t, c.S,
                                                                   c.A8, ring, nring, samples, asamples, (double*)F,
                                                                   flags);
}

void launch_transpose(const Ctx& c, const double* Lf, const double* Df, double* Lb, hipStream_t st) {
    k_transpose_factors<<<c.nblocks * c.groups, 256, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, c.S, Lf, Df, Lb);
}

void launch_qr_stream(const Ctx& c, const QrJob* jobs, int njobs, int level0, int m, const double* samples,
                      const double* in, double* out, int grid, int nruns, hipStream_t st) {
    const int threads = (m + 63) / 64 * 64;
    k_qr_stream<<<grid, threads, 0, st>>>(c.tets, jobs, njobs, level0, m, samples, in, out, nruns);
}

void launch_qr_solve(const QrJob* jobs, int njobs, int m, const double* R, double* coef, int* flags, hipStream_t st) {
    k_qr_solve<<<(njobs + 63) / 64, 64, 0, st>>>(jobs, njobs, m, R, coef, flags);
}

void launch_row_tables(const Ctx& c, int nslots, const double* coef, int NC, double* tab, float* tab32, hipStream_t st) {
    k_row_tables<<<(nslots + 127) / 128, 128, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, nslots, coef, NC, tab, tab32);
}

void launch_build_v1b(const Ctx& c, const double* tab, const void* F, void* Bw, bool f32, hipStream_t st) {
    if (f32)
        k_build_v1b<float><<<c.nblocks * c.groups, 256, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, tab, c.NC,
                                                                 (const float*)F, (float*)Bw);
    else
        k_build_v1b<double><<<c.nblocks * c.groups, 256, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, tab, c.NC,
                                                                  (const double*)F, (double*)Bw);
}

void launch_permute(const Ctx& c, int mode, int count, const double* src, double* dst, int64_t sstride, int lmul,
                    int only_tet, hipStream_t st) {
    if (count == 1 && lmul == 1) {
        if (mode == 0)
            k_permute_tile<0, 1><<<c.nblocks * c.groups, 256, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, src,
                                                                       dst, nullptr, nullptr, only_tet);
        else
            k_permute_tile<1, 1><<<c.nblocks * c.groups, 256, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, src,
                                                                       dst, nullptr, nullptr, only_tet);
        return;
    }
    k_permute<<<c.nblocks * c.groups, 256, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, mode, count, src, dst, sstride, lmul, only_tet);
}

void launch_permute_in2(const Ctx& c, const double* x, double* xs, const double* b, double* bs, hipStream_t st) {
    k_permute_tile<1, 2><<<c.nblocks * c.groups, 256, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, x, xs, b, bs,
                                                               -1);
}


}  // namespace ilu
