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
__global__ void k_assemble(const TetDev* __restrict__ tets, const BlockDev* __restrict__ blocks,
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
// of Alg. 1).  Factors are written to Lf[7][S] (lower weights) and Df[S].
// The first point with D <= 0 is reported through flags[0].
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

// Samples of one factored point (Sec. 4.1, reading of the garbled formula):
// for every fitted direction whose sample set S_d holds p (p = shift_d mod
// stride componentwise, shift_d = 1 - min(d, 0), and p + d interior), the
// value L^p_d (lower directions) or 1/D^p (centre) at its lexicographic
// position k = (p - shift)/stride in the lattice simplex of S_d.
__device__ __forceinline__ int64_t simplex_index(int M, int kx, int ky, int kz);
__device__ __forceinline__ void put_samples(const TetDev& T, int x, int y, int z, const double (&Lp)[NLOW], double Dp,
                                            double* __restrict__ samples) {
    const int n = T.n, st = T.stride;
    for (int f = 0; f < NFIT; ++f) {
        const int dx = f < NLOW ? low_dx(f) : 0, dy = f < NLOW ? low_dy(f) : 0, dz = f < NLOW ? low_dz(f) : 0;
        const int sx = 1 - (dx < 0 ? dx : 0), sy = 1 - (dy < 0 ? dy : 0), sz = 1 - (dz < 0 ? dz : 0);
        if ((x - sx) % st || (y - sy) % st || (z - sz) % st) continue;
        if (!interior(n, x + dx, y + dy, z + dz)) continue;
        const int kx = (x - sx) / st, ky = (y - sy) / st, kz = (z - sz) / st;
        samples[T.samp_off[f] + simplex_index(T.samp_M[f], kx, ky, kz)] = f < NLOW ? Lp[f] : 1.0 / Dp;
    }
}

// Alg. 1 in O(h^-2) memory (surrogate variants): the factors of hyperplane t
// go to slot t mod 4 of a ring of four hyperplanes, ring[(k * 4 + slot) *
// nring + global lane], k = 0..6 the lower factors and 7 the pivot, nring =
// lanes + 1 (the last lane is zero and stands for rows outside the lattice);
// the stencil equations at t read t-1 .. t-3 only.  Each factored point
// leaves its samples (and, variant V1, its boundary record [L_0..L_6, 1/D])
// right away, so no full factor array is ever held.
template <typename FT>
__global__ void k_factor_ring(const TetDev* __restrict__ tets, const BlockDev* __restrict__ blocks,
                              const LaneDev* __restrict__ lanes, int lpb, int groups, int t_glob, int64_t S,
                              const double* __restrict__ A8, double* __restrict__ ring, int64_t nring,
                              double* __restrict__ samples, FT* __restrict__ F, int* __restrict__ flags) {
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
    double Dn[NLOW], a[NLOW];
#pragma unroll
    for (int s = 0; s < NLOW; ++s) {
        const int32_t g = Ln.gl[low_row(s)];
        const int slot = (t + low_dt(s)) & 3;
        q[s] = (int64_t)slot * nring + (g >= 0 ? g : nring - 1);
        in[s] = interior(n, x + low_dx(s), y + low_dy(s), z + low_dz(s));
        Dn[s] = in[s] ? ring[(int64_t)7 * 4 * nring + q[s]] : 1.0;
        a[s] = A8[(int64_t)(1 + s) * S + idx];
    }
    auto Lq = [&](int s, int d) -> double { return in[s] ? ring[(int64_t)d * 4 * nring + q[s]] : 0.0; };
    double Lp[NLOW], Dp;
    stencil_equations(a, A8[idx], Dn, Lq, Lp, Dp);
#pragma unroll
    for (int s = 0; s < NLOW; ++s) Lp[s] = in[s] ? Lp[s] : 0.0;
    const int64_t me = (int64_t)(t & 3) * nring + Ln.gl[R_SELF];
#pragma unroll
    for (int s = 0; s < NLOW; ++s) ring[(int64_t)s * 4 * nring + me] = Lp[s];
    ring[(int64_t)7 * 4 * nring + me] = Dp;
    if (!(Dp > 0.0)) atomicOr(&flags[0], 1);
    if (samples) put_samples(T, x, y, z, Lp, Dp, samples);
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
// position (k_z slowest).  Values: L^p_d for the lower directions, 1/D^p for c.
__device__ __forceinline__ int64_t simplex_index(int M, int kx, int ky, int kz) {
    // points with k_z' < k_z: C(M+3,3) - C(M+3-kz,3)
    const int64_t Mz = M - kz;  // layer side
    return choose3(M + 3) - choose3(M + 3 - kz) + (int64_t)ky * (Mz + 1) - (int64_t)ky * (ky - 1) / 2 + kx;
}

// Samples of the assembled stencil (centre and lower weights) on the sample
// sets of the factors (the factors' own samples leave k_factor_ring).
__global__ void k_gather_a_samples(const TetDev* __restrict__ tets, const BlockDev* __restrict__ blocks,
                                   const LaneDev* __restrict__ lanes, int lpb, int groups, int64_t S,
                                   const double* __restrict__ A8, double* __restrict__ samples) {
    int b, lane;
    decode_group(groups, b, lane);
    const BlockDev B = blocks[b];
    const LaneDev& Ln = lanes[(int64_t)b * lpb + lane];
    if (Ln.v == 0) return;
    const TetDev& T = tets[B.tet];
    const int n = T.n, v = Ln.v, w = Ln.w, y = v - w, z = w, st = T.stride;
    for (int t = B.tb + (int)(threadIdx.x >> 6); t <= B.te; t += (int)(blockDim.x >> 6)) {
        const int x = t - 2 * v - w;
        if (x < 1 || x > n - 1 - v) continue;
        const int64_t idx = Ln.rp[R_SELF] + (int64_t)lpb * t;
        for (int f = 0; f < NFIT; ++f) {
            const int dx = f < NLOW ? low_dx(f) : 0, dy = f < NLOW ? low_dy(f) : 0, dz = f < NLOW ? low_dz(f) : 0;
            const int sx = 1 - (dx < 0 ? dx : 0), sy = 1 - (dy < 0 ? dy : 0), sz = 1 - (dz < 0 ? dz : 0);
            if ((x - sx) % st || (y - sy) % st || (z - sz) % st) continue;
            if (!interior(n, x + dx, y + dy, z + dz)) continue;
            const int kx = (x - sx) / st, ky = (y - sy) / st, kz = (z - sz) / st;
            const int64_t si = simplex_index(T.samp_M[f], kx, ky, kz);
            samples[T.samp_off[f] + si] = f < NLOW ? A8[(int64_t)(1 + f) * S + idx] : A8[idx];
        }
    }
}

// ------------------------------------------------------------ least squares

constexpr int QB = 8;  // Householder panel width of the chunk QR

// Sums of NV per-thread values over the workgroup (256 threads): each
// wavefront reduces by shuffles, then the four wavefront sums are added in a
// fixed order.  lds: 4 * NV doubles.  Every thread gets the sums.
template <int NV>
__device__ __forceinline__ void block_sums(double (&v)[NV], double* lds) {
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[wv * NV + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = ((lds[k] + lds[NV + k]) + lds[2 * NV + k]) + lds[3 * NV + k];
    __syncthreads();
}

// Householder QR of chunks of rows, one workgroup per chunk, FP64.  A chunk
// is copied into the workgroup's row-major scratch (rows x m, zero-padded),
// reduced in place, and its m x m triangular factor R is written as m rows of
// the output.  Stacking the R factors of the chunks and factoring again yields
// the R of the whole least-squares matrix (TSQR).
// Level 0 streams: chunk c of a problem is a run of `run_pieces` pieces of
// chunk_rows - m sample rows ([basis values | sample value]); each piece is
// stacked under the R of the run so far (the first under zeros) and the stack
// is factored again, so a run leaves one R however many samples it covers.
// Later levels read stacked R factors, chunk_rows of them per chunk.
__global__ void __launch_bounds__(256) k_qr_chunks(const TetDev* __restrict__ tets, const QrJob* __restrict__ jobs,
                                                   int njobs, int level0, int m, int chunk_rows, int run_pieces,
                                                   const double* __restrict__ samples, const double* __restrict__ in,
                                                   double* __restrict__ out, double* __restrict__ scratch_all,
                                                   int nchunks_total) {
    extern __shared__ double sh[];  // reduction scratch
    for (int cid = blockIdx.x; cid < nchunks_total; cid += gridDim.x) {
        // locate job
        int lo = 0, hi = njobs - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (jobs[mid].chunk0 <= cid) lo = mid; else hi = mid - 1;
        }
        const QrJob J = jobs[lo];
        const int c = cid - J.chunk0;
        double* A = scratch_all + (int64_t)blockIdx.x * chunk_rows * m;
        const int pr = level0 ? chunk_rows - m : chunk_rows;  // new rows per piece
        const int64_t rbeg = level0 ? (int64_t)c * run_pieces * pr : (int64_t)c * chunk_rows;
        const int64_t rend = level0 ? min<int64_t>(J.in_rows, rbeg + (int64_t)run_pieces * pr)
                                    : min<int64_t>(J.in_rows, rbeg + chunk_rows);
        for (int64_t p0 = rbeg; p0 < rend; p0 += pr) {
        // fill
        if (level0) {
            const TetDev& T = tets[J.tet];
            const int K = m - 1;
            const int dgx = T.deg[0], dgy = T.deg[1], dgz = T.deg[2];
            const int M = T.samp_M[J.fit];
            const int dx = J.fit < NLOW ? low_dx(J.fit) : 0, dy = J.fit < NLOW ? low_dy(J.fit) : 0,
                      dz = J.fit < NLOW ? low_dz(J.fit) : 0;
            const int sx = 1 - (dx < 0 ? dx : 0), sy = 1 - (dy < 0 ? dy : 0), sz = 1 - (dz < 0 ? dz : 0);
            const double invn = 1.0 / T.n;
            // the R of the run so far (zeros before the first piece): clear
            // the reflectors left below its diagonal
            for (int64_t e = threadIdx.x; e < (int64_t)m * m; e += blockDim.x) {
                const int r = (int)(e / m), k = (int)(e % m);
                if (p0 == rbeg || k < r) A[e] = 0.0;
            }
            for (int r = m + threadIdx.x; r < chunk_rows; r += blockDim.x) {
                double* row = A + (int64_t)r * m;
                int64_t si = p0 + (r - m);
                if (si >= rend) {
                    for (int k = 0; k < m; ++k) row[k] = 0.0;
                    continue;
                }
                const double val = samples[J.in_off + si];
                // decode the lexicographic simplex index back to k
                int kz = 0;
                while (choose3(M + 3) - choose3(M + 3 - (kz + 1)) <= si) ++kz;
                si -= choose3(M + 3) - choose3(M + 3 - kz);
                const int Mz = M - kz;
                int ky = 0;
                while ((int64_t)(ky + 1) * (Mz + 1) - (int64_t)(ky + 1) * ky / 2 <= si) ++ky;
                si -= (int64_t)ky * (Mz + 1) - (int64_t)ky * (ky - 1) / 2;
                const int kx = (int)si;
                const double X = (sx + T.stride * kx) * invn, Y = (sy + T.stride * ky) * invn,
                             Z = (sz + T.stride * kz) * invn;
                double px[9], py[9], pz[9];
                legendre(2 * X - 1, dgx, px);
                legendre(2 * Y - 1, dgy, py);
                legendre(2 * Z - 1, dgz, pz);
                int col = 0;
                for (int kk = 0; kk <= dgz; ++kk)
                    for (int j = 0; j <= dgy; ++j)
                        for (int i = 0; i <= dgx; ++i) row[col++] = px[i] * py[j] * pz[kk];
                row[K] = val;
            }
        } else {
            const int nr = (int)(rend - rbeg);
            for (int64_t e = threadIdx.x; e < (int64_t)chunk_rows * m; e += blockDim.x) {
                const int r = (int)(e / m), k = (int)(e % m);
                A[e] = r < nr ? in[(J.in_off + rbeg + r) * m + k] : 0.0;
            }
        }
        __syncthreads();
        const int rows = chunk_rows;
        // Blocked Householder: panels of QB columns.  Inside a panel each
        // reflector H_j = I - tau_j v_j v_j^T (v_j(j) = 1, below it the scaled
        // column, stored in place) is applied to the panel's remaining
        // columns; the panel's product H_j0 ... H_j0+b-1 = I - Y T Y^T (T upper
        // triangular) is then applied to the trailing columns at once,
        // A_k <- A_k - Y (T^T (Y^T A_k)): two passes over the trailing
        // matrix per panel instead of two per column.
        double* taus = sh;                      // [QB] reflector scales of the panel
        double* Tm = taus + QB;                 // [QB][QB] the panel's T
        double* red = Tm + QB * QB;             // [4][QB*QB] block sums
        const int NTH = 256;                    // rows are split over the threads: i = tid (mod 256)
        const int tid = (int)threadIdx.x;
        for (int j0 = 0; j0 < m && j0 < rows; j0 += QB) {
            const int jb = min(QB, min(m, rows) - j0);
            for (int q = 0; q < jb; ++q) {
                const int j = j0 + q;
                double sg[1] = {0.0};
                for (int i = j + 1 + tid; i < rows; i += NTH) {
                    const double a = A[(int64_t)i * m + j];
                    sg[0] += a * a;
                }
                block_sums<1>(sg, red);
                const double sigma = sg[0];
                const double alpha = A[(int64_t)j * m + j];
                if (sigma == 0.0) {  // column already reduced: H = I
                    if (tid == 0) taus[q] = 0.0;
                    __syncthreads();
                    continue;
                }
                const double nrm = sqrt(alpha * alpha + sigma);
                const double beta = alpha > 0.0 ? -nrm : nrm;
                const double tau = (beta - alpha) / beta;
                const double scl = 1.0 / (alpha - beta);
                for (int i = j + 1 + tid; i < rows; i += NTH) A[(int64_t)i * m + j] *= scl;
                __syncthreads();
                // the panel's remaining columns: dots over the rows below j, then the update
                const int nk = j0 + jb - 1 - j;
                if (nk > 0) {
                    double d[QB];
#pragma unroll
                    for (int c = 0; c < QB; ++c) d[c] = 0.0;
                    for (int i = j + 1 + tid; i < rows; i += NTH) {
                        const double vi = A[(int64_t)i * m + j];
#pragma unroll
                        for (int c = 0; c < QB; ++c)
                            if (c < nk) d[c] += vi * A[(int64_t)i * m + j + 1 + c];
                    }
                    block_sums<QB>(d, red);
                    double wk[QB];
#pragma unroll
                    for (int c = 0; c < QB; ++c) wk[c] = c < nk ? tau * (A[(int64_t)j * m + j + 1 + c] + d[c]) : 0.0;
                    __syncthreads();
                    if (tid == 0)
#pragma unroll
                        for (int c = 0; c < QB; ++c)
                            if (c < nk) A[(int64_t)j * m + j + 1 + c] -= wk[c];
                    for (int i = j + 1 + tid; i < rows; i += NTH) {
                        const double vi = A[(int64_t)i * m + j];
#pragma unroll
                        for (int c = 0; c < QB; ++c)
                            if (c < nk) A[(int64_t)i * m + j + 1 + c] -= wk[c] * vi;
                    }
                }
                __syncthreads();
                if (tid == 0) {
                    taus[q] = tau;
                    A[(int64_t)j * m + j] = beta;
                }
                __syncthreads();
            }
            if (j0 + jb >= m) break;  // no trailing columns
            // T of the panel: T[q][q] = tau_q, T[0:q][q] = -tau_q T[0:q][0:q] g,
            // g[r] = v_r^T v_q, from the Gram entries of the reflectors (v_p is 0
            // above row j0+p, 1 at it, the stored column below it)
            double g[QB * QB];
#pragma unroll
            for (int e = 0; e < QB * QB; ++e) g[e] = 0.0;
            for (int i = j0 + tid; i < rows; i += NTH) {
                double y[QB];
#pragma unroll
                for (int c = 0; c < QB; ++c)
                    y[c] = c < jb ? (i > j0 + c ? A[(int64_t)i * m + j0 + c] : (i == j0 + c ? 1.0 : 0.0)) : 0.0;
#pragma unroll
                for (int pp = 0; pp < QB; ++pp)
#pragma unroll
                    for (int qq = pp + 1; qq < QB; ++qq) g[pp * QB + qq] += y[pp] * y[qq];
            }
            block_sums<QB * QB>(g, red);
            if (tid == 0) {
                for (int qq = 0; qq < jb; ++qq) {
                    double z[QB];
                    for (int pp = 0; pp < qq; ++pp) {
                        double acc = 0.0;
                        for (int r = pp; r < qq; ++r) acc += Tm[pp * QB + r] * g[r * QB + qq];
                        z[pp] = acc;
                    }
                    for (int pp = 0; pp < qq; ++pp) Tm[pp * QB + qq] = -taus[qq] * z[pp];
                    Tm[qq * QB + qq] = taus[qq];
                }
            }
            __syncthreads();
            // trailing columns, one thread per column: w = Y^T A_k, u = T^T w,
            // A_k -= Y u
            for (int k = j0 + jb + tid; k < m; k += NTH) {
                double w[QB];
#pragma unroll
                for (int c = 0; c < QB; ++c) w[c] = 0.0;
                for (int i = j0; i < rows; ++i) {
                    const double a = A[(int64_t)i * m + k];
                    const double* yr = A + (int64_t)i * m + j0;
#pragma unroll
                    for (int c = 0; c < QB; ++c) {
                        const double y = c < jb ? (i > j0 + c ? yr[c] : (i == j0 + c ? 1.0 : 0.0)) : 0.0;
                        w[c] += y * a;
                    }
                }
                double u[QB];
#pragma unroll
                for (int pp = 0; pp < QB; ++pp) {
                    double acc = 0.0;
                    for (int c = 0; c <= pp && c < jb; ++c) acc += Tm[c * QB + pp] * w[c];
                    u[pp] = pp < jb ? acc : 0.0;
                }
                for (int i = j0; i < rows; ++i) {
                    const double* yr = A + (int64_t)i * m + j0;
                    double dd = 0.0;
#pragma unroll
                    for (int c = 0; c < QB; ++c) {
                        const double y = c < jb ? (i > j0 + c ? yr[c] : (i == j0 + c ? 1.0 : 0.0)) : 0.0;
                        dd += y * u[c];
                    }
                    A[(int64_t)i * m + k] -= dd;
                }
            }
            __syncthreads();
        }
        }  // pieces
        // write R (upper triangle, zeros below)
        for (int64_t e = threadIdx.x; e < (int64_t)m * m; e += blockDim.x) {
            const int r = (int)(e / m), k = (int)(e % m);
            out[(J.out_off + (int64_t)c * m + r) * m + k] = (k >= r && r < chunk_rows) ? A[(int64_t)r * m + k] : 0.0;
        }
        __syncthreads();
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
__global__ void k_row_tables(const TetDev* __restrict__ tets, const BlockDev* __restrict__ blocks,
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

// mode 0: stream -> lex (dst[lex] = src[stream]); mode 1: lex -> stream.
// Stencil/factor exports use `count` arrays spaced `sstride` / `lstride` apart.
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

void launch_factor_ring(const Ctx& c, int t, double* ring, int64_t nring, double* samples, void* F, bool f32,
                        int* flags, hipStream_t st) {
    if (f32)
        k_factor_ring<float><<<c.nblocks * c.groups, 64, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, t, c.S,
                                                                  c.A8, ring, nring, samples, (float*)F, flags);
    else
        k_factor_ring<double><<<c.nblocks * c.groups, 64, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, t, c.S,
                                                                   c.A8, ring, nring, samples, (double*)F, flags);
}

void launch_transpose(const Ctx& c, const double* Lf, const double* Df, double* Lb, hipStream_t st) {
    k_transpose_factors<<<c.nblocks * c.groups, 256, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, c.S, Lf, Df, Lb);
}

void launch_gather_a_samples(const Ctx& c, double* samples, hipStream_t st) {
    k_gather_a_samples<<<c.nblocks * c.groups, 256, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, c.S, c.A8,
                                                             samples);
}

void launch_qr_chunks(const Ctx& c, const QrJob* jobs, int njobs, int level0, int m, int chunk_rows,
                      int run_pieces, const double* samples, const double* in, double* out, double* scratch, int grid,
                      int nchunks, hipStream_t st) {
    k_qr_chunks<<<grid, 256, (QB + QB * QB + 4 * QB * QB) * sizeof(double), st>>>(
        c.tets, jobs, njobs, level0, m, chunk_rows, run_pieces, samples, in, out, scratch, nchunks);
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
    k_permute<<<c.nblocks * c.groups, 256, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, mode, count, src, dst, sstride, lmul, only_tet);
}


}  // namespace ilu
