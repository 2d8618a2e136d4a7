// Vector kernels of libilu around the smoother: preconditioned CG with the
// ILU (stored or surrogate) as preconditioner (the CG experiment of Sec. 4.2),
// its symmetric Gauss-Seidel comparator (Sec. 2.1), and the normalisation of
// the contraction-factor power iteration.  They run over the active points of
// stream-layout vectors with the work items of the residual kernel; the CG
// scalars live in device memory, so one CG iteration is a fixed sequence of
// launches without host round trips (and can be captured in a graph).
#include <hip/hip_runtime.h>

#include "kernels_common.h"
#include "krylov_kernels.h"

namespace ilu {

namespace {

// Call f(stream index) for every active point of this thread's work item:
// the four wavefronts of a workgroup share one 64-lane group and take the
// item's hyperplanes round robin.
template <typename F>
__device__ __forceinline__ void for_active(const TetDev* __restrict__ tets, const BlockDev* __restrict__ blocks,
                                           const LaneDev* __restrict__ lanes, int lpb, const Item& it, F&& f) {
    if (!it.live) return;
    const BlockDev& B = blocks[it.blk];
    const LaneDev& Ln = lanes[(int64_t)it.blk * lpb + it.lane];
    const int t0 = B.tb + it.chunk * RES_T;
    if (Ln.v == 0 || t0 > B.te) return;
    const int n = tets[B.tet].n;
    const int t1 = min(min(B.te, t0 + RES_T - 1), Ln.gt[1]);
    for (int t = max(t0, Ln.gt[0]) + (int)(threadIdx.x >> 6); t <= t1; t += 4) {
        const int x = t - 2 * Ln.v - Ln.w;
        if (x < 1 || x > n - 1 - Ln.v) continue;
        f(Ln.rp[R_SELF] + (int64_t)lpb * t);
    }
}

// Workgroup sum (fixed order) of one value per thread into partial[id].
__device__ __forceinline__ void group_sum(double a, double* __restrict__ partial, int64_t id) {
    __shared__ double red[256];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[id] = red[0];
}

}  // namespace

#define ILU_VEC_PARAMS                                                                                     \
    const TetDev *__restrict__ tets, const BlockDev *__restrict__ blocks, const LaneDev *__restrict__ lanes, \
        int lpb, int groups, int nblocks
#define ILU_VEC_ARGS c.tets, c.blocks, c.lanes, c.lpb, c.groups, c.nblocks

__global__ void __launch_bounds__(256) k_dot(ILU_VEC_PARAMS, const double* __restrict__ a,
                                             const double* __restrict__ b, double* __restrict__ partial) {
    const Item it = res_item(groups, nblocks);
    double acc = 0.0;
    for_active(tets, blocks, lanes, lpb, it, [&](int64_t i) { acc += a[i] * b[i]; });
    group_sum(acc, partial, it.id);
}

__global__ void __launch_bounds__(256) k_scale_rsqrt(ILU_VEC_PARAMS, double* __restrict__ v,
                                                     const double* __restrict__ sc, int slot) {
    const Item it = res_item(groups, nblocks);
    const double nn = sc[slot];
    const double s = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
    for_active(tets, blocks, lanes, lpb, it, [&](int64_t i) { v[i] *= s; });
}

template <typename RT>
__global__ void __launch_bounds__(256) k_cg_update(ILU_VEC_PARAMS, double* __restrict__ x, const double* __restrict__ p,
                                                   double* __restrict__ r, const double* __restrict__ q,
                                                   double* __restrict__ z, RT* __restrict__ rs,
                                                   const double* __restrict__ sc, double* __restrict__ partial) {
    const Item it = res_item(groups, nblocks);
    const bool live = sc[CG_DONE] == 0.0;
    const double al = live ? sc[CG_ALPHA] : 0.0;
    double acc = 0.0;
    for_active(tets, blocks, lanes, lpb, it, [&](int64_t i) {
        double ri = r[i];
        if (live) {
            x[i] += al * p[i];
            ri -= al * q[i];
            r[i] = ri;
        }
        rs[i] = (RT)ri;
        z[i] = 0.0;
        acc += ri * ri;
    });
    group_sum(acc, partial, it.id);
}

__global__ void __launch_bounds__(256) k_cg_direction(ILU_VEC_PARAMS, double* __restrict__ p,
                                                      const double* __restrict__ z, const double* __restrict__ sc) {
    const Item it = res_item(groups, nblocks);
    if (sc[CG_DONE] != 0.0) return;
    const double be = sc[CG_BETA];
    if (be == 0.0)
        for_active(tets, blocks, lanes, lpb, it, [&](int64_t i) { p[i] = z[i]; });
    else
        for_active(tets, blocks, lanes, lpb, it, [&](int64_t i) { p[i] = z[i] + be * p[i]; });
}

// The scalar recurrences of preconditioned CG (one thread).  Non-positive
// p.q or r.z (an indefinite A or C, e.g. a surrogate with D^-1 <= 0 somewhere)
// ends the iteration with CG_BREAK set.
__global__ void k_cg_scalar(double* __restrict__ sc, int step, double rel_tol, double abs_tol) {
    if (threadIdx.x != 0) return;
    const bool done = sc[CG_DONE] != 0.0;
    switch (step) {
        case CG_SETUP:
            sc[CG_TOL2] = fmax(rel_tol * rel_tol * sc[CG_BB], abs_tol * abs_tol);
            sc[CG_ALPHA] = sc[CG_BETA] = sc[CG_DONE] = sc[CG_ITERS] = sc[CG_BREAK] = sc[CG_RZ] = 0.0;
            break;
        case CG_INIT:
            sc[CG_RZ] = sc[CG_RZNEW];
            sc[CG_BETA] = 0.0;
            if (sc[CG_RR] <= sc[CG_TOL2]) sc[CG_DONE] = 1.0;
            else if (!(sc[CG_RZNEW] > 0.0)) sc[CG_DONE] = sc[CG_BREAK] = 1.0;
            break;
        case CG_STEP_ALPHA:
            if (done) break;
            if (sc[CG_PQ] > 0.0) {
                sc[CG_ALPHA] = sc[CG_RZ] / sc[CG_PQ];
            } else {
                sc[CG_ALPHA] = 0.0;
                sc[CG_DONE] = sc[CG_BREAK] = 1.0;
            }
            break;
        case CG_CHECK:
            if (done) break;
            sc[CG_ITERS] += 1.0;
            if (sc[CG_RR] <= sc[CG_TOL2]) sc[CG_DONE] = 1.0;
            break;
        case CG_STEP_BETA:
            if (done) break;
            if (sc[CG_RZNEW] > 0.0) {
                sc[CG_BETA] = sc[CG_RZNEW] / sc[CG_RZ];
                sc[CG_RZ] = sc[CG_RZNEW];
            } else {
                sc[CG_DONE] = sc[CG_BREAK] = 1.0;
            }
            break;
        default:
            break;
    }
}

// Symmetric Gauss-Seidel factors: one pass over every active point (no
// dependence between points).
__global__ void __launch_bounds__(256) k_sgs_factors(const TetDev* __restrict__ tets, const BlockDev* __restrict__ blocks,
                                                     const LaneDev* __restrict__ lanes, int lpb, int groups, int64_t S,
                                                     const double* __restrict__ A8, double* __restrict__ Lf,
                                                     double* __restrict__ Df, int* __restrict__ flags) {
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
        const double c = A8[idx];
        Df[idx] = c;
        if (!(c > 0.0)) atomicOr(&flags[0], 1);
#pragma unroll
        for (int s = 0; s < NLOW; ++s) {
            const bool in = interior(n, x + low_dx(s), y + low_dy(s), z + low_dz(s));
            const int64_t q = Ln.rp[low_row(s)] + (int64_t)lpb * (t + low_dt(s));
            Lf[(int64_t)s * S + idx] = in ? A8[(int64_t)(1 + s) * S + idx] / A8[q] : 0.0;
        }
    }
}

namespace {
dim3 item_grid(const Ctx& c) { return dim3((unsigned)(c.nblocks * c.groups), (unsigned)c.res_chunks); }
}  // namespace

void launch_dot(const Ctx& c, const double* a, const double* b, double* partial, hipStream_t st) {
    k_dot<<<item_grid(c), 256, 0, st>>>(ILU_VEC_ARGS, a, b, partial);
}

void launch_scale_rsqrt(const Ctx& c, double* v, const double* sc, int slot, hipStream_t st) {
    k_scale_rsqrt<<<item_grid(c), 256, 0, st>>>(ILU_VEC_ARGS, v, sc, slot);
}

void launch_cg_update(const Ctx& c, bool f32, double* x, const double* p, double* r, const double* q, double* z,
                      void* rs, const double* sc, double* partial, hipStream_t st) {
    if (f32) k_cg_update<float><<<item_grid(c), 256, 0, st>>>(ILU_VEC_ARGS, x, p, r, q, z, (float*)rs, sc, partial);
    else k_cg_update<double><<<item_grid(c), 256, 0, st>>>(ILU_VEC_ARGS, x, p, r, q, z, (double*)rs, sc, partial);
}

void launch_cg_direction(const Ctx& c, double* p, const double* z, const double* sc, hipStream_t st) {
    k_cg_direction<<<item_grid(c), 256, 0, st>>>(ILU_VEC_ARGS, p, z, sc);
}

void launch_cg_scalar(double* sc, int step, double rel_tol, double abs_tol, hipStream_t st) {
    k_cg_scalar<<<1, 64, 0, st>>>(sc, step, rel_tol, abs_tol);
}

void launch_sgs_factors(const Ctx& c, double* Lf, double* Df, int* flags, hipStream_t st) {
    k_sgs_factors<<<c.nblocks * c.groups, 256, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, c.S, c.A8, Lf, Df,
                                                        flags);
}

#undef ILU_VEC_PARAMS
#undef ILU_VEC_ARGS

}  // namespace ilu
