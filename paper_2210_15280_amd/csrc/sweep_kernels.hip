// Per-sweep kernels of libilu: FP64 residual (stencil matvec), the forward
// and backward substitutions of Alg. 2 on the hyperplane schedule (one launch
// per hyperplane t = x + 2y + 3z), and norm reductions.
#include <hip/hip_runtime.h>

#include "kernels_common.h"
#include "sweep_kernels.h"
#include "residual_stage.h"
#include "tagged_device.h"

namespace ilu {

// ---------------------------------------------------------------- residual

template <typename RT, bool SUB>
__global__ void __launch_bounds__(256) k_residual(const TetDev* __restrict__ tets, const BlockDev* __restrict__ blocks,
                                                  const LaneDev* __restrict__ lanes, int lpb, int groups, int nblocks,
                                                  int64_t S,
                                                  const double* __restrict__ A8, const double* __restrict__ x,
                                                  const double* __restrict__ b, RT* __restrict__ r,
                                                  double* __restrict__ partial) {
    __shared__ double red[256];
    const Item it = res_item(groups, nblocks);
    const int sub = threadIdx.x >> 6;
    double acc2 = 0.0;
    const BlockDev& B = blocks[it.live ? it.blk : 0];
    const LaneDev& Ln = lanes[(int64_t)(it.live ? it.blk : 0) * lpb + (it.live ? it.lane : 0)];
    const int t0 = B.tb + it.chunk * RES_T;
    if (it.live && t0 <= B.te) {
        const int n = tets[B.tet].n, v = Ln.v, w = Ln.w;
        const bool valid = v != 0;
        const int64_t rs = Ln.rp[R_SELF];
        int64_t rpl[NLOW], rpu[NLOW];
#pragma unroll
        for (int s = 0; s < NLOW; ++s) {
            rpl[s] = Ln.rp[low_row(s)] + (int64_t)lpb * low_dt(s);
            rpu[s] = Ln.rp[up_row(s)] + (int64_t)lpb * up_dt(s);
        }
        // the chunk, clipped to the hyperplanes where this 64-lane group has an active point
        const int t1 = min(min(B.te, t0 + RES_T - 1), Ln.gt[1]);
        for (int t = max(t0, Ln.gt[0]) + sub; t <= t1; t += 8) {
            const int tp[2] = {t, min(t + 4, B.te + 1)};
            bool act[2];
            double a[2][15], xv[2][15], bv[2];
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const int xx = tp[p] - 2 * v - w;
                act[p] = valid && xx >= 1 && xx <= n - 1 - v && (p == 0 || t + 4 <= t1);
                // inactive points read the zero region (cache resident) instead of
                // padding slots, so padding costs no memory traffic
                const int64_t off = act[p] ? (int64_t)lpb * tp[p] : 0;
                const int64_t idx = act[p] ? rs + off : 0;
                // the centre weight and b are read once per launch: streaming
                // loads, so they do not take L2 space from x and the lower
                // weights, which the neighbours read again
                a[p][0] = __builtin_nontemporal_load(A8 + idx);
                xv[p][0] = x[idx];
                bv[p] = SUB ? __builtin_nontemporal_load(b + idx) : 0.0;
#pragma unroll
                for (int s = 0; s < NLOW; ++s) {
                    const int64_t ql = act[p] ? rpl[s] + off : 0, qu = act[p] ? rpu[s] + off : 0;
                    a[p][1 + 2 * s] = A8[(int64_t)(1 + s) * S + idx];
                    xv[p][1 + 2 * s] = x[ql];
                    a[p][2 + 2 * s] = A8[(int64_t)(1 + s) * S + qu];
                    xv[p][2 + 2 * s] = x[qu];
                }
            }
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                // the order and the fused multiply-adds of residual_point
                double acc = a[p][0] * xv[p][0];
#pragma unroll
                for (int k = 1; k < 15; ++k) acc = fma(a[p][k], xv[p][k], acc);
                const double rv = act[p] ? (SUB ? bv[p] - acc : acc) : 0.0;
                // only active points: the second point of a pair may lie in the next
                // chunk (the clipped range need not be a multiple of 8 long), whose
                // item writes it; inactive slots stay 0 from the allocation.  A
                // streaming store: r is read back only by the next kernel.
                if (act[p]) __builtin_nontemporal_store((RT)rv, r + rs + (int64_t)lpb * tp[p]);
                acc2 += rv * rv;
            }
        }
    }
    red[threadIdx.x] = acc2;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && partial) partial[it.id] = red[0];
}

// ------------------------------------------------------ LDS-staged residual

// Raw buffer stores (gfx9 buffer resource: no swizzle, byte range rbytes): a
// lane whose offset is RL_DROP, beyond every range, writes nothing.
constexpr uint32_t RL_DROP = 0xFFFFFFF0u;
constexpr int RL_RSRC_WORD3 = 0x00020000;
typedef unsigned int rl_u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void store_dropped(float v, __amdgpu_buffer_rsrc_t rs, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), rs, (int)off, 0, 2);  // aux 2: nontemporal
}
__device__ __forceinline__ void store_dropped(double v, __amdgpu_buffer_rsrc_t rs, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(rl_u32x2, v), rs, (int)off, 0, 2);
}

//
// The same r = b - A x as k_residual (the values and the order of the
// products of residual_point), reading every value from memory once: the
// workgroup owns one block of BV x BW rows (one thread per row) and walks
// tlen of its hyperplanes (RES_T or 2 RES_T, the handle's choice).  A point at t reads x at t - 3 .. t + 3 (LDS ring
// of hyperplane slices: the block's rows and the one-row halo on all four
// sides) and arrays 2..7 of the stencil at t .. t + 3 (LDS ring: the block's
// rows and, at the upper halo rows, the upper weights the block's edge rows
// read there); arrays 0 and 1, which only the own row reads, and b come from
// registers, loaded for the step itself.  Step t stages the slices of t + 3,
// loaded during step t - RL_P, so RL_P slice loads are in flight while the
// workgroup computes.  A second barrier after the arithmetic lets the rings
// hold exactly the slices in use (7 of x, 4 of the stencil), so that two
// 256-row workgroups fit in the LDS of a CU.  Halo rows are reached through
// the row pointers of the block's edge lanes.  Every value a point uses comes
// from the address k_residual forms for it, or from the zero slot at 0 where
// that address holds a point outside the lattice (the host layout check
// replays these indices).
//
// TAG: the residual for a forward sweep running at the same time (as
// k_residual_tag): workgroup (blk, y) covers the absolute hyperplanes
// [y RES_T, (y+1) RES_T) of its block, so the grid runs band by band in the
// order the sweep consumes; r goes out as tagged entries (tag *tagp) and each
// of the block's lane groups gets its band mark once the workgroup is done.
template <typename RT, bool SUB, int BV, int BW, bool TAG>
__global__ void __launch_bounds__(BV* BW, 2) k_residual_lds(const TetDev* __restrict__ tets,
                                                         const BlockDev* __restrict__ blocks,
                                                         const LaneDev* __restrict__ lanes, int nblocks, int groups,
                                                         int64_t S, const double* __restrict__ A8,
                                                         const double* __restrict__ x, const double* __restrict__ b,
                                                         RT* __restrict__ r, uint32_t rbytes,
                                                         uint64_t* __restrict__ rt, const int32_t* __restrict__ tagp,
                                                         uint64_t* __restrict__ rflag, double* __restrict__ partial,
                                                         int tlen, int pchunks) {
    using G = RlGeo<BV, BW>;
    constexpr int NT = G::NT, XC = G::XC, AC = G::AC, RX = G::RX, RA = G::RA, HJ = G::HJ;
    static_assert(RL_P == 4, "four register slice groups");
    // r through a buffer resource of rbytes bytes: stores at RL_DROP are dropped
    const __amdgpu_buffer_rsrc_t rbuf = __builtin_amdgcn_make_buffer_rsrc(r, 0, (int)rbytes, RL_RSRC_WORD3);
    __shared__ double lds[G::LDS];
    double* const LX = lds;
    double* const LA = lds + RX * XC;
    const int blk = (int)blockIdx.x, chunk = (int)blockIdx.y, l = (int)threadIdx.x;
    double acc2 = 0.0;
    const BlockDev& B = blocks[blk];
    const uint32_t tag = TAG ? (uint32_t)tagp[0] : 0u;
    const int t0 = TAG ? max(B.tb, chunk * RES_T) : B.tb + chunk * tlen;
    const int t1 = min(B.te + 1, TAG ? (chunk + 1) * RES_T : t0 + tlen);
    if (t0 < t1) {
        const int64_t lpb = NT;
        const LaneDev& Ln = lanes[(int64_t)blk * NT + l];
        const int n = tets[B.tet].n;
        int vl = 0, wl = 0;
        lane_rc(l, BV, &vl, &wl);
        const int64_t rs = Ln.rp[R_SELF];
        const RlRow own = rl_row(n, Ln.v, Ln.w);  // v = 0 (no row) is outside the lattice
        // this thread's halo loads of a slice: job j = l + k NT.  Branch-free,
        // so that the compiler's wait counts stay exact: a job without a cell
        // loads the zero slot at 0 and writes it to this thread's own x cell,
        // which the thread writes again right after.
        const double* hsrc[HJ];  // x or the halo row's stencil array
        int64_t hp[HJ];          // row pointer of the halo row
        RlRow hrow[HJ];          // activity of the halo row
        int hcell[HJ];           // LDS cell inside the slice
        int hkind[HJ];           // 0: x, 1: stencil, 2: none
#pragma unroll
        for (int k = 0; k < HJ; ++k) {
            const RlHalo o = rl_halo<BV, BW>(l + k * NT);
            hsrc[k] = o.arr < 0 ? x : A8 + (int64_t)o.arr * S;
            hcell[k] = o.dst < 0 ? l : o.dst;
            hkind[k] = o.dst < 0 ? 2 : o.arr < 0 ? 0 : 1;
            hp[k] = 0;
            hrow[k] = RlRow{0, 0};
            if (o.dst >= 0) {
                int sv = 0, sw = 0;
                lane_rc(o.src, BV, &sv, &sw);
                hp[k] = lanes[(int64_t)blk * NT + o.src].rp[o.slot];
                hrow[k] = rl_row(n, B.V0 + sv + rl_slot_dv(o.slot), B.W0 + sw + rl_slot_dw(o.slot));
            }
        }
        // LDS cells of the point's neighbours
        int xl[NLOW], xu[NLOW], au[NLOW];
#pragma unroll
        for (int s = 0; s < NLOW; ++s) rl_cells<BV, BW>(vl, wl, s, &xl[s], &xu[s], &au[s]);
        // the loads of step u: x and arrays 2..7 of slice u + 3 (staged in LDS),
        // arrays 0, 1 and b of slice u (used by step u itself), the halo of u + 3
        struct Regs {
            double xo, an[6], a01[2], bo, h[HJ];
        };
        const int ucap = t1 + 2;  // the last slice the chunk reads
        // A slot of a point outside the lattice holds zero: its load reads the
        // zero region at 0 instead (cache resident), so only interior points
        // cost memory traffic.
        auto load = [&](int u, Regs& R) {
            const int ux = min(u + 3, ucap), uo = min(u, ucap);
            const int64_t ix = rl_active(own, ux) ? rs + lpb * ux : 0;
            const int64_t io = rl_active(own, uo) ? rs + lpb * uo : 0;
            R.xo = x[ix];
#pragma unroll
            for (int a = 0; a < 6; ++a) R.an[a] = A8[(int64_t)(2 + a) * S + ix];
            R.a01[0] = A8[io];
            R.a01[1] = A8[S + io];
            R.bo = SUB ? b[io] : 0.0;
#pragma unroll
            for (int k = 0; k < HJ; ++k) R.h[k] = hsrc[k][rl_active(hrow[k], ux) ? hp[k] + lpb * ux : 0];
        };
        // stage slice u + 3: the halo first, so that a job without a cell is
        // overwritten by the thread's own x
        auto put = [&](int u, const Regs& R) {
            double* lx = LX + ((u + 3) % RX) * XC;
            double* la = LA + ((u + 3) % RA) * AC;
#pragma unroll
            for (int k = 0; k < HJ; ++k) (hkind[k] == 1 ? la : lx)[hcell[k]] = R.h[k];
            lx[l] = R.xo;
#pragma unroll
            for (int a = 0; a < 6; ++a) la[a * NT + l] = R.an[a];
        };
        // x of t0-3 .. t0+2 and arrays 2..7 of t0 .. t0+2.  Only what the
        // first steps read is loaded: x alone for the three earlier slices (the
        // stencil cells of those slots are written but overwritten before they
        // are read), no weights of arrays 0 and 1 and no b (steps load their own).
        for (int u = t0 - 6; u < t0; ++u) {
            Regs R;
            const int ux = u + 3;
            const bool stencil = ux >= t0;
            const int64_t ix = rl_active(own, ux) ? rs + lpb * ux : 0;
            R.xo = x[ix];
#pragma unroll
            for (int a = 0; a < 6; ++a) R.an[a] = stencil ? A8[(int64_t)(2 + a) * S + ix] : 0.0;
#pragma unroll
            for (int k = 0; k < HJ; ++k)
                R.h[k] = (stencil || hkind[k] != 1) ? hsrc[k][rl_active(hrow[k], ux) ? hp[k] + lpb * ux : 0] : 0.0;
            put(u, R);
        }
        Regs R[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) load(t0 + k, R[k]);
        // every step runs (loads, stores to LDS and the barrier), points beyond
        // the chunk are not computed: a loop without conditional steps keeps
        // RL_P slice loads in flight across its back edge
        auto step = [&](int t, int k) {
            Regs& Rk = R[k];
            put(t, Rk);
            const double a0 = Rk.a01[0], a1 = Rk.a01[1], a1u = R[(k + 1) & 3].a01[1], bt = Rk.bo;
            lds_barrier();
            // branch-free (a point outside the chunk or the lattice computes on
            // defined LDS values and its store is dropped as out of range), so
            // that the wait counts do not depend on the path
            {
                const bool act = t < t1 && rl_active(own, t);
                double a[15], xv[15];
                a[0] = a0;
                const double* at = LA + (t % RA) * AC;
                xv[0] = LX[(t % RX) * XC + l];
                a[1] = a1;
                a[2] = a1u;
                xv[1] = LX[((t + low_dt(0)) % RX) * XC + xl[0]];
                xv[2] = LX[((t + up_dt(0)) % RX) * XC + xu[0]];
#pragma unroll
                for (int s = 1; s < NLOW; ++s) {
                    a[1 + 2 * s] = at[(s - 1) * NT + l];
                    xv[1 + 2 * s] = LX[((t + low_dt(s)) % RX) * XC + xl[s]];
                    a[2 + 2 * s] = LA[((t + up_dt(s)) % RA) * AC + au[s]];
                    xv[2 + 2 * s] = LX[((t + up_dt(s)) % RX) * XC + xu[s]];
                }
                // the order and the fused multiply-adds of residual_point
                double acc = a[0] * xv[0];
#pragma unroll
                for (int q = 1; q < 15; ++q) acc = fma(a[q], xv[q], acc);
                const double rv = SUB ? bt - acc : acc;
                if (TAG) {
                    if (act) x_put(rt + (rs + lpb * t) * XEnt<RT>::W, (RT)rv, tag);
                } else {
                    store_dropped((RT)rv, rbuf, act ? (uint32_t)((rs + lpb * t) * (int64_t)sizeof(RT)) : RL_DROP);
                }
                acc2 += act ? rv * rv : 0.0;
            }
            // the next step overwrites the slices of t - 3 (x) and t (stencil)
            lds_barrier();
            // the loads of step t + RL_P, issued once this step's own registers
            // are consumed (so that no loaded register is copied)
            load(t + RL_P, Rk);
        };
        for (int t = t0; t < t1; t += RL_P) {
            step(t, 0);
            step(t + 1, 1);
            step(t + 2, 2);
            step(t + 3, 3);
        }
    }
    // the partial sums (the LDS rings are free once every wave is here)
    double* const red = lds;
    __syncthreads();
    // the band marks: a pacing hint for the sweep, which relies on the
    // entries' own tags; no fence (an agent-scope release writes back the L2)
    if (TAG && l < groups) st_dev(rflag + ((int64_t)blk * groups + l) * gridDim.y + chunk, (uint64_t)tag);
    red[l] = acc2;
    __syncthreads();
    for (int o = NT / 2; o > 0; o >>= 1) {
        if (l < o) red[l] += red[l + o];
        __syncthreads();
    }
    // the partial-sum layout of k_residual (pchunks chunks of RES_T
    // hyperplanes): the block's first lane group holds the sum, its other
    // groups 0; a chunk of tlen = k RES_T hyperplanes fills the slots of the k
    // chunks it covers, its sum in the first
    if (partial && l < groups) {
        const int k = TAG ? 1 : tlen / RES_T, pc = chunk * k;
        for (int j = 0; j < k; ++j)
            if (TAG || pc + j < pchunks)
                partial[((int64_t)(pc + j) * nblocks + blk) * groups + l] = l == 0 && j == 0 ? red[0] : 0.0;
    }
}

// Residual for a forward sweep running at the same time: tagged entries
// (XEnt<RT> words, tag *tagp) instead of plain values, produced in the order
// the sweep consumes them -- workgroup (x, y) takes the lanes of its block
// over the absolute hyperplanes [y RES_T, (y+1) RES_T), so the grid sweeps the
// whole batch band by band in hyperplane order.  The per-thread work is that
// of k_residual (two points per iteration, every load of both issued before
// the arithmetic); values and the order of the products are those of
// residual_point.
template <typename RT>
__global__ void __launch_bounds__(256)
    k_residual_tag(const TetDev* __restrict__ tets, const BlockDev* __restrict__ blocks,
                   const LaneDev* __restrict__ lanes, int lpb, int groups, int nblocks, int64_t S,
                   const double* __restrict__ A8, const double* __restrict__ x, const double* __restrict__ b,
                   uint64_t* __restrict__ rt, const int32_t* __restrict__ tagp, uint64_t* __restrict__ rflag,
                   double* __restrict__ partial) {
    __shared__ double red[256];
    const Item it = res_item(groups, nblocks);
    const uint32_t tag = (uint32_t)tagp[0];
    const int sub = threadIdx.x >> 6;
    double acc2 = 0.0;
    const BlockDev& B = blocks[it.live ? it.blk : 0];
    const LaneDev& Ln = lanes[(int64_t)(it.live ? it.blk : 0) * lpb + (it.live ? it.lane : 0)];
    const int t0 = max(max(B.tb, it.chunk * RES_T), Ln.gt[0]);
    const int t1 = min(min(B.te, it.chunk * RES_T + RES_T - 1), Ln.gt[1]);
    if (it.live && t0 <= t1) {
        const int n = tets[B.tet].n, v = Ln.v, w = Ln.w;
        const bool valid = v != 0;
        const int64_t rs = Ln.rp[R_SELF];
        int64_t rpl[NLOW], rpu[NLOW];
#pragma unroll
        for (int s = 0; s < NLOW; ++s) {
            rpl[s] = Ln.rp[low_row(s)] + (int64_t)lpb * low_dt(s);
            rpu[s] = Ln.rp[up_row(s)] + (int64_t)lpb * up_dt(s);
        }
        for (int t = t0 + sub; t <= t1; t += 8) {
            const int tp[2] = {t, t + 4};
            bool act[2];
            double a[2][15], xv[2][15], bv[2];
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                const int xx = tp[p] - 2 * v - w;
                act[p] = valid && xx >= 1 && xx <= n - 1 - v && tp[p] <= t1;
                const int64_t off = act[p] ? (int64_t)lpb * tp[p] : 0;
                const int64_t idx = act[p] ? rs + off : 0;
                a[p][0] = __builtin_nontemporal_load(A8 + idx);
                xv[p][0] = x[idx];
                bv[p] = __builtin_nontemporal_load(b + idx);
#pragma unroll
                for (int s = 0; s < NLOW; ++s) {
                    const int64_t ql = act[p] ? rpl[s] + off : 0, qu = act[p] ? rpu[s] + off : 0;
                    a[p][1 + 2 * s] = A8[(int64_t)(1 + s) * S + idx];
                    xv[p][1 + 2 * s] = x[ql];
                    a[p][2 + 2 * s] = A8[(int64_t)(1 + s) * S + qu];
                    xv[p][2 + 2 * s] = x[qu];
                }
            }
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                double acc = a[p][0] * xv[p][0];
#pragma unroll
                for (int k = 1; k < 15; ++k) acc = fma(a[p][k], xv[p][k], acc);
                const double rv = act[p] ? bv[p] - acc : 0.0;
                if (act[p]) x_put(rt + (rs + (int64_t)lpb * tp[p]) * XEnt<RT>::W, (RT)rv, tag);
                acc2 += rv * rv;
            }
        }
    }
    red[threadIdx.x] = acc2;
    // the band mark is a pacing hint for the sweep, which relies on the
    // entries' own tags; no fence (an agent-scope release writes back the L2)
    __syncthreads();
    if (threadIdx.x == 0 && it.live) st_dev(rflag + (int64_t)blockIdx.x * gridDim.y + blockIdx.y, (uint64_t)tag);
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && partial) partial[it.id] = red[0];
}

// Residual with the surrogate operator (Sec. 4.2 approximates A by surrogate
// polynomials too): the neighbour weights come from the row's table -- the
// seven lower weights at p, the seven upper weights as the lower polynomials
// at p - d -- evaluated by Horner in the table's precision TT, and the centre
// is minus their sum (the full rows of A sum to zero, a(phi_p, 1) = 0), so
//     r = b - sum_{d != c} A~_d (x_{p+d} - x_p)
// in FP64.  A fitted centre would break the row sums by the fit error, which
// exceeds the O(h^3) smallest eigenvalues of A at fine levels.  Per point it
// loads x at p and its 14 neighbours and b, and no stencil weights.  One
// point per thread and iteration.
template <int NC, typename TT>
__device__ __forceinline__ TT horner_c(const TT* c, TT eta) {
    TT acc = c[NC - 1];
#pragma unroll
    for (int i = NC - 2; i >= 0; --i) acc = acc * eta + c[i];
    return acc;
}

template <typename RT, typename TT, int NC, bool SUB>
__global__ void __launch_bounds__(256) k_residual_sa(const TetDev* __restrict__ tets, const BlockDev* __restrict__ blocks,
                                                     const LaneDev* __restrict__ lanes, int lpb, int groups,
                                                     int nblocks, const TT* __restrict__ tab,
                                                     const double* __restrict__ x, const double* __restrict__ b,
                                                     RT* __restrict__ r, double* __restrict__ partial) {
    __shared__ double red[256];
    const Item it = res_item(groups, nblocks);
    const int sub = threadIdx.x >> 6;
    double acc2 = 0.0;
    const int64_t slot = (int64_t)(it.live ? it.blk : 0) * lpb + (it.live ? it.lane : 0);
    const BlockDev& B = blocks[it.live ? it.blk : 0];
    const LaneDev& Ln = lanes[slot];
    const int t0 = B.tb + it.chunk * RES_T;
    if (it.live && t0 <= B.te) {
        const int n = tets[B.tet].n, v = Ln.v, w = Ln.w;
        const bool valid = v != 0;
        const int64_t rs = Ln.rp[R_SELF];
        int64_t rpl[NLOW], rpu[NLOW];
#pragma unroll
        for (int s = 0; s < NLOW; ++s) {
            rpl[s] = Ln.rp[low_row(s)] + (int64_t)lpb * low_dt(s);
            rpu[s] = Ln.rp[up_row(s)] + (int64_t)lpb * up_dt(s);
        }
        // row record [xm, 1/hw, lower 7*NC, centre NC (unused), upper 7*NC] (zeros for unused lanes)
        const TT* tr = tab + slot * (2 + 15 * NC);
        const TT xm = tr[0], ihw = tr[1];
        TT c[15 * NC];
#pragma unroll
        for (int i = 0; i < 15 * NC; ++i) c[i] = tr[2 + i];
        const int t1 = min(min(B.te, t0 + RES_T - 1), Ln.gt[1]);  // clipped as in k_residual
        for (int t = max(t0, Ln.gt[0]) + sub; t <= t1; t += 4) {
            const int xx = t - 2 * v - w;
            const bool act = valid && xx >= 1 && xx <= n - 1 - v;
            // inactive points read the zero region, as in the assembled residual
            const int64_t off = act ? (int64_t)lpb * t : 0;
            const int64_t idx = act ? rs + off : 0;
            double xl[NLOW], xu[NLOW];
            const double xc = x[idx];
#pragma unroll
            for (int s = 0; s < NLOW; ++s) {
                xl[s] = x[act ? rpl[s] + off : 0];
                xu[s] = x[act ? rpu[s] + off : 0];
            }
            const double bv = SUB ? b[idx] : 0.0;
            const TT eta = ((TT)xx - xm) * ihw;
            double acc = 0.0;
#pragma unroll
            for (int s = 0; s < NLOW; ++s)
                acc += (double)horner_c<NC>(c + s * NC, eta) * (xl[s] - xc) +
                       (double)horner_c<NC>(c + (8 + s) * NC, eta) * (xu[s] - xc);
            const double rv = act ? (SUB ? bv - acc : acc) : 0.0;
            r[rs + (int64_t)lpb * t] = (RT)rv;
            acc2 += rv * rv;
        }
    }
    red[threadIdx.x] = acc2;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0 && partial) partial[it.id] = red[0];
}

// sum of squares of a stream vector restricted to active points (for ||b||)
__global__ void __launch_bounds__(256) k_sumsq(const TetDev* __restrict__ tets, const BlockDev* __restrict__ blocks,
                                               const LaneDev* __restrict__ lanes, int lpb, int groups, int nblocks,
                                               const double* __restrict__ v_s,
                                               double* __restrict__ partial) {
    __shared__ double red[256];
    const Item it = res_item(groups, nblocks);
    double acc2 = 0.0;
    const BlockDev& B = blocks[it.live ? it.blk : 0];
    const LaneDev& Ln = lanes[(int64_t)(it.live ? it.blk : 0) * lpb + (it.live ? it.lane : 0)];
    const int t0 = B.tb + it.chunk * RES_T;
    if (it.live && Ln.v != 0 && t0 <= B.te) {
        const int n = tets[B.tet].n;
        const int t1 = min(min(B.te, t0 + RES_T - 1), Ln.gt[1]);
        for (int t = max(t0, Ln.gt[0]) + (int)(threadIdx.x >> 6); t <= t1; t += 4) {
            const int xx = t - 2 * Ln.v - Ln.w;
            if (xx < 1 || xx > n - 1 - Ln.v) continue;
            const double a = v_s[Ln.rp[R_SELF] + (int64_t)lpb * t];
            acc2 += a * a;
        }
    }
    red[threadIdx.x] = acc2;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[it.id] = red[0];
}

// out[slot] = sum of partial[0..count) (single workgroup, fixed order)
__global__ void __launch_bounds__(256) k_reduce(const double* __restrict__ partial, int64_t count,
                                                double* __restrict__ out, int slot) {
    __shared__ double red[256];
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += 256) a += partial[i];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[slot] = red[0];
}

// ------------------------------------------------- hyperplane-schedule sweeps

// Surrogate weight of table entry e at eta (Horner; NC = dg_x + 1 coefficients).
template <typename T>
__device__ __forceinline__ T horner(const T* __restrict__ c, int NC, T eta) {
    T acc = c[NC - 1];
    for (int i = NC - 2; i >= 0; --i) acc = acc * eta + c[i];
    return acc;
}

// Forward substitution on hyperplane t (Alg. 2, first loop, after the
// residual):  w^p = r^p - sum_{d in D_l} L^p_d w^{p+d}.  The products are
// accumulated in the order s, bnw, bc, be, w, se, bn (neighbours on older
// hyperplanes first), the order the dataflow kernels use.
// Variant V1 (v1 != null): the exact factors of the points of set F.
template <typename T, bool STORED>
__global__ void __launch_bounds__(64) k_fwd_plane(const TetDev* __restrict__ tets, const BlockDev* __restrict__ blocks,
                                                  const LaneDev* __restrict__ lanes, int lpb, int groups, int t, int64_t S,
                                                  const double* __restrict__ Lf, const T* __restrict__ tab, int NC,
                                                  const T* __restrict__ v1, const T* __restrict__ r,
                                                  T* __restrict__ w) {
    int b, lane;
    decode_group(groups, b, lane);
    const BlockDev& B = blocks[b];
    if (t < B.tb || t > B.te) return;
    const LaneDev& Ln = lanes[(int64_t)b * lpb + lane];
    if (Ln.v == 0) return;
    const int n = tets[B.tet].n, v = Ln.v;
    const int x = t - 2 * v - Ln.w;
    if (x < 1 || x > n - 1 - v) return;
    const int64_t off = (int64_t)lpb * t;
    const int64_t idx = Ln.rp[R_SELF] + off;
    T acc = r[idx];
    constexpr int ord[7] = {1, 3, 5, 6, 0, 2, 4};
    if (STORED) {
#pragma unroll
        for (int j = 0; j < NLOW; ++j) {
            const int s = ord[j];
            acc -= (T)Lf[(int64_t)s * S + idx] * w[Ln.rp[low_row(s)] + off + lpb * low_dt(s)];
        }
    } else {
        const T* c = tab + ((int64_t)b * lpb + lane) * (2 + 15 * NC);
        const T eta = ((T)x - c[0]) * c[1];
        const int pos = v1 ? v1f_pos(x, n - 1 - v, v - Ln.w, Ln.w) : -1;
#pragma unroll
        for (int j = 0; j < NLOW; ++j) {
            const int s = ord[j];
            const T Ls = pos >= 0 ? v1[((int64_t)Ln.v1f[0] + pos) * 8 + s] : horner(c + 2 + s * NC, NC, eta);
            acc -= Ls * w[Ln.rp[low_row(s)] + off + lpb * low_dt(s)];
        }
    }
    w[idx] = acc;
}

// Backward substitution with the diagonal scaling and the update on
// hyperplane t (Alg. 2, second loop):
//   w^p = (D^p)^{-1} w^p - sum_{d in D_l} L^{p-d}_d w^{p-d};  x^p += w^p.
// Variant V1 (v1 != null): the weights of set B.
template <typename T, bool STORED>
__global__ void __launch_bounds__(64) k_bwd_plane(const TetDev* __restrict__ tets, const BlockDev* __restrict__ blocks,
                                                  const LaneDev* __restrict__ lanes, int lpb, int groups, int t, int64_t S,
                                                  const double* __restrict__ Lb, const T* __restrict__ tab, int NC,
                                                  const T* __restrict__ v1, T* __restrict__ w,
                                                  double* __restrict__ x) {
    int b, lane;
    decode_group(groups, b, lane);
    const BlockDev& B = blocks[b];
    if (t < B.tb || t > B.te) return;
    const LaneDev& Ln = lanes[(int64_t)b * lpb + lane];
    if (Ln.v == 0) return;
    const int n = tets[B.tet].n, v = Ln.v;
    const int xx = t - 2 * v - Ln.w;
    if (xx < 1 || xx > n - 1 - v) return;
    const int64_t off = (int64_t)lpb * t;
    const int64_t idx = Ln.rp[R_SELF] + off;
    T acc;
    constexpr int ord[7] = {1, 3, 5, 6, 0, 2, 4};
    if (STORED) {
        acc = w[idx] * (T)Lb[idx];
#pragma unroll
        for (int j = 0; j < NLOW; ++j) {
            const int s = ord[j];
            acc -= (T)Lb[(int64_t)(1 + s) * S + idx] * w[Ln.rp[up_row(s)] + off + lpb * up_dt(s)];
        }
    } else {
        const T* c = tab + ((int64_t)b * lpb + lane) * (2 + 15 * NC);
        const T eta = ((T)xx - c[0]) * c[1];
        const int pos = v1 ? v1b_pos(xx, n - 1 - v, v - Ln.w, Ln.w) : -1;
        const int64_t j1 = (int64_t)Ln.v1b + pos;
        acc = w[idx] * (pos >= 0 ? v1[j1 * 8] : horner(c + 2 + 7 * NC, NC, eta));
#pragma unroll
        for (int j = 0; j < NLOW; ++j) {
            const int s = ord[j];
            const T Us = pos >= 0 ? v1[j1 * 8 + 1 + s] : horner(c + 2 + (8 + s) * NC, NC, eta);
            acc -= Us * w[Ln.rp[up_row(s)] + off + lpb * up_dt(s)];
        }
    }
    w[idx] = acc;
    x[idx] += (double)acc;
}

// Surrogate weights exactly as the sweeps evaluate them, exported in
// lexicographic order (inspection only).
// Variant V1 (F != null): the exact factors at the points of set F.
template <typename T>
__global__ void k_export_surrogate(const TetDev* __restrict__ tets, const BlockDev* __restrict__ blocks,
                                   const LaneDev* __restrict__ lanes, int lpb, int groups, const T* __restrict__ tab, int NC, int only_tet,
                                   const T* __restrict__ F, double* __restrict__ L_out,
                                   double* __restrict__ Dinv_out) {
    int b, lane;
    decode_group(groups, b, lane);
    const BlockDev B = blocks[b];
    if (B.tet != only_tet) return;
    const LaneDev& Ln = lanes[(int64_t)b * lpb + lane];
    if (Ln.v == 0) return;
    const int n = tets[B.tet].n, v = Ln.v, w = Ln.w, y = v - w, z = w;
    const T* c = tab + ((int64_t)b * lpb + lane) * (2 + 15 * NC);
    for (int t = B.tb + (int)(threadIdx.x >> 6); t <= B.te; t += (int)(blockDim.x >> 6)) {
        const int x = t - 2 * v - w;
        if (x < 1 || x > n - 1 - v) continue;
        const int64_t li = lex_index(n, x, y, z);
        const T eta = ((T)x - c[0]) * c[1];
        const int pos = F ? v1f_pos(x, n - 1 - v, y, z) : -1;
        const int64_t j = (int64_t)Ln.v1f[0] + pos;
        if (L_out)
            for (int s = 0; s < NLOW; ++s)
                L_out[li * NLOW + s] = (double)(pos >= 0 ? F[j * 8 + s] : horner(c + 2 + s * NC, NC, eta));
        if (Dinv_out) Dinv_out[li] = (double)(pos >= 0 ? F[j * 8 + NLOW] : horner(c + 2 + 7 * NC, NC, eta));
    }
}

// ------------------------------------------------------------- host launchers

void launch_export_surrogate(const Ctx& c, bool f32, int tet, double* L_out, double* Dinv_out, hipStream_t st) {
    if (f32)
        k_export_surrogate<float><<<c.nblocks * c.groups, 256, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups,
                                                                        c.tab32, c.NC, tet, (const float*)c.v1f,
                                                                        L_out, Dinv_out);
    else
        k_export_surrogate<double><<<c.nblocks * c.groups, 256, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups,
                                                                         c.tab64, c.NC, tet, (const double*)c.v1f,
                                                                         L_out, Dinv_out);
}

int64_t res_partials(const Ctx& c) { return (int64_t)c.nblocks * c.groups * c.res_chunks; }

namespace {
template <typename TT, int NC>
void launch_residual_sa(const Ctx& c, const TT* tab, const double* x, const double* b, void* r, bool f32, int subtract,
                        double* partial, hipStream_t st) {
    const dim3 grid((unsigned)(c.nblocks * c.groups), (unsigned)c.res_chunks);
#define ILU_RSA_ARGS c.tets, c.blocks, c.lanes, c.lpb, c.groups, c.nblocks, tab, x, b
    if (f32 && subtract) k_residual_sa<float, TT, NC, true><<<grid, 256, 0, st>>>(ILU_RSA_ARGS, (float*)r, partial);
    else if (f32) k_residual_sa<float, TT, NC, false><<<grid, 256, 0, st>>>(ILU_RSA_ARGS, (float*)r, partial);
    else if (subtract) k_residual_sa<double, TT, NC, true><<<grid, 256, 0, st>>>(ILU_RSA_ARGS, (double*)r, partial);
    else k_residual_sa<double, TT, NC, false><<<grid, 256, 0, st>>>(ILU_RSA_ARGS, (double*)r, partial);
#undef ILU_RSA_ARGS
}

template <typename TT>
void launch_residual_sa_nc(const Ctx& c, const TT* tab, const double* x, const double* b, void* r, bool f32,
                           int subtract, double* partial, hipStream_t st) {
    switch (c.NC) {
    case 1: launch_residual_sa<TT, 1>(c, tab, x, b, r, f32, subtract, partial, st); break;
    case 2: launch_residual_sa<TT, 2>(c, tab, x, b, r, f32, subtract, partial, st); break;
    case 3: launch_residual_sa<TT, 3>(c, tab, x, b, r, f32, subtract, partial, st); break;
    case 4: launch_residual_sa<TT, 4>(c, tab, x, b, r, f32, subtract, partial, st); break;
    case 5: launch_residual_sa<TT, 5>(c, tab, x, b, r, f32, subtract, partial, st); break;
    case 6: launch_residual_sa<TT, 6>(c, tab, x, b, r, f32, subtract, partial, st); break;
    default: launch_residual_sa<TT, 7>(c, tab, x, b, r, f32, subtract, partial, st); break;
    }
}
}  // namespace

namespace {
template <int BV, int BW>
void launch_residual_lds(const Ctx& c, const double* x, const double* b, void* r, bool f32, int subtract,
                         double* partial, hipStream_t st) {
    // chunks of res_lds_t hyperplanes, k of the RES_T chunks of the partial sums
    const int k = c.res_lds_t / RES_T;
    const dim3 grid((unsigned)c.nblocks, (unsigned)((c.res_chunks + k - 1) / k));
    const uint32_t rb = (uint32_t)(c.S * (f32 ? 4 : 8));
#define ILU_RL_ARGS c.tets, c.blocks, c.lanes, c.nblocks, c.groups, c.S, c.A8, x, b
#define ILU_RL_NOTAG nullptr, nullptr, nullptr, partial, c.res_lds_t, c.res_chunks
    if (f32 && subtract)
        k_residual_lds<float, true, BV, BW, false><<<grid, BV * BW, 0, st>>>(ILU_RL_ARGS, (float*)r, rb, ILU_RL_NOTAG);
    else if (f32)
        k_residual_lds<float, false, BV, BW, false><<<grid, BV * BW, 0, st>>>(ILU_RL_ARGS, (float*)r, rb, ILU_RL_NOTAG);
    else if (subtract)
        k_residual_lds<double, true, BV, BW, false><<<grid, BV * BW, 0, st>>>(ILU_RL_ARGS, (double*)r, rb, ILU_RL_NOTAG);
    else
        k_residual_lds<double, false, BV, BW, false><<<grid, BV * BW, 0, st>>>(ILU_RL_ARGS, (double*)r, rb, ILU_RL_NOTAG);
#undef ILU_RL_NOTAG
}

template <int BV, int BW>
void launch_residual_lds_tagged(const Ctx& c, const double* x, const double* b, uint64_t* rt, bool f32,
                                const int32_t* tagp, uint64_t* rflag, double* partial, hipStream_t st) {
    const dim3 grid((unsigned)c.nblocks, (unsigned)c.res_bands);
    if (f32)
        k_residual_lds<float, true, BV, BW, true><<<grid, BV * BW, 0, st>>>(ILU_RL_ARGS, nullptr, 0, rt, tagp, rflag,
                                                                           partial, RES_T, c.res_bands);
    else
        k_residual_lds<double, true, BV, BW, true><<<grid, BV * BW, 0, st>>>(ILU_RL_ARGS, nullptr, 0, rt, tagp, rflag,
                                                                            partial, RES_T, c.res_bands);
#undef ILU_RL_ARGS
}
}  // namespace

void launch_residual(const Ctx& c, const double* x, const double* b, void* r, bool f32, int subtract, double* partial,
                     hipStream_t st) {
    if (c.tabA32) return launch_residual_sa_nc<float>(c, c.tabA32, x, b, r, f32, subtract, partial, st);
    if (c.tabA64) return launch_residual_sa_nc<double>(c, c.tabA64, x, b, r, f32, subtract, partial, st);
    // the LDS-staged kernel addresses r by 32-bit byte offsets below RL_DROP
    const bool lds_ok = c.res_lds && c.S * 8 < (int64_t)RL_DROP;
    if (lds_ok && c.bv == 8 && c.bw == 8) return launch_residual_lds<8, 8>(c, x, b, r, f32, subtract, partial, st);
    if (lds_ok && c.bv == 16 && c.bw == 16) return launch_residual_lds<16, 16>(c, x, b, r, f32, subtract, partial, st);
    const dim3 grid((unsigned)(c.nblocks * c.groups), (unsigned)c.res_chunks);
#define ILU_RES_ARGS c.tets, c.blocks, c.lanes, c.lpb, c.groups, c.nblocks, c.S, c.A8, x, b
    if (f32 && subtract) k_residual<float, true><<<grid, 256, 0, st>>>(ILU_RES_ARGS, (float*)r, partial);
    else if (f32) k_residual<float, false><<<grid, 256, 0, st>>>(ILU_RES_ARGS, (float*)r, partial);
    else if (subtract) k_residual<double, true><<<grid, 256, 0, st>>>(ILU_RES_ARGS, (double*)r, partial);
    else k_residual<double, false><<<grid, 256, 0, st>>>(ILU_RES_ARGS, (double*)r, partial);
}

int64_t res_tag_partials(const Ctx& c) { return (int64_t)c.nblocks * c.groups * c.res_bands; }

void launch_residual_tagged(const Ctx& c, const double* x, const double* b, uint64_t* rt, bool f32,
                            const int32_t* tagp, uint64_t* rflag, double* partial, hipStream_t st) {
    if (c.res_lds && c.bv == 8 && c.bw == 8)
        return launch_residual_lds_tagged<8, 8>(c, x, b, rt, f32, tagp, rflag, partial, st);
    if (c.res_lds && c.bv == 16 && c.bw == 16)
        return launch_residual_lds_tagged<16, 16>(c, x, b, rt, f32, tagp, rflag, partial, st);
    const dim3 grid((unsigned)(c.nblocks * c.groups), (unsigned)c.res_bands);
    if (f32) k_residual_tag<float><<<grid, 256, 0, st>>>(ILU_RES_ARGS, rt, tagp, rflag, partial);
    else k_residual_tag<double><<<grid, 256, 0, st>>>(ILU_RES_ARGS, rt, tagp, rflag, partial);
#undef ILU_RES_ARGS
}

void launch_sumsq(const Ctx& c, const double* v, double* partial, hipStream_t st) {
    const dim3 grid((unsigned)(c.nblocks * c.groups), (unsigned)c.res_chunks);
    k_sumsq<<<grid, 256, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, c.nblocks, v, partial);
}

void launch_reduce(const double* partial, int64_t count, double* out, int slot, hipStream_t st) {
    k_reduce<<<1, 256, 0, st>>>(partial, count, out, slot);
}

void launch_fwd_plane(const Ctx& c, int variant, int t, hipStream_t st) {
    if (variant == 0)
        k_fwd_plane<double, true><<<c.nblocks * c.groups, 64, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, t, c.S, c.Lf, nullptr, 0,
                                                            nullptr, (const double*)c.r, (double*)c.w);
    else if (variant == 1)
        k_fwd_plane<double, false><<<c.nblocks * c.groups, 64, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, t, c.S, nullptr, c.tab64, c.NC,
                                                             (const double*)c.v1f, (const double*)c.r, (double*)c.w);
    else
        k_fwd_plane<float, false><<<c.nblocks * c.groups, 64, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, t, c.S, nullptr, c.tab32, c.NC,
                                                            (const float*)c.v1f, (const float*)c.r, (float*)c.w);
}

void launch_bwd_plane(const Ctx& c, int variant, int t, double* x, hipStream_t st) {
    if (variant == 0)
        k_bwd_plane<double, true><<<c.nblocks * c.groups, 64, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, t, c.S, c.Lb, nullptr, 0,
                                                            nullptr, (double*)c.w, x);
    else if (variant == 1)
        k_bwd_plane<double, false><<<c.nblocks * c.groups, 64, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, t, c.S, nullptr, c.tab64, c.NC,
                                                             (const double*)c.v1b, (double*)c.w, x);
    else
        k_bwd_plane<float, false><<<c.nblocks * c.groups, 64, 0, st>>>(c.tets, c.blocks, c.lanes, c.lpb, c.groups, t, c.S, nullptr, c.tab32, c.NC,
                                                            (const float*)c.v1b, (float*)c.w, x);
}

}  // namespace ilu
