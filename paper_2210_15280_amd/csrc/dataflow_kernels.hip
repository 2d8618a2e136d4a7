// Persistent dataflow sweeps (Alg. 2 on the hyperplane schedule without a
// global barrier per hyperplane).
//
// One workgroup of BV*BW threads owns one BV x BW block of rows at a time.  A
// workgroup takes blocks from a ticket counter in a topological order of the
// block dependency graph, so every block it waits for is owned by a resident
// workgroup that took its ticket earlier: the wait chain always ends.
//
// Inside a block all lanes advance hyperplane by hyperplane in lock step (one
// LDS-only workgroup barrier per hyperplane).  The values of the last three
// hyperplanes live in a 4-slot LDS grid of (BV+1) x (BW+1) cells: the block's
// own rows plus one halo column and one halo row holding rows of the
// neighbouring blocks.
//
// Blocks hand boundary values to each other through an exchange buffer.
// Extra waves in every workgroup do all of this traffic, so the compute waves
// never wait on another block's memory.  After every hyperplane the outgoing
// wave copies the block's edge values (last column and last row in sweep
// direction) from LDS to the buffer, each with a 32-bit launch tag in one
// 64-bit word (FP64 values: two words, one per half).  D incoming waves take
// turns by hyperplane: each loads the entries of its next hyperplane D ahead
// and checks the tag right before the value goes into the LDS grid; only a
// stale entry is polled again.  No block
// ever waits for its own stores, and no progress counter sits between
// producer and consumer.  The tag is a device counter that the reset kernel advances
// before every sweep, so graph replays never see entries of earlier sweeps
// (tags repeat after 2^32 sweeps).
//
// Per-lane operands (r, w, x, stored factors) stream through register rings
// loaded U hyperplanes ahead.  The seven products of a point are accumulated
// oldest hyperplane first (the t-2 / t-3 neighbours, then the three t-1
// neighbours), so only three fused multiply-adds sit on the
// hyperplane-to-hyperplane dependency chain.
//
// A poll that exceeds a fixed bound sets flags[2] and gives up, so a logic
// error can never hang the device.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels_common.h"
#include "sweep_kernels.h"
#include "tagged_device.h"

namespace ilu {

namespace {

constexpr long SPIN_LIMIT = 1L << 20;
// accumulation order over D_l: s, bnw, bc, be (older hyperplanes) then w, se, bn
constexpr int ORD[7] = {1, 3, 5, 6, 0, 2, 4};

template <int N>
struct IC {
    static constexpr int value = N;
};

template <bool C, typename A, typename B>
struct Pick {
    using type = B;
};
template <typename A, typename B>
struct Pick<true, A, B> {
    using type = A;
};

// Batch depth of the streamed path of variant V1 (blocks with a row y <= 2 or
// z = 1): seven or eight factors per hyperplane ride along with the operands.
template <typename T>
constexpr int V1_UE() {
    return sizeof(T) == 4 ? 4 : 2;
}

// One 8-value record of the V1 sets (32 B FP32, 64 B FP64) in 16-byte loads.
__device__ __forceinline__ void load8(const float* p, float (&o)[8]) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    const float4 b = *reinterpret_cast<const float4*>(p + 4);
    o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
    o[4] = b.x; o[5] = b.y; o[6] = b.z; o[7] = b.w;
}
__device__ __forceinline__ void load8(const double* p, double (&o)[8]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double2 a = *reinterpret_cast<const double2*>(p + 2 * k);
        o[2 * k] = a.x;
        o[2 * k + 1] = a.y;
    }
}

template <int NC, typename T>
__device__ __forceinline__ T horner(const T* c, T eta) {
    T acc = c[NC - 1];
#pragma unroll
    for (int i = NC - 2; i >= 0; --i) acc = acc * eta + c[i];
    return acc;
}

// A residual entry that did not carry this sweep's tag when the forward sweep
// reached it: poll it up to `spins` times, then compute the value here (and
// poll less from then on).  Kept out of line: it is the rare path, and inlined
// it would hold registers across the whole sweep loop.
template <typename T>
__device__ __noinline__ T late_residual(const uint64_t* e, uint32_t tag, int& spins, const LaneDev& Ln, int lpb,
                                         int64_t S, int t, const double* A8, const double* xo, const double* bo) {
    XEnt<T> re;
    for (int k = 0; k < spins; ++k) {
        __builtin_amdgcn_s_sleep(2);
        x_get(re, e);
        if (x_ok(re, tag)) return x_val(re);
    }
    spins = 2;
    return (T)residual_point(Ln, lpb, S, t, A8, xo, bo);
}

// Halo role of a thread: one incoming row (column halo, row halo or corner).
struct Halo {
    bool role = false;
    int cell = 0;          // grid cell the row's value goes to
    int ptb = 1, pte = 0;  // producer's hyperplane range (empty: no producer, value 0)
    int ptlo = 0, j = 0;   // producer's time origin and the entry of this row
    int64_t pxoff = 0;     // producer's exchange window
    __device__ bool has(int s) const { return s >= ptb && s <= pte; }
};

template <typename T>
__device__ __forceinline__ const uint64_t* halo_at(const Halo& h, const uint64_t* xch, int nx, int s) {
    return xch + xch_word(h.pxoff, h.ptlo, nx, XEnt<T>::W, s, h.j);
}

template <typename T>
__device__ __forceinline__ void halo_issue(const Halo& h, const uint64_t* xch, int nx, int s, XEnt<T>& e) {
    if (h.has(s)) x_get(e, halo_at<T>(h, xch, nx, s));
}

// Value of the halo row at hyperplane s from an entry loaded earlier; a stale
// entry is polled until the producer's store with this launch's tag arrives.
template <typename T>
__device__ __forceinline__ T halo_take(const Halo& h, const uint64_t* xch, int nx, int s, XEnt<T>& e, uint32_t tag,
                                       int32_t* flags) {
    if (!h.has(s)) return (T)0;
    if (!x_ok(e, tag)) {
        long spins = 0;
        for (;;) {
            __builtin_amdgcn_s_sleep(1);
            x_get(e, halo_at<T>(h, xch, nx, s));
            if (x_ok(e, tag)) break;
            ++spins;
            if ((spins & 255) == 0 && ld_dev(&flags[2])) break;
            if (spins > SPIN_LIMIT) {
                atomicOr(&flags[2], 1);
                break;
            }
        }
    }
    return x_val(e);
}

}  // namespace

// ------------------------------------------------------------------ forward
//
// Workgroup = BV*BW compute threads (one per row) + D incoming waves + an
// outgoing wave.  Incoming lane i < BW+BV+1 owns halo row i (column, row,
// corner); outgoing lane i < BW+BV owns exchange entry i, whose producer lane
// is the one xch_out_lane names.  Loads and stores live in different waves
// because one wave's memory counter completes in issue order: a wait for a
// halo load would otherwise also wait for the slow device-coherent stores
// issued before it.  All paths pass the same barriers.

//
// OVL: the residual comes from the tagged stream rt that the residual kernel
// fills while this kernel runs.  A point whose entry does not yet carry this
// sweep's tag is polled a bounded number of times and then computed here
// (residual_point, bitwise the residual kernel's value), so the sweep never
// depends on the residual kernel being scheduled alongside it.
template <typename T, bool STORED, bool V1, bool OVL, int U, int D, int NC, int BV, int BW>
__global__ void __launch_bounds__(BV* BW + (D + 1) * WAVE)
    k_fwd_flow(const TetDev* __restrict__ tets, const BlockDev* __restrict__ blocks, const LaneDev* __restrict__ lanes,
               int nblocks, int64_t S, const double* __restrict__ Lf, const T* __restrict__ tab,
               const T* __restrict__ v1, int64_t v1s, const T* __restrict__ r, const uint64_t* __restrict__ rt,
               const double* __restrict__ A8, const double* __restrict__ xo, const double* __restrict__ bo,
               int rspin0, const uint64_t* __restrict__ rflag, int nbands, T* __restrict__ w,
               const int32_t* __restrict__ order, uint64_t* __restrict__ xch, int32_t* __restrict__ ticket,
               int32_t* __restrict__ flags) {
    constexpr int NT = BV * BW;
    constexpr int GW = BV + 1;
    constexpr int GC = (BV + 1) * (BW + 1);
    constexpr int NX = BV + BW;
    constexpr int XW = XEnt<T>::W;
    static_assert(NT % WAVE == 0 && NX + 1 <= WAVE, "block shape");
    __shared__ T grid[4 * GC];
    __shared__ int s_ticket;
    const int l = threadIdx.x;
    const uint32_t tag = (uint32_t)ticket[2];
    for (;;) {
        if (l == 0) s_ticket = atomicAdd(&ticket[0], 1);
        __syncthreads();
        const int k = s_ticket;
        __syncthreads();
        if (k >= nblocks) return;
        const int b = order[k];
        const BlockDev B = blocks[b];
        const int tb = B.tb, te = B.te;
        for (int i = l; i < 4 * GC; i += NT + (D + 1) * WAVE) grid[i] = (T)0;
        if (l >= NT + D * WAVE) {
            // ---------------- outgoing wave: copies the block's edge values of
            // hyperplane t-1 (published by the last barrier) to the exchange
            // buffer.  It only stores, so it never waits on memory in the loop.
            const int hlane = l - NT - D * WAVE;
            const bool out = hlane < NX;
            int ovl = 0, owl = 0;
            if (out) xch_out_lane(0, hlane, BV, BW, &ovl, &owl);
            const int ocell = (owl + 1) * GW + (ovl + 1);
            __syncthreads();
            __syncthreads();
            for (int t = tb; t <= te; ++t) {
                if (out && t > tb)
                    x_put(xch + xch_word(B.xoff, B.tlo, NX, XW, t - 1, hlane), grid[((t - 1) & 3) * GC + ocell], tag);
                lds_barrier();
            }
            if (out) x_put(xch + xch_word(B.xoff, B.tlo, NX, XW, te, hlane), grid[(te & 3) * GC + ocell], tag);
        } else if (l >= NT) {
            // ---------------- incoming waves: loads and checks only.  Wave iw serves
            // the hyperplanes t with (t - tb) % D == iw and loads the entry of its next
            // one (t + D) right after taking t, so each wave has one load in flight and
            // a wait for it never waits for another hyperplane's load.
            const int hlane = (l - NT) % WAVE, iw = (l - NT) / WAVE;
            Halo hin;
            int kk = 0, j = 0;
            if (xch_halo_role(0, hlane, BV, BW, &kk, &j)) {
                hin.role = true;
                hin.cell = kk == 0 ? (hlane + 1) * GW : kk == 1 ? hlane - BW + 1 : 0;
                const int prod = kk == 0 ? B.pred[0] : kk == 1 ? B.pred[1] : B.pred[2];
                if (prod >= 0) {
                    const BlockDev& P = blocks[prod];
                    hin.ptb = P.tb;
                    hin.pte = P.te;
                    hin.ptlo = P.tlo;
                    hin.pxoff = P.xoff;
                    hin.j = j;
                }
            }
            __syncthreads();
            XEnt<T> hx;
            if (hin.role) {
                if (iw == 0) {
                    for (int s = tb - 3; s < tb; ++s) {
                        XEnt<T> e;
                        halo_issue(hin, xch, NX, s, e);
                        grid[(s & 3) * GC + hin.cell] = halo_take<T>(hin, xch, NX, s, e, tag, flags);
                    }
                }
                halo_issue(hin, xch, NX, tb + iw, hx);
            }
            __syncthreads();
            for (int T0 = tb; T0 <= te; T0 += D) {
#pragma unroll
                for (int q = 0; q < D; ++q) {
                    const int t = T0 + q;
                    if (t > te) break;
                    if (hin.role && q == iw) {
                        grid[(t & 3) * GC + hin.cell] = halo_take<T>(hin, xch, NX, t, hx, tag, flags);
                        halo_issue(hin, xch, NX, t + D, hx);
                    }
                    lds_barrier();
                }
            }
        } else {
            // ---------------- compute waves
            int vl = 0, wl = 0;
            lane_rc(l, BV, &vl, &wl);
            const int cell = (wl + 1) * GW + (vl + 1);
            const LaneDev& Ln = lanes[(int64_t)b * NT + l];
            const bool valid = Ln.v != 0;
            const int n = tets[B.tet].n, v = Ln.v, wrow = Ln.w, y = v - wrow, xmax = n - 1 - v;
            const int64_t rp = Ln.rp[R_SELF];
            T coef[7 * (NC > 0 ? NC : 1)];
            T xm = 0, ihw = 0;
            if (!STORED && valid) {
                const T* c = tab + ((int64_t)b * NT + l) * (2 + 15 * NC);
                xm = c[0];
                ihw = c[1];
#pragma unroll
                for (int i = 0; i < 7 * NC; ++i) coef[i] = c[2 + i];
            }
            // MODE 0: factors from the stored arrays (STORED) or the surrogate only;
            // V1, MODE 1 (no row with y = 1 or z = 1 in the block): the exact factors
            // of the row's two boundary points x = 1 and x = xmax held in registers;
            // V1, MODE 2: exact factors streamed from set F with the operands
            // (zero entry for points outside F).
            auto compute = [&](auto mode_c, auto u_c) {
                constexpr int MODE = decltype(mode_c)::value, UU = decltype(u_c)::value;
                using LT = typename Pick<STORED, double, T>::type;
                // the lane's set index, read once (a lazy read inside the loop would
                // sit in a branch and wait for every load in flight)
                const int64_t f0 = V1 && valid ? (int64_t)Ln.v1f[0] : 0;
                T P0[MODE == 1 ? 7 : 1], P1[MODE == 1 ? 7 : 1];
                if constexpr (MODE == 1) {
                    const int64_t j0 = valid ? f0 : v1s - 1;
                    const int64_t j1 = valid ? f0 + (xmax >= 2 ? 1 : 0) : v1s - 1;
                    T a[8], bq[8];
                    load8(v1 + j0 * 8, a);
                    load8(v1 + j1 * 8, bq);
#pragma unroll
                    for (int s = 0; s < 7; ++s) {
                        P0[s] = a[s];
                        P1[s] = bq[s];
                    }
                }
                // Operands of two batches of UU hyperplanes in flight, in ping-pong buffers:
                // a batch issues the next batch's loads, then runs its UU hyperplanes.  Every
                // load and store is issued unconditionally (hyperplanes clamped to the block
                // window; inactive points and unused lanes load from the zero region), so
                // the number of memory operations between a load and its use is the same on
                // every path and the wait before a use covers that load only.
                constexpr int NL = (STORED || MODE == 2) ? 7 * UU : 1;
                using RE = typename Pick<OVL, XEnt<T>, T>::type;
                RE rA[UU], rB[UU];
                LT LA[NL], LB[NL];
                int rspin = rspin0;  // polls of a stale residual entry before computing it here
                // OVL: the residual kernel marks every (64-lane group, hyperplane band)
                // it has finished; before loading the residuals of a new band the
                // wave waits for its group's mark, so it does not poll the entries
                // point by point.  The wait is short and bounded (the per-point tags
                // stay the guarantee): if a mark does not come, the residual kernel
                // is not running beside this one (kernels serialised, e.g. under a
                // counter profiler), and the wave stops waiting for marks and
                // computes missing residuals itself.
                int band_ok = -1;
                auto wait_band = [&](const int th) {
                    if constexpr (OVL) {
                        const int k = min(th, te) / RES_T;
                        if (k > band_ok) {
                            const uint64_t* fl = rflag + ((int64_t)b * (NT / WAVE) + l / WAVE) * nbands + k;
                            int it = 0;
                            for (; it < 512 && (uint32_t)ld_dev(fl) != tag; ++it) __builtin_amdgcn_s_sleep(8);
                            band_ok = it < 512 ? k : (1 << 30);
                        }
                    }
                };
                auto prefetch = [&](const int T0, RE (&rx)[UU], LT (&Lx)[NL]) {
                    wait_band(T0 + UU - 1);
#pragma unroll
                    for (int q = 0; q < UU; ++q) {
                        // inactive points read the (cache-resident) zero region, not padding
                        const int t = min(T0 + q, te), xq = t - 2 * v - wrow;
                        const bool act = valid && xq >= 1 && xq <= xmax;
                        const int64_t i = act ? rp + (int64_t)NT * t : 0;
                        if constexpr (OVL) x_get(rx[q], rt + i * XW);
                        else rx[q] = r[i];
                        if constexpr (STORED) {
#pragma unroll
                            for (int s = 0; s < 7; ++s) Lx[q * 7 + s] = Lf[(int64_t)s * S + i];
                        }
                        if constexpr (MODE == 2) {
                            const int pos = v1f_pos_sel(xq, xmax, y, wrow);
                            const int64_t j = act && pos >= 0 ? f0 + pos : v1s - 1;
                            T a[8];
                            load8(v1 + j * 8, a);
#pragma unroll
                            for (int s = 0; s < 7; ++s) Lx[q * 7 + s] = a[s];
                        }
                    }
                };
                auto batch = [&](const int T0, RE (&rcur)[UU], LT (&Lcur)[NL], RE (&rnxt)[UU], LT (&Lnxt)[NL]) {
                    prefetch(T0 + UU, rnxt, Lnxt);
#pragma unroll
                    for (int q = 0; q < UU; ++q) {
                        const int t = T0 + q;
                        if (t > te) break;
                        const int x = t - 2 * v - wrow;
                        T val = (T)0;
                        if (valid && x >= 1 && x <= xmax) {
                            const T* g1 = grid + ((t - 1) & 3) * GC;
                            const T* g2 = grid + ((t - 2) & 3) * GC;
                            const T* g3 = grid + ((t - 3) & 3) * GC;
                            // neighbours p + d: w (own, t-1), s (v-1, t-2), se (v-1, t-1), bnw (w-1, t-2),
                            // bn (w-1, t-1), bc (v-1 w-1, t-3), be (v-1 w-1, t-2)
                            const T nb[7] = {g1[cell], g2[cell - 1], g1[cell - 1], g2[cell - GW],
                                             g1[cell - GW], g3[cell - GW - 1], g2[cell - GW - 1]};
                            T acc;
                            if constexpr (OVL) {
                                acc = x_val(rcur[q]);
                                if (!x_ok(rcur[q], tag))
                                    acc = late_residual<T>(rt + (rp + (int64_t)NT * t) * XW, tag, rspin, Ln, NT, S, t,
                                                           A8, xo, bo);
                            } else {
                                acc = rcur[q];
                            }
                            if constexpr (STORED) {
#pragma unroll
                                for (int jj = 0; jj < 7; ++jj) acc -= (T)Lcur[q * 7 + ORD[jj]] * nb[ORD[jj]];
                            } else {
                                const T eta = ((T)x - xm) * ihw;
                                T Lv[7];
#pragma unroll
                                for (int s = 0; s < 7; ++s) Lv[s] = horner<NC>(coef + s * NC, eta);
                                // plain selects (no branches: the choice differs lane by lane)
                                if constexpr (MODE == 1) {
                                    const bool b0 = x == 1, b1 = x == xmax;
#pragma unroll
                                    for (int s = 0; s < 7; ++s) {
                                        T sel = b1 ? P1[s] : Lv[s];
                                        Lv[s] = b0 ? P0[s] : sel;
                                    }
                                } else if constexpr (MODE == 2) {
                                    const bool bf = v1f_pos_sel(x, xmax, y, wrow) >= 0;
#pragma unroll
                                    for (int s = 0; s < 7; ++s) Lv[s] = bf ? (T)Lcur[q * 7 + s] : Lv[s];
                                }
#pragma unroll
                                for (int jj = 0; jj < 7; ++jj) acc -= Lv[ORD[jj]] * nb[ORD[jj]];
                            }
                            val = acc;
                        }
                        // inactive points store 0 into a slot that stays 0 (own padding or the zero region)
                        w[rp + (int64_t)NT * t] = val;
                        grid[(t & 3) * GC + cell] = val;
                        lds_barrier();
                    }
                };
                __syncthreads();
                prefetch(tb, rA, LA);
                __syncthreads();
                for (int T0 = tb; T0 <= te; T0 += 2 * UU) {
                    batch(T0, rA, LA, rB, LB);
                    if (T0 + UU > te) break;
                    batch(T0 + UU, rB, LB, rA, LA);
                }
            };
            if constexpr (!V1) compute(IC<0>{}, IC<U>{});
            else if (B.edge) compute(IC<2>{}, IC<V1_UE<T>()>{});
            else compute(IC<1>{}, IC<U>{});
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------- backward

template <typename T, bool STORED, bool V1, int U, int D, int NC, int BV, int BW>
__global__ void __launch_bounds__(BV* BW + (D + 1) * WAVE)
    k_bwd_flow(const TetDev* __restrict__ tets, const BlockDev* __restrict__ blocks, const LaneDev* __restrict__ lanes,
               int nblocks, int64_t S, const double* __restrict__ Lb, const T* __restrict__ tab,
               const T* __restrict__ v1, int64_t v1s, const T* __restrict__ w, double* __restrict__ xs,
               const int32_t* __restrict__ order, uint64_t* __restrict__ xch, int32_t* __restrict__ ticket,
               int32_t* __restrict__ flags) {
    constexpr int NT = BV * BW;
    constexpr int GW = BV + 1;
    constexpr int GC = (BV + 1) * (BW + 1);
    constexpr int NX = BV + BW;
    constexpr int XW = XEnt<T>::W;
    static_assert(NT % WAVE == 0 && NX + 1 <= WAVE, "block shape");
    __shared__ T grid[4 * GC];
    __shared__ int s_ticket;
    const int l = threadIdx.x;
    const uint32_t tag = (uint32_t)ticket[2];
    for (;;) {
        if (l == 0) s_ticket = atomicAdd(&ticket[1], 1);
        __syncthreads();
        const int k = s_ticket;
        __syncthreads();
        if (k >= nblocks) return;
        const int b = order[k];
        const BlockDev B = blocks[b];
        const int tb = B.tb, te = B.te;
        for (int i = l; i < 4 * GC; i += NT + (D + 1) * WAVE) grid[i] = (T)0;
        if (l >= NT + D * WAVE) {
            // ---------------- outgoing wave (edge values of hyperplane t+1)
            const int hlane = l - NT - D * WAVE;
            const bool out = hlane < NX;
            int ovl = 0, owl = 0;
            if (out) xch_out_lane(1, hlane, BV, BW, &ovl, &owl);
            const int ocell = owl * GW + ovl;
            __syncthreads();
            __syncthreads();
            for (int t = te; t >= tb; --t) {
                if (out && t < te)
                    x_put(xch + xch_word(B.xoff, B.tlo, NX, XW, t + 1, hlane), grid[((t + 1) & 3) * GC + ocell], tag);
                lds_barrier();
            }
            if (out) x_put(xch + xch_word(B.xoff, B.tlo, NX, XW, tb, hlane), grid[(tb & 3) * GC + ocell], tag);
        } else if (l >= NT) {
            // ---------------- incoming waves (halo at column BV and row BW of the grid);
            // wave iw serves the hyperplanes t with (te - t) % D == iw
            const int hlane = (l - NT) % WAVE, iw = (l - NT) / WAVE;
            Halo hin;
            int kk = 0, j = 0;
            if (xch_halo_role(1, hlane, BV, BW, &kk, &j)) {
                hin.role = true;
                hin.cell = kk == 0 ? hlane * GW + BV : kk == 1 ? BW * GW + (hlane - BW) : BW * GW + BV;
                const int prod = kk == 0 ? B.succ[0] : kk == 1 ? B.succ[1] : B.succ[2];
                if (prod >= 0) {
                    const BlockDev& P = blocks[prod];
                    hin.ptb = P.tb;
                    hin.pte = P.te;
                    hin.ptlo = P.tlo;
                    hin.pxoff = P.xoff;
                    hin.j = j;
                }
            }
            __syncthreads();
            XEnt<T> hx;
            if (hin.role) {
                if (iw == 0) {
                    for (int s = te + 3; s > te; --s) {
                        XEnt<T> e;
                        halo_issue(hin, xch, NX, s, e);
                        grid[(s & 3) * GC + hin.cell] = halo_take<T>(hin, xch, NX, s, e, tag, flags);
                    }
                }
                halo_issue(hin, xch, NX, te - iw, hx);
            }
            __syncthreads();
            for (int T0 = te; T0 >= tb; T0 -= D) {
#pragma unroll
                for (int q = 0; q < D; ++q) {
                    const int t = T0 - q;
                    if (t < tb) break;
                    if (hin.role && q == iw) {
                        grid[(t & 3) * GC + hin.cell] = halo_take<T>(hin, xch, NX, t, hx, tag, flags);
                        halo_issue(hin, xch, NX, t - D, hx);
                    }
                    lds_barrier();
                }
            }
        } else {
            // ---------------- compute waves
            int vl = 0, wl = 0;
            lane_rc(l, BV, &vl, &wl);
            const int cell = wl * GW + vl;
            const LaneDev& Ln = lanes[(int64_t)b * NT + l];
            const bool valid = Ln.v != 0;
            const int n = tets[B.tet].n, v = Ln.v, wrow = Ln.w, y = v - wrow, xmax = n - 1 - v;
            const int64_t rp = Ln.rp[R_SELF];
            T coef[8 * (NC > 0 ? NC : 1)];
            T xm = 0, ihw = 0;
            if (!STORED && valid) {
                const T* c = tab + ((int64_t)b * NT + l) * (2 + 15 * NC);
                xm = c[0];
                ihw = c[1];
#pragma unroll
                for (int i = 0; i < 8 * NC; ++i) coef[i] = c[2 + 7 * NC + i];
            }
            // MODE 0: weights from the stored arrays (STORED) or the surrogate only;
            // V1, MODE 1 (no row with y <= 2 or z = 1 in the block): the weights of the
            // row's points of set B (x in {1, 2, xmax-1, xmax}) held in registers;
            // V1, MODE 2: weights of set B streamed with the operands.
            auto compute = [&](auto mode_c, auto u_c) {
                constexpr int MODE = decltype(mode_c)::value, UU = decltype(u_c)::value;
                using LT = typename Pick<STORED, double, T>::type;
                // the lane's set index, read once (see the forward sweep)
                const int64_t b0 = V1 && valid ? (int64_t)Ln.v1b : 0;
                T P[MODE == 1 ? 32 : 1];
                if constexpr (MODE == 1) {
                    const int cnt = valid ? v1b_count(xmax, y, wrow) : 0;
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int64_t j = k < cnt ? b0 + k : v1s - 1;
                        T a[8];
                        load8(v1 + j * 8, a);
#pragma unroll
                        for (int e = 0; e < 8; ++e) P[k * 8 + e] = a[e];
                    }
                }
                // ping-pong operand buffers and unconditional memory operations, as in the
                // forward sweep
                constexpr int NL = (STORED || MODE == 2) ? 8 * UU : 1;
                T wA[UU], wB[UU];
                double xA[UU], xB[UU];
                LT LA[NL], LB[NL];
                auto prefetch = [&](const int T0, T (&wx)[UU], double (&xx)[UU], LT (&Lx)[NL]) {
#pragma unroll
                    for (int q = 0; q < UU; ++q) {
                        const int t = max(T0 - q, tb), xq = t - 2 * v - wrow;
                        const bool act = valid && xq >= 1 && xq <= xmax;
                        const int64_t i = act ? rp + (int64_t)NT * t : 0;
                        wx[q] = w[i];
                        xx[q] = xs[i];
                        if constexpr (STORED) {
#pragma unroll
                            for (int s = 0; s < 8; ++s) Lx[q * 8 + s] = Lb[(int64_t)s * S + i];
                        }
                        if constexpr (MODE == 2) {
                            const int pos = v1b_pos_sel(xq, xmax, y, wrow);
                            const int64_t j = act && pos >= 0 ? b0 + pos : v1s - 1;
                            T a[8];
                            load8(v1 + j * 8, a);
#pragma unroll
                            for (int e = 0; e < 8; ++e) Lx[q * 8 + e] = a[e];
                        }
                    }
                };
                auto batch = [&](const int T0, T (&wcur)[UU], double (&xcur)[UU], LT (&Lcur)[NL], T (&wnxt)[UU],
                                 double (&xnxt)[UU], LT (&Lnxt)[NL]) {
                    prefetch(T0 - UU, wnxt, xnxt, Lnxt);
#pragma unroll
                    for (int q = 0; q < UU; ++q) {
                        const int t = T0 - q;
                        if (t < tb) break;
                        const int x = t - 2 * v - wrow;
                        T val = (T)0;
                        if (valid && x >= 1 && x <= xmax) {
                            const T* g1 = grid + ((t + 1) & 3) * GC;
                            const T* g2 = grid + ((t + 2) & 3) * GC;
                            const T* g3 = grid + ((t + 3) & 3) * GC;
                            // upper neighbours p - d: e (own, t+1), n (v+1, t+2), nw (v+1, t+1),
                            // tse (w+1, t+2), ts (w+1, t+1), tc (v+1 w+1, t+3), tw (v+1 w+1, t+2)
                            const T nb[7] = {g1[cell], g2[cell + 1], g1[cell + 1], g2[cell + GW],
                                             g1[cell + GW], g3[cell + GW + 1], g2[cell + GW + 1]};
                            T acc;
                            if constexpr (STORED) {
                                acc = wcur[q] * (T)Lcur[q * 8];
#pragma unroll
                                for (int jj = 0; jj < 7; ++jj) acc -= (T)Lcur[q * 8 + 1 + ORD[jj]] * nb[ORD[jj]];
                            } else {
                                const T eta = ((T)x - xm) * ihw;
                                T Wv[8];  // 1/D, then the seven upper weights
#pragma unroll
                                for (int e = 0; e < 8; ++e) Wv[e] = horner<NC>(coef + e * NC, eta);
                                // plain selects (no branches: the choice differs lane by lane)
                                if constexpr (MODE == 1) {
                                    const int pos = v1b_pos_sel(x, xmax, y, wrow);
                                    const bool s0 = pos == 0, s1 = pos == 1, s2 = pos == 2, s3 = pos == 3;
#pragma unroll
                                    for (int e = 0; e < 8; ++e) {
                                        T sel = s3 ? P[24 + e] : Wv[e];
                                        sel = s2 ? P[16 + e] : sel;
                                        sel = s1 ? P[8 + e] : sel;
                                        Wv[e] = s0 ? P[e] : sel;
                                    }
                                } else if constexpr (MODE == 2) {
                                    const bool bb = v1b_pos_sel(x, xmax, y, wrow) >= 0;
#pragma unroll
                                    for (int e = 0; e < 8; ++e) Wv[e] = bb ? (T)Lcur[q * 8 + e] : Wv[e];
                                }
                                acc = wcur[q] * Wv[0];
#pragma unroll
                                for (int jj = 0; jj < 7; ++jj) acc -= Wv[1 + ORD[jj]] * nb[ORD[jj]];
                            }
                            val = acc;
                        }
                        // inactive points write their (zero) x slot back unchanged
                        xs[rp + (int64_t)NT * t] = xcur[q] + (double)val;
                        grid[(t & 3) * GC + cell] = val;
                        lds_barrier();
                    }
                };
                __syncthreads();
                prefetch(te, wA, xA, LA);
                __syncthreads();
                for (int T0 = te; T0 >= tb; T0 -= 2 * UU) {
                    batch(T0, wA, xA, LA, wB, xB, LB);
                    if (T0 - UU < tb) break;
                    batch(T0 - UU, wB, xB, LB, wA, xA, LA);
                }
            };
            if constexpr (!V1) compute(IC<0>{}, IC<U>{});
            else if (B.edge) compute(IC<2>{}, IC<V1_UE<T>()>{});
            else compute(IC<1>{}, IC<U>{});
        }
        __syncthreads();
    }
}

// Before every dataflow sweep: reset the work counters and advance the tag.
__global__ void k_flow_reset(int32_t* __restrict__ ticket) {
    if (threadIdx.x == 0) {
        ticket[0] = 0;
        ticket[1] = 0;
        uint32_t e = (uint32_t)ticket[2] + 1u;
        if (e == 0) e = 1;  // tag 0 is the cleared buffer
        ticket[2] = (int32_t)e;
    }
}

// ------------------------------------------------------------------ launchers

namespace {

// Batch depth U (operands of the next U hyperplanes are loaded while the
// current U run) and halo lead D = number of incoming waves.  Both batches of
// loads must fit the 63-entry vector memory counter: stored factors load 8
// (forward) or 10 (backward) values per hyperplane.
//
// With one incoming wave the entry of hyperplane t+1 is loaded during
// hyperplane t and every hyperplane waits one exchange round trip (a
// device-coherent load, ~0.45 us): the stale-entry poll loop makes the
// compiler wait for all of a wave's outstanding loads, so a deeper lead in one
// wave hid nothing.  D waves with one load in flight each hide the round trip
// over D hyperplanes.  Level 9, FP32 surrogate, 16 x 16 blocks: forward /
// backward 0.674 / 0.687 ms with D = 1, 0.487 / 0.555 with D = 2, 0.507 /
// 0.563 with D = 3 (D = 3 is slower on the small tetrahedra of a batch).
// Making a block wait until its producers are several hyperplanes ahead
// before it starts only added lag per block hop, at every D tried.
constexpr int U_F64 = 3, U_F64B = 2, D_F64 = 2;  // stored factors
constexpr int U_S64 = 4, D_S64 = 2;              // FP64 surrogate
constexpr int U_F32 = 8, D_F32 = 2;              // FP32 surrogate
constexpr int UB_F32 = 6;                        // FP32 backward (level 9, 16 x 16: 0.529 vs 0.537 ms with 8)
// With the overlapped residual the forward sweep advances at the rate the
// residual kernel produces its input, and every register it holds is one the
// residual kernel beside it cannot use: shallower operand batches.  The
// residual's traffic also lengthens the exchange round trip, which a third
// incoming wave hides for the FP32 sweep (level 9, 16 x 16: 1.414 vs 1.442 ms
// per step; four waves leave the residual no room beside a full grid).
constexpr int UO_F64 = 2, UO_S64 = 2, UO_F32 = 4;
constexpr int DO_F32 = 3;

template <int BV, int BW>
struct Shape {
    static constexpr int NT = BV * BW;
    template <bool OVL>
    static const void* fwd_stored_ptr() {
        return (const void*)k_fwd_flow<double, true, false, OVL, (OVL ? UO_F64 : U_F64), D_F64, 0, BV, BW>;
    }
    static const void* bwd_stored_ptr() {
        return (const void*)k_bwd_flow<double, true, false, U_F64B, D_F64, 0, BV, BW>;
    }
    template <int NC, bool V1, bool OVL>
    static const void* fwd_ptr(int variant) {
        if (variant == 1) return (const void*)k_fwd_flow<double, false, V1, OVL, (OVL ? UO_S64 : U_S64), D_S64, NC, BV, BW>;
        return (const void*)k_fwd_flow<float, false, V1, OVL, (OVL ? UO_F32 : U_F32), (OVL ? DO_F32 : D_F32), NC, BV, BW>;
    }
    template <int NC, bool V1>
    static const void* bwd_ptr(int variant) {
        if (variant == 1) return (const void*)k_bwd_flow<double, false, V1, U_S64, D_S64, NC, BV, BW>;
        return (const void*)k_bwd_flow<float, false, V1, UB_F32, D_F32, NC, BV, BW>;
    }
    template <bool OVL>
    static void fwd_stored(const Ctx& c, const Flow& f, hipStream_t st) {
        k_fwd_flow<double, true, false, OVL, (OVL ? UO_F64 : U_F64), D_F64, 0, BV, BW><<<f.grid, NT + (D_F64 + 1) * WAVE, 0, st>>>(
            c.tets, c.blocks, c.lanes, c.nblocks, c.S, c.Lf, nullptr, nullptr, 0, (const double*)c.r, f.rt, c.A8,
            f.xo, f.bo, f.rspin, f.rflag, f.nbands, (double*)c.w, f.order_fwd, f.xch, f.ticket, f.flags);
    }
    static void bwd_stored(const Ctx& c, const Flow& f, double* x, hipStream_t st) {
        k_bwd_flow<double, true, false, U_F64B, D_F64, 0, BV, BW><<<f.grid, NT + (D_F64 + 1) * WAVE, 0, st>>>(
            c.tets, c.blocks, c.lanes, c.nblocks, c.S, c.Lb, nullptr, nullptr, 0, (const double*)c.w, x, f.order_bwd,
            f.xch, f.ticket, f.flags);
    }
    template <int NC, bool V1, bool OVL>
    static void fwd(const Ctx& c, const Flow& f, int variant, hipStream_t st) {
        if (variant == 1)
            k_fwd_flow<double, false, V1, OVL, (OVL ? UO_S64 : U_S64), D_S64, NC, BV, BW><<<f.grid, NT + (D_S64 + 1) * WAVE, 0, st>>>(
                c.tets, c.blocks, c.lanes, c.nblocks, c.S, nullptr, c.tab64, (const double*)c.v1f, c.v1f_stride,
                (const double*)c.r, f.rt, c.A8, f.xo, f.bo, f.rspin, f.rflag, f.nbands, (double*)c.w, f.order_fwd, f.xch, f.ticket, f.flags);
        else
            k_fwd_flow<float, false, V1, OVL, (OVL ? UO_F32 : U_F32), (OVL ? DO_F32 : D_F32), NC, BV, BW>
                <<<f.grid, NT + ((OVL ? DO_F32 : D_F32) + 1) * WAVE, 0, st>>>(
                c.tets, c.blocks, c.lanes, c.nblocks, c.S, nullptr, c.tab32, (const float*)c.v1f, c.v1f_stride,
                (const float*)c.r, f.rt, c.A8, f.xo, f.bo, f.rspin, f.rflag, f.nbands, (float*)c.w, f.order_fwd, f.xch, f.ticket, f.flags);
    }
    template <int NC, bool V1>
    static void bwd(const Ctx& c, const Flow& f, int variant, double* x, hipStream_t st) {
        if (variant == 1)
            k_bwd_flow<double, false, V1, U_S64, D_S64, NC, BV, BW><<<f.grid, NT + (D_S64 + 1) * WAVE, 0, st>>>(
                c.tets, c.blocks, c.lanes, c.nblocks, c.S, nullptr, c.tab64, (const double*)c.v1b, c.v1b_stride,
                (const double*)c.w, x, f.order_bwd, f.xch, f.ticket, f.flags);
        else
            k_bwd_flow<float, false, V1, UB_F32, D_F32, NC, BV, BW><<<f.grid, NT + (D_F32 + 1) * WAVE, 0, st>>>(
                c.tets, c.blocks, c.lanes, c.nblocks, c.S, nullptr, c.tab32, (const float*)c.v1b, c.v1b_stride,
                (const float*)c.w, x, f.order_bwd, f.xch, f.ticket, f.flags);
    }
};

// NC = dg_x + 1 in [1, 7]; stored factors use NC = 0 (one instantiation)
#define ILU_NC_SWITCH(NCV, CALL) \
    switch ((NCV)) {             \
    case 1: CALL(1); break;      \
    case 2: CALL(2); break;      \
    case 3: CALL(3); break;      \
    case 4: CALL(4); break;      \
    case 5: CALL(5); break;      \
    case 6: CALL(6); break;      \
    default: CALL(7); break;     \
    }

// Resident workgroups per CU of both sweep kernels (the forward one in both
// residual modes where the handle can use the overlapped one).
template <int BV, int BW>
int resident(int variant, int NC, bool v1) {
    const void* kf = nullptr;
    const void* ko = nullptr;
    const void* kb = nullptr;
    if (variant == 0) {
        kf = Shape<BV, BW>::template fwd_stored_ptr<false>();
        ko = Shape<BV, BW>::template fwd_stored_ptr<true>();
        kb = Shape<BV, BW>::bwd_stored_ptr();
    } else if (v1) {
#define ILU_PTRS(N)                                                       \
    (kf = ko = Shape<BV, BW>::template fwd_ptr<N, true, false>(variant), \
     kb = Shape<BV, BW>::template bwd_ptr<N, true>(variant))
        ILU_NC_SWITCH(NC, ILU_PTRS)
#undef ILU_PTRS
    } else {
#define ILU_PTRS(N)                                                    \
    (kf = Shape<BV, BW>::template fwd_ptr<N, false, false>(variant), \
     ko = Shape<BV, BW>::template fwd_ptr<N, false, true>(variant),  \
     kb = Shape<BV, BW>::template bwd_ptr<N, false>(variant))
        ILU_NC_SWITCH(NC, ILU_PTRS)
#undef ILU_PTRS
    }
    const int nthreads = BV * BW + (1 + (variant == 0 ? D_F64 : variant == 1 ? D_S64 : D_F32)) * WAVE;
    // the overlapped FP32 forward sweep has one more incoming wave (not with V1, whose kernel is kf)
    const int nthreads_o = variant == 2 && !v1 ? BV * BW + (1 + DO_F32) * WAVE : nthreads;
    int a = 0, b = 0, o = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, kf, nthreads, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, ko, nthreads_o, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kb, nthreads, 0) != hipSuccess)
        return 1;
    return std::min(a, std::min(o, b));
}

template <int BV, int BW>
void run_fwd(const Ctx& c, const Flow& f, int variant, hipStream_t st) {
    if (variant == 0) {
        if (f.rt) Shape<BV, BW>::template fwd_stored<true>(c, f, st);
        else Shape<BV, BW>::template fwd_stored<false>(c, f, st);
        return;
    }
    if (c.v1f) {
#define ILU_FWD(N) Shape<BV, BW>::template fwd<N, true, false>(c, f, variant, st)
        ILU_NC_SWITCH(c.NC, ILU_FWD)
#undef ILU_FWD
    } else if (f.rt) {
#define ILU_FWD(N) Shape<BV, BW>::template fwd<N, false, true>(c, f, variant, st)
        ILU_NC_SWITCH(c.NC, ILU_FWD)
#undef ILU_FWD
    } else {
#define ILU_FWD(N) Shape<BV, BW>::template fwd<N, false, false>(c, f, variant, st)
        ILU_NC_SWITCH(c.NC, ILU_FWD)
#undef ILU_FWD
    }
}

template <int BV, int BW>
void run_bwd(const Ctx& c, const Flow& f, int variant, double* x, hipStream_t st) {
    if (variant == 0) {
        Shape<BV, BW>::bwd_stored(c, f, x, st);
        return;
    }
    if (c.v1b) {
#define ILU_BWD(N) Shape<BV, BW>::template bwd<N, true>(c, f, variant, x, st)
        ILU_NC_SWITCH(c.NC, ILU_BWD)
#undef ILU_BWD
    } else {
#define ILU_BWD(N) Shape<BV, BW>::template bwd<N, false>(c, f, variant, x, st)
        ILU_NC_SWITCH(c.NC, ILU_BWD)
#undef ILU_BWD
    }
}

}  // namespace

bool flow_shape_supported(int bv, int bw) {
    return (bv == 8 && bw == 8) || (bv == 16 && bw == 16) || (bv == 16 && bw == 32);
}

int flow_max_resident(int variant, int NC, bool v1, int bv, int bw) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        cus = 1;
    int per_cu = 1;
    if (bv == 8 && bw == 8) per_cu = resident<8, 8>(variant, NC, v1);
    else if (bv == 16 && bw == 16) per_cu = resident<16, 16>(variant, NC, v1);
    else per_cu = resident<16, 32>(variant, NC, v1);
    if (per_cu < 1) per_cu = 1;
    return per_cu * cus;
}

void launch_flow_reset(const Flow& f, hipStream_t st) { k_flow_reset<<<1, 64, 0, st>>>(f.ticket); }

void launch_fwd_flow(const Ctx& c, const Flow& f, int variant, hipStream_t st) {
    if (c.bv == 8 && c.bw == 8) run_fwd<8, 8>(c, f, variant, st);
    else if (c.bv == 16 && c.bw == 16) run_fwd<16, 16>(c, f, variant, st);
    else run_fwd<16, 32>(c, f, variant, st);
}

void launch_bwd_flow(const Ctx& c, const Flow& f, int variant, double* x, hipStream_t st) {
    if (c.bv == 8 && c.bw == 8) run_bwd<8, 8>(c, f, variant, x, st);
    else if (c.bv == 16 && c.bw == 16) run_bwd<16, 16>(c, f, variant, x, st);
    else run_bwd<16, 32>(c, f, variant, x, st);
}

}  // namespace ilu
