// Persistent dataflow sweeps (Alg. 2 on the hyperplane schedule without a
// global barrier per hyperplane).
//
// One workgroup = one wavefront = one 8 x 8 block of rows at a time.  A
// workgroup takes blocks from a ticket counter in a topological order of the
// block dependency graph, so every block it waits for is owned by a resident
// workgroup that took its ticket earlier: the wait chain always ends.
//
// Inside a block the 64 lanes advance hyperplane by hyperplane in lock step.
// Values of the last few hyperplanes live in an LDS ring of 9 x 9 cells per
// hyperplane: 8 x 8 own rows plus one halo column and one halo row holding
// rows of the neighbouring blocks.  Halo values are produced by other
// workgroups; they are read from the w stream with device-coherent loads once
// the producer's progress counter shows them finished, H hyperplanes ahead of
// use, and committed to the ring a batch later.  w is written with
// device-coherent stores and each block publishes its progress every H
// hyperplanes after waiting for those stores.
//
// A wait that exceeds a fixed bound sets flags[2] and gives up, so a logic
// error can never hang the device.
#include <hip/hip_runtime.h>

#include "kernels_common.h"
#include "sweep_kernels.h"

namespace ilu {

namespace {

constexpr int GRIDC = 81;           // 9 x 9 cells per hyperplane
constexpr long SPIN_LIMIT = 1L << 24;

template <typename T>
__device__ __forceinline__ void st_dev(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_dev(const T* p) {
    return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void wait_stores() {
    // s_waitcnt vmcnt(0): every earlier vector memory access of this wave
    // (including the device-coherent w stores) has completed.
    __builtin_amdgcn_s_waitcnt(0x0F70);
}

template <int NC, typename T>
__device__ __forceinline__ T horner(const T* c, T eta) {
    T acc = c[NC - 1];
#pragma unroll
    for (int i = NC - 2; i >= 0; --i) acc = acc * eta + c[i];
    return acc;
}

struct Halo {
    int cell = -1;     // ring cell this lane fills (-1: no halo role)
    int64_t rp = 0;    // row pointer of the halo row
    int prod = -1;     // producing block (-1: row outside the lattice, value 0)
    int ptb = 0, pte = 0;
};

// Wait until block `prod` has published at least `need` finished hyperplanes.
// `known` caches the last value observed, so most calls return at once.
// A wait that exceeds the bound (or a bound hit anywhere else) gives up.
__device__ __forceinline__ void wait_progress(const int32_t* progress, int prod, int need, int& known,
                                              int32_t* flags) {
    if (known >= need) return;
    long spins = 0;
    int v = ld_dev(&progress[prod]);
    while (v < need) {
        __builtin_amdgcn_s_sleep(1);
        ++spins;
        if ((spins & 1023) == 0 && ld_dev(&flags[2])) break;
        if (spins > SPIN_LIMIT) {
            atomicOr(&flags[2], 1);
            break;
        }
        v = ld_dev(&progress[prod]);
    }
    known = v;
}

}  // namespace

// ------------------------------------------------------------------ forward

template <typename T, bool STORED, int H, int NC>
__global__ void __launch_bounds__(64) k_fwd_flow(const TetDev* __restrict__ tets, const BlockDev* __restrict__ blocks,
                                                 const LaneDev* __restrict__ lanes, int nblocks, int64_t S,
                                                 const double* __restrict__ Lf, const T* __restrict__ tab,
                                                 const T* __restrict__ r, T* __restrict__ w,
                                                 const int32_t* __restrict__ order, int32_t* __restrict__ progress,
                                                 int32_t* __restrict__ ticket, int32_t* __restrict__ flags) {
    constexpr int RING = 2 * H >= 8 ? 2 * H : 8;
    static_assert((RING & (RING - 1)) == 0 && RING >= H + 2, "ring size");
    __shared__ T ring[RING * GRIDC];
    __shared__ int s_ticket;
    const int lane = threadIdx.x;
    const int vl = lane & 7, wl = lane >> 3;
    const int cell = (wl + 1) * 9 + (vl + 1);
    for (;;) {
        if (lane == 0) s_ticket = atomicAdd(&ticket[0], 1);
        __syncthreads();
        const int k = s_ticket;
        __syncthreads();
        if (k >= nblocks) return;
        const int b = order[k];
        const BlockDev B = blocks[b];
        const LaneDev& Ln = lanes[(int64_t)b * LANES + lane];
        const bool valid = Ln.v != 0;
        const int n = tets[B.tet].n, v = Ln.v, wrow = Ln.w;
        const int64_t rp = Ln.rp[R_SELF];
        // halo role of this lane
        Halo hl;
        if (lane < 8) {
            hl.cell = (lane + 1) * 9;
            hl.rp = lanes[(int64_t)b * LANES + lane * 8].rp[R_VM];
            hl.prod = B.pred[0];
        } else if (lane < 16) {
            hl.cell = lane - 7;
            hl.rp = lanes[(int64_t)b * LANES + (lane - 8)].rp[R_WM];
            hl.prod = B.pred[1];
        } else if (lane == 16) {
            hl.cell = 0;
            hl.rp = lanes[(int64_t)b * LANES].rp[R_VMWM];
            hl.prod = B.pred[2];
        }
        if (hl.prod >= 0) {
            hl.ptb = blocks[hl.prod].tb;
            hl.pte = blocks[hl.prod].te;
        }
        // surrogate coefficients of this row (forward table: 7 x NC)
        T coef[7 * (NC > 0 ? NC : 1)];
        T xm = 0, ihw = 0;
        if (!STORED && valid) {
            const T* c = tab + ((int64_t)b * LANES + lane) * (2 + 15 * NC);
            xm = c[0];
            ihw = c[1];
            #pragma unroll
            for (int i = 0; i < 7 * NC; ++i) coef[i] = c[2 + i];
        }
        for (int i = lane; i < RING * GRIDC; i += 64) ring[i] = (T)0;
        __syncthreads();
        const int tb = B.tb, te = B.te;
        // prologue: halo slots tb-3 .. tb+H-2 (one wait for the furthest slot)
        T hreg[H];
        int known = 0, pending = 0;
        if (hl.cell >= 0) {
            if (hl.prod >= 0) {
                const int smax = min(tb + H - 2, hl.pte);
                if (smax >= hl.ptb) wait_progress(progress, hl.prod, smax - hl.ptb + 1, known, flags);
            }
            for (int s = tb - 3; s <= tb + H - 2; ++s) {
                const bool ld = hl.prod >= 0 && s >= hl.ptb && s <= hl.pte;
                ring[(s & (RING - 1)) * GRIDC + hl.cell] = ld ? ld_dev(&w[hl.rp + (int64_t)LANES * s]) : (T)0;
            }
        }
        // operand prefetch registers for the current batch
        T rcur[H];
        double Lcur[STORED ? H * 7 : 1];
#pragma unroll
        for (int q = 0; q < H; ++q) {
            const int t = tb + q;
            rcur[q] = (T)0;
            if (valid && t <= te) {
                rcur[q] = r[rp + (int64_t)LANES * t];
                if (STORED)
#pragma unroll
                    for (int s = 0; s < 7; ++s) Lcur[q * 7 + s] = Lf[(int64_t)s * S + rp + (int64_t)LANES * t];
            }
        }
        __syncthreads();
        for (int T0 = tb; T0 <= te; T0 += H) {
            // commit the halo slots of this batch (loaded during the previous one)
            if (T0 > tb && hl.cell >= 0) {
#pragma unroll
                for (int q = 0; q < H; ++q) ring[((T0 - 1 + q) & (RING - 1)) * GRIDC + hl.cell] = hreg[q];
            }
            // issue halo loads for the next batch: slots T0+H-1 .. T0+2H-2
            if (hl.cell >= 0) {
                const bool more = T0 + H <= te;
                if (hl.prod >= 0 && more) {
                    known = max(known, pending);
                    const int smax = min(T0 + 2 * H - 2, hl.pte);
                    if (smax >= hl.ptb) wait_progress(progress, hl.prod, smax - hl.ptb + 1, known, flags);
                }
#pragma unroll
                for (int q = 0; q < H; ++q) {
                    const int s = T0 + H - 1 + q;
                    const bool ld = more && hl.prod >= 0 && s >= hl.ptb && s <= hl.pte;
                    hreg[q] = ld ? ld_dev(&w[hl.rp + (int64_t)LANES * s]) : (T)0;
                }
                // refresh the producer's progress for the next batch (arrives with the batch)
                if (hl.prod >= 0 && more) pending = ld_dev(&progress[hl.prod]);
            }
            // prefetch operands of the next batch
            T rnxt[H];
            double Lnxt[STORED ? H * 7 : 1];
#pragma unroll
            for (int q = 0; q < H; ++q) {
                const int t = T0 + H + q;
                rnxt[q] = (T)0;
                if (valid && t <= te) {
                    rnxt[q] = r[rp + (int64_t)LANES * t];
                    if (STORED)
#pragma unroll
                        for (int s = 0; s < 7; ++s) Lnxt[q * 7 + s] = Lf[(int64_t)s * S + rp + (int64_t)LANES * t];
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < H; ++q) {
                const int t = T0 + q;
                if (t > te) break;
                const int x = t - 2 * v - wrow;
                T val = (T)0;
                if (valid && x >= 1 && x <= n - 1 - v) {
                    const T* s1 = ring + ((t - 1) & (RING - 1)) * GRIDC;
                    const T* s2 = ring + ((t - 2) & (RING - 1)) * GRIDC;
                    const T* s3 = ring + ((t - 3) & (RING - 1)) * GRIDC;
                    // neighbours: w (own, t-1), s (VM, t-2), se (VM, t-1), bnw (WM, t-2),
                    // bn (WM, t-1), bc (VMWM, t-3), be (VMWM, t-2)
                    const T nb[7] = {s1[cell], s2[cell - 1], s1[cell - 1], s2[cell - 9],
                                     s1[cell - 9], s3[cell - 10], s2[cell - 10]};
                    T acc = rcur[q];
                    if (STORED) {
#pragma unroll
                        for (int s = 0; s < 7; ++s) acc -= (T)Lcur[q * 7 + s] * nb[s];
                    } else {
                        const T eta = ((T)x - xm) * ihw;
#pragma unroll
                        for (int s = 0; s < 7; ++s) acc -= horner<NC>(coef + s * NC, eta) * nb[s];
                    }
                    val = acc;
                    st_dev(&w[rp + (int64_t)LANES * t], val);
                }
                ring[(t & (RING - 1)) * GRIDC + cell] = val;
                __syncthreads();
            }
            // publish progress: all w stores of this batch have completed
            wait_stores();
            __syncthreads();
            if (lane == 0) st_dev(&progress[b], (int32_t)(min(T0 + H - 1, te) - tb + 1));
#pragma unroll
            for (int q = 0; q < H; ++q) {
                rcur[q] = rnxt[q];
                if (STORED)
#pragma unroll
                    for (int s = 0; s < 7; ++s) Lcur[q * 7 + s] = Lnxt[q * 7 + s];
            }
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------- backward

template <typename T, bool STORED, int H, int NC>
__global__ void __launch_bounds__(64) k_bwd_flow(const TetDev* __restrict__ tets, const BlockDev* __restrict__ blocks,
                                                 const LaneDev* __restrict__ lanes, int nblocks, int64_t S,
                                                 const double* __restrict__ Lb, const T* __restrict__ tab,
                                                 T* __restrict__ w, double* __restrict__ xs,
                                                 const int32_t* __restrict__ order, int32_t* __restrict__ progress,
                                                 int32_t* __restrict__ ticket, int32_t* __restrict__ flags) {
    constexpr int RING = 2 * H >= 8 ? 2 * H : 8;
    __shared__ T ring[RING * GRIDC];
    __shared__ int s_ticket;
    const int lane = threadIdx.x;
    const int vl = lane & 7, wl = lane >> 3;
    const int cell = wl * 9 + vl;  // halo at column 8 and row 8
    for (;;) {
        if (lane == 0) s_ticket = atomicAdd(&ticket[1], 1);
        __syncthreads();
        const int k = s_ticket;
        __syncthreads();
        if (k >= nblocks) return;
        const int b = order[k];
        const BlockDev B = blocks[b];
        const LaneDev& Ln = lanes[(int64_t)b * LANES + lane];
        const bool valid = Ln.v != 0;
        const int n = tets[B.tet].n, v = Ln.v, wrow = Ln.w;
        const int64_t rp = Ln.rp[R_SELF];
        Halo hl;
        if (lane < 8) {
            hl.cell = lane * 9 + 8;
            hl.rp = lanes[(int64_t)b * LANES + lane * 8 + 7].rp[R_VP];
            hl.prod = B.succ[0];
        } else if (lane < 16) {
            hl.cell = 72 + (lane - 8);
            hl.rp = lanes[(int64_t)b * LANES + 56 + (lane - 8)].rp[R_WP];
            hl.prod = B.succ[1];
        } else if (lane == 16) {
            hl.cell = 80;
            hl.rp = lanes[(int64_t)b * LANES + 63].rp[R_VPWP];
            hl.prod = B.succ[2];
        }
        if (hl.prod >= 0) {
            hl.ptb = blocks[hl.prod].tb;
            hl.pte = blocks[hl.prod].te;
        }
        T coef[8 * (NC > 0 ? NC : 1)];
        T xm = 0, ihw = 0;
        if (!STORED && valid) {
            const T* c = tab + ((int64_t)b * LANES + lane) * (2 + 15 * NC);
            xm = c[0];
            ihw = c[1];
            #pragma unroll
            for (int i = 0; i < 8 * NC; ++i) coef[i] = c[2 + 7 * NC + i];
        }
        for (int i = lane; i < RING * GRIDC; i += 64) ring[i] = (T)0;
        __syncthreads();
        const int tb = B.tb, te = B.te;
        // prologue: halo slots te+3 .. te-H+2 (descending; one wait for the furthest slot)
        T hreg[H];
        int known = 0, pending = 0;
        if (hl.cell >= 0) {
            if (hl.prod >= 0) {
                const int smin = max(te - H + 2, hl.ptb);
                if (smin <= hl.pte) wait_progress(progress, hl.prod, hl.pte - smin + 1, known, flags);
            }
            for (int s = te + 3; s >= te - H + 2; --s) {
                const bool ld = hl.prod >= 0 && s >= hl.ptb && s <= hl.pte;
                ring[(s & (RING - 1)) * GRIDC + hl.cell] = ld ? ld_dev(&w[hl.rp + (int64_t)LANES * s]) : (T)0;
            }
        }
        T wcur[H];
        double xcur[H];
        double Lcur[STORED ? H * 8 : 1];
#pragma unroll
        for (int q = 0; q < H; ++q) {
            const int t = te - q;
            wcur[q] = (T)0;
            xcur[q] = 0.0;
            if (valid && t >= tb) {
                wcur[q] = w[rp + (int64_t)LANES * t];
                xcur[q] = xs[rp + (int64_t)LANES * t];
                if (STORED)
#pragma unroll
                    for (int s = 0; s < 8; ++s) Lcur[q * 8 + s] = Lb[(int64_t)s * S + rp + (int64_t)LANES * t];
            }
        }
        __syncthreads();
        for (int T0 = te; T0 >= tb; T0 -= H) {
            if (T0 < te && hl.cell >= 0) {
#pragma unroll
                for (int q = 0; q < H; ++q) ring[((T0 + 1 - q) & (RING - 1)) * GRIDC + hl.cell] = hreg[q];
            }
            if (hl.cell >= 0) {
                const bool more = T0 - H >= tb;
                if (hl.prod >= 0 && more) {
                    known = max(known, pending);
                    const int smin = max(T0 - 2 * H + 2, hl.ptb);
                    if (smin <= hl.pte) wait_progress(progress, hl.prod, hl.pte - smin + 1, known, flags);
                }
#pragma unroll
                for (int q = 0; q < H; ++q) {
                    const int s = T0 - H + 1 - q;
                    const bool ld = more && hl.prod >= 0 && s >= hl.ptb && s <= hl.pte;
                    hreg[q] = ld ? ld_dev(&w[hl.rp + (int64_t)LANES * s]) : (T)0;
                }
                if (hl.prod >= 0 && more) pending = ld_dev(&progress[hl.prod]);
            }
            T wnxt[H];
            double xnxt[H];
            double Lnxt[STORED ? H * 8 : 1];
#pragma unroll
            for (int q = 0; q < H; ++q) {
                const int t = T0 - H - q;
                wnxt[q] = (T)0;
                xnxt[q] = 0.0;
                if (valid && t >= tb) {
                    wnxt[q] = w[rp + (int64_t)LANES * t];
                    xnxt[q] = xs[rp + (int64_t)LANES * t];
                    if (STORED)
#pragma unroll
                        for (int s = 0; s < 8; ++s) Lnxt[q * 8 + s] = Lb[(int64_t)s * S + rp + (int64_t)LANES * t];
                }
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < H; ++q) {
                const int t = T0 - q;
                if (t < tb) break;
                const int x = t - 2 * v - wrow;
                T val = (T)0;
                if (valid && x >= 1 && x <= n - 1 - v) {
                    const T* s1 = ring + ((t + 1) & (RING - 1)) * GRIDC;
                    const T* s2 = ring + ((t + 2) & (RING - 1)) * GRIDC;
                    const T* s3 = ring + ((t + 3) & (RING - 1)) * GRIDC;
                    // upper neighbours p - d: e (own, t+1), n (VP, t+2), nw (VP, t+1),
                    // tse (WP, t+2), ts (WP, t+1), tc (VPWP, t+3), tw (VPWP, t+2)
                    const T nb[7] = {s1[cell], s2[cell + 1], s1[cell + 1], s2[cell + 9],
                                     s1[cell + 9], s3[cell + 10], s2[cell + 10]};
                    T acc;
                    if (STORED) {
                        acc = wcur[q] * (T)Lcur[q * 8];
#pragma unroll
                        for (int s = 0; s < 7; ++s) acc -= (T)Lcur[q * 8 + 1 + s] * nb[s];
                    } else {
                        const T eta = ((T)x - xm) * ihw;
                        acc = wcur[q] * horner<NC>(coef, eta);
#pragma unroll
                        for (int s = 0; s < 7; ++s) acc -= horner<NC>(coef + (1 + s) * NC, eta) * nb[s];
                    }
                    val = acc;
                    const int64_t idx = rp + (int64_t)LANES * t;
                    st_dev(&w[idx], val);
                    xs[idx] = xcur[q] + (double)val;
                }
                ring[(t & (RING - 1)) * GRIDC + cell] = val;
                __syncthreads();
            }
            wait_stores();
            __syncthreads();
            if (lane == 0) st_dev(&progress[b], (int32_t)(te - max(T0 - H + 1, tb) + 1));
#pragma unroll
            for (int q = 0; q < H; ++q) {
                wcur[q] = wnxt[q];
                xcur[q] = xnxt[q];
                if (STORED)
#pragma unroll
                    for (int s = 0; s < 8; ++s) Lcur[q * 8 + s] = Lnxt[q * 8 + s];
            }
        }
        __syncthreads();
    }
}

__global__ void k_flow_reset(int32_t* __restrict__ progress, int n, int32_t* __restrict__ ticket) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) progress[i] = 0;
    if (i < 2) ticket[i] = 0;
}

// ------------------------------------------------------------------ launchers

constexpr int H_F64 = 4;   // stored factors: 8 operands per step are prefetched
constexpr int H_S64 = 8;   // FP64 surrogate
constexpr int H_F32 = 16;  // FP32 surrogate

template <int NC>
struct FlowK {
    static const void* fwd(int variant) {
        if (variant == 1) return (const void*)k_fwd_flow<double, false, H_S64, NC>;
        return (const void*)k_fwd_flow<float, false, H_F32, NC>;
    }
    static const void* bwd(int variant) {
        if (variant == 1) return (const void*)k_bwd_flow<double, false, H_S64, NC>;
        return (const void*)k_bwd_flow<float, false, H_F32, NC>;
    }
    static void run_fwd(const Ctx& c, const Flow& f, int variant, hipStream_t st) {
        if (variant == 1)
            k_fwd_flow<double, false, H_S64, NC><<<f.grid, 64, 0, st>>>(
                c.tets, c.blocks, c.lanes, c.nblocks, c.S, nullptr, c.tab64, (const double*)c.r, (double*)c.w,
                f.order_fwd, f.progress, f.ticket, f.flags);
        else
            k_fwd_flow<float, false, H_F32, NC><<<f.grid, 64, 0, st>>>(
                c.tets, c.blocks, c.lanes, c.nblocks, c.S, nullptr, c.tab32, (const float*)c.r, (float*)c.w,
                f.order_fwd, f.progress, f.ticket, f.flags);
    }
    static void run_bwd(const Ctx& c, const Flow& f, int variant, double* x, hipStream_t st) {
        if (variant == 1)
            k_bwd_flow<double, false, H_S64, NC><<<f.grid, 64, 0, st>>>(c.tets, c.blocks, c.lanes, c.nblocks, c.S,
                                                                        nullptr, c.tab64, (double*)c.w, x,
                                                                        f.order_bwd, f.progress, f.ticket, f.flags);
        else
            k_bwd_flow<float, false, H_F32, NC><<<f.grid, 64, 0, st>>>(c.tets, c.blocks, c.lanes, c.nblocks, c.S,
                                                                       nullptr, c.tab32, (float*)c.w, x, f.order_bwd,
                                                                       f.progress, f.ticket, f.flags);
    }
};

#define ILU_NC_DISPATCH(NCV, EXPR)      \
    switch (NCV) {                      \
    case 1: { constexpr int N_ = 1; EXPR; } break; \
    case 2: { constexpr int N_ = 2; EXPR; } break; \
    case 3: { constexpr int N_ = 3; EXPR; } break; \
    case 4: { constexpr int N_ = 4; EXPR; } break; \
    case 5: { constexpr int N_ = 5; EXPR; } break; \
    case 6: { constexpr int N_ = 6; EXPR; } break; \
    default: { constexpr int N_ = 7; EXPR; } break; \
    }

int flow_max_resident(int variant, int NC) {
    int dev = 0;
    hipGetDevice(&dev);
    int cus = 0;
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const void* kf = nullptr;
    const void* kb = nullptr;
    if (variant == 0) {
        kf = (const void*)k_fwd_flow<double, true, H_F64, 0>;
        kb = (const void*)k_bwd_flow<double, true, H_F64, 0>;
    } else {
        ILU_NC_DISPATCH(NC, (kf = FlowK<N_>::fwd(variant), kb = FlowK<N_>::bwd(variant)));
    }
    int a = 0, b = 0;
    hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, kf, 64, 0);
    hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, kb, 64, 0);
    int per_cu = a < b ? a : b;
    if (per_cu < 1) per_cu = 1;
    return per_cu * cus;
}

void launch_flow_reset(const Ctx& c, const Flow& f, hipStream_t st) {
    const int n = c.nblocks > 2 ? c.nblocks : 2;
    k_flow_reset<<<(n + 255) / 256, 256, 0, st>>>(f.progress, c.nblocks, f.ticket);
}

void launch_fwd_flow(const Ctx& c, const Flow& f, int variant, hipStream_t st) {
    if (variant == 0)
        k_fwd_flow<double, true, H_F64, 0><<<f.grid, 64, 0, st>>>(c.tets, c.blocks, c.lanes, c.nblocks, c.S, c.Lf,
                                                                   nullptr, (const double*)c.r, (double*)c.w,
                                                                   f.order_fwd, f.progress, f.ticket, f.flags);
    else
        ILU_NC_DISPATCH(c.NC, FlowK<N_>::run_fwd(c, f, variant, st));
}

void launch_bwd_flow(const Ctx& c, const Flow& f, int variant, double* x, hipStream_t st) {
    if (variant == 0)
        k_bwd_flow<double, true, H_F64, 0><<<f.grid, 64, 0, st>>>(c.tets, c.blocks, c.lanes, c.nblocks, c.S, c.Lb,
                                                                   nullptr, (double*)c.w, x, f.order_bwd, f.progress,
                                                                   f.ticket, f.flags);
    else
        ILU_NC_DISPATCH(c.NC, FlowK<N_>::run_bwd(c, f, variant, x, st));
}

}  // namespace ilu
