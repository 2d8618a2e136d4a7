// Tagged device-coherent values shared between concurrently running kernels
// and workgroups, and the residual of a single point.
//
// A tagged entry packs a 32-bit payload and a 32-bit launch tag into each
// 64-bit word (FP64 values take two words, one per half), written and read
// with device-scope relaxed atomics.  A reader knows a value is the current
// launch's when every word carries that launch's tag, so producer and
// consumer need no flag and no fence between them.  Used by the dataflow
// exchange buffer (boundary values of neighbouring blocks) and by the tagged
// residual stream that the forward sweep consumes while the residual kernel is
// still running.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels_common.h"

namespace ilu {

template <typename T>
__device__ __forceinline__ void st_dev(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_dev(const T* p) {
    return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
struct XEnt;
template <>
struct XEnt<float> {
    static constexpr int W = 1;
    uint64_t u[1];
};
template <>
struct XEnt<double> {
    static constexpr int W = 2;
    uint64_t u[2];
};

__device__ __forceinline__ void x_put(uint64_t* p, float v, uint32_t tag) {
    st_dev(p, ((uint64_t)tag << 32) | (uint64_t)__float_as_uint(v));
}
__device__ __forceinline__ void x_put(uint64_t* p, double v, uint32_t tag) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    st_dev(p, ((uint64_t)tag << 32) | (b & (uint64_t)0xffffffffu));
    st_dev(p + 1, ((uint64_t)tag << 32) | (b >> 32));
}
template <typename T>
__device__ __forceinline__ void x_get(XEnt<T>& e, const uint64_t* p) {
#pragma unroll
    for (int k = 0; k < XEnt<T>::W; ++k) e.u[k] = ld_dev(p + k);
}
template <typename T>
__device__ __forceinline__ bool x_ok(const XEnt<T>& e, uint32_t tag) {
    bool ok = true;
#pragma unroll
    for (int k = 0; k < XEnt<T>::W; ++k) ok = ok && (uint32_t)(e.u[k] >> 32) == tag;
    return ok;
}
__device__ __forceinline__ float x_val(const XEnt<float>& e) { return __uint_as_float((uint32_t)e.u[0]); }
__device__ __forceinline__ double x_val(const XEnt<double>& e) {
    return __longlong_as_double((long long)((e.u[0] & (uint64_t)0xffffffffu) | (e.u[1] << 32)));
}

// r^p = b^p - sum_{d in D} A^p_d x^{p+d} of the point at hyperplane t of lane
// Ln (Alg. 2, first loop), one term at a time: the centre, then for each
// lower direction d_s the pair (A^p_{d_s} x^{p+d_s}, A^{p-d_s}_{d_s} x^{p-d_s})
// -- the upper weight of p is the lower weight of p - d_s.  The residual
// kernel adds the same products in the same order with the same fused
// multiply-adds, so both give bitwise the same value.
__device__ inline double residual_point(const LaneDev& Ln, int lpb, int64_t S, int t, const double* __restrict__ A8,
                                        const double* __restrict__ x, const double* __restrict__ b) {
    const int64_t off = (int64_t)lpb * t;
    const int64_t idx = Ln.rp[R_SELF] + off;
    double acc = A8[idx] * x[idx];
#pragma unroll 1  // few registers: this is the forward sweep's rare path
    for (int s = 0; s < NLOW; ++s) {
        const int64_t ql = Ln.rp[low_row(s)] + (int64_t)lpb * low_dt(s) + off;
        const int64_t qu = Ln.rp[up_row(s)] + (int64_t)lpb * up_dt(s) + off;
        acc = fma(A8[(int64_t)(1 + s) * S + idx], x[ql], acc);
        acc = fma(A8[(int64_t)(1 + s) * S + qu], x[qu], acc);
    }
    return b[idx] - acc;
}

}  // namespace ilu
