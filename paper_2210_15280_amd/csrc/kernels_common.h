// Device helpers shared by the libilu kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ilu_internal.h"

namespace ilu {

// Lower stencil directions of D_l in the paper's listing order
// (w, s, se, bnw, bn, bc, be), as lattice offsets (dx, dy, dz).
__host__ __device__ constexpr int low_dx(int s) { return s == 0 ? -1 : s == 2 ? 1 : s == 3 ? -1 : s == 6 ? 1 : 0; }
__host__ __device__ constexpr int low_dy(int s) { return s == 1 ? -1 : s == 2 ? -1 : s == 3 ? 1 : s == 4 ? 1 : 0; }
__host__ __device__ constexpr int low_dz(int s) { return (s == 3 || s == 4 || s == 5 || s == 6) ? -1 : 0; }
// Row slot holding p + d_s and hyperplane shift of p + d_s (du+dv+dw).
__host__ __device__ constexpr int low_row(int s) {
    return s == 0 ? R_SELF : (s == 1 || s == 2) ? R_VM : (s == 3 || s == 4) ? R_WM : R_VMWM;
}
__host__ __device__ constexpr int low_dt(int s) { return low_dx(s) + 2 * low_dy(s) + 3 * low_dz(s); }
// p - d_s (the upper neighbour e = -d_s): row slot and hyperplane shift.
__host__ __device__ constexpr int up_row(int s) {
    return s == 0 ? R_SELF : (s == 1 || s == 2) ? R_VP : (s == 3 || s == 4) ? R_WP : R_VPWP;
}
__host__ __device__ constexpr int up_dt(int s) { return -low_dt(s); }

// Point-parallel kernels launch (blocks x 64-lane groups) workgroups: decode
// the block and the lane of this thread (the single place this mapping lives).
__device__ __forceinline__ void decode_group(int groups, int& b, int& lane) {
    b = (int)blockIdx.x / groups;
    lane = (int)(blockIdx.x % groups) * WAVE + (int)(threadIdx.x & (WAVE - 1));
}

// Point-parallel work items of the residual, norm and vector kernels: workgroup
// (x, y) runs lanes [64 (x % groups), +64) of block x / groups over the y-th
// chunk of RES_T hyperplanes, so the grid sweeps one band of hyperplanes of
// every block at a time.  (Remapping the items so that each XCD gets a
// contiguous range of blocks measured 10-20% slower.)
struct Item {
    int blk, chunk, lane;
    int64_t id;
    bool live;
};
__device__ __forceinline__ Item res_item(int groups, int nblocks) {
    Item it;
    decode_group(groups, it.blk, it.lane);
    it.chunk = (int)blockIdx.y;
    it.live = it.blk < nblocks;
    it.id = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    return it;
}

__device__ __forceinline__ bool interior(int n, int x, int y, int z) {
    return x >= 1 && y >= 1 && z >= 1 && x + y + z <= n - 1;
}

// Interior lexicographic index (z slowest, then y, then x) of an interior point:
// layers z' < z hold C(n-1,3) - C(n-z,3) points, rows y' < y of layer z hold
// (y-1) m - (y-1) y / 2 points with m = n - 1 - z.
__host__ __device__ __forceinline__ int64_t choose3(int64_t k) { return k < 3 ? 0 : k * (k - 1) * (k - 2) / 6; }
__host__ __device__ __forceinline__ int64_t lex_index(int n, int x, int y, int z) {
    int64_t m = n - 1 - z;
    return choose3(n - 1) - choose3(n - z) + (int64_t)(y - 1) * m - (int64_t)(y - 1) * y / 2 + (x - 1);
}

// Workgroup barrier that orders LDS traffic only: a full __syncthreads()
// would also wait for this wave's outstanding global stores and loads.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Shifted Legendre values P_0..P_deg at s = 2 xhat - 1.
__device__ __forceinline__ void legendre(double s, int deg, double* P) {
    P[0] = 1.0;
    if (deg >= 1) P[1] = s;
    for (int k = 1; k < deg; ++k) P[k + 1] = ((2 * k + 1) * s * P[k] - k * P[k - 1]) / (k + 1);
}

}  // namespace ilu
