// Launch context shared by the host code and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ilu_internal.h"

namespace ilu {

constexpr int RES_T = 64;  // hyperplanes per workgroup in the point-parallel kernels

struct Ctx {
    const TetDev* tets = nullptr;
    const BlockDev* blocks = nullptr;
    const LaneDev* lanes = nullptr;
    int nblocks = 0;
    int bv = 8, bw = 8;      // block shape in rows
    int lpb = 64;            // lanes per block = bv * bw
    int groups = 1;          // 64-lane groups per block
    int res_chunks = 0;      // ceil(max block window / RES_T)
    int res_bands = 0;       // ceil((last hyperplane + 1) / RES_T): absolute hyperplane bands
    int64_t S = 0;           // stream length (elements)
    bool res_lds = true;     // exact-operator residual with LDS staging (8x8 and 16x16 blocks)
    int res_lds_t = RES_T;   // hyperplanes per workgroup of that residual run on its own (RES_T or 2 RES_T)
    const double* A8 = nullptr;   // [8][S]: centre, then lower weights w..be
    const double* Lf = nullptr;   // [7][S] stored forward weights
    const double* Lb = nullptr;   // [8][S] stored backward weights (1/D, L^{p-d}_d)
    const double* tab64 = nullptr;
    const float* tab32 = nullptr;
    int NC = 0;                   // dg_x + 1
    void* r = nullptr;            // residual stream (FP64, or FP32 for the mixed variant)
    void* w = nullptr;            // substitution stream (same type as r)
    // surrogate operator (null: the residual uses the assembled A8): per-row
    // records [xm, 1/hw, lower 7*NC, centre NC, upper 7*NC], FP32 for the mixed variant
    const double* tabA64 = nullptr;
    const float* tabA32 = nullptr;
    // variant V1 (null otherwise), FP32 for the mixed variant; 8-value records,
    // one per set point (one 32 B / 64 B read per point):
    //   v1f: [L_0..L_6, 1/D], the exact factors of the points of set F
    //        (boundary points), v1f_stride records;
    //   v1b: [1/D, L^{p-d}_d for d in D_l], the backward weights of the points of
    //        set B (exact where the point holding the factor is in F, the
    //        surrogate elsewhere, 0 outside), v1b_stride records.
    // The last record is 0: points outside the sets read it.
    const void* v1f = nullptr;
    const void* v1b = nullptr;
    int64_t v1f_stride = 0, v1b_stride = 0;
};

}  // namespace ilu
