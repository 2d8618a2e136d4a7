// Launchers of the vector kernels behind preconditioned CG and the
// contraction-factor measurement.  All of them touch only the active points of
// stream-layout vectors (padding and the zero region are never written) and
// write one partial sum per work item where they reduce.
#pragma once

#include "ctx.h"

namespace ilu {

// Scalar slots of the CG state vector (device FP64 array of CG_NSLOT).
enum CgSlot {
    CG_RZ = 0,     // r.z of the current iterate
    CG_PQ = 1,     // p.q (reduction target)
    CG_RR = 2,     // r.r (reduction target)
    CG_RZNEW = 3,  // r.z after the preconditioner (reduction target)
    CG_ALPHA = 4,
    CG_BETA = 5,
    CG_DONE = 6,   // 1 once the tolerance is met (or on breakdown): later steps change nothing
    CG_ITERS = 7,  // completed iterations
    CG_TOL2 = 8,   // squared residual threshold
    CG_BB = 9,     // b.b (reduction target)
    CG_BREAK = 10, // 1 if p.q <= 0 or r.z <= 0 (C or A not positive definite)
    CG_NSLOT = 16
};

// Scalar steps (one thread).
enum CgStep {
    CG_SETUP = 0,  // TOL2 = max(rel^2 BB, abs^2); ALPHA = BETA = DONE = ITERS = BREAK = 0
    CG_INIT = 1,   // RZ = RZNEW; DONE if RR <= TOL2
    CG_STEP_ALPHA = 2,
    CG_CHECK = 3,  // after the update: ITERS += 1, DONE if RR <= TOL2
    CG_STEP_BETA = 4
};

// partial[item] = sum of a .* b over the item's active points
void launch_dot(const Ctx& c, const double* a, const double* b, double* partial, hipStream_t st);
// v *= 1 / sqrt(sc[slot]) on the active points
void launch_scale_rsqrt(const Ctx& c, double* v, const double* sc, int slot, hipStream_t st);
// x += alpha p, r -= alpha q (unless done); rs = r in the sweep precision; z = 0;
// partial = r.r
void launch_cg_update(const Ctx& c, bool f32, double* x, const double* p, double* r, const double* q, double* z,
                      void* rs, const double* sc, double* partial, hipStream_t st);
// p = z + beta p (p = z when beta = 0), unless done
void launch_cg_direction(const Ctx& c, double* p, const double* z, const double* sc, hipStream_t st);
void launch_cg_scalar(double* sc, int step, double rel_tol, double abs_tol, hipStream_t st);

// Stored factors of the symmetric Gauss-Seidel preconditioner
// C = (D_A + L_A) D_A^{-1} (D_A + L_A)^T in the unit-lower form L D L^T:
// L^p_d = A^p_d / A^{p+d}_c, D^p = A^p_c (same layout as the ILU factors).
void launch_sgs_factors(const Ctx& c, double* Lf, double* Df, int* flags, hipStream_t st);

}  // namespace ilu
