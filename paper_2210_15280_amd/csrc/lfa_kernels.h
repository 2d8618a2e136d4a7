// Launchers of the LFA orientation kernels (Sec. 3.1, strategy on macro-elements).
#pragma once

#include <hip/hip_runtime.h>

namespace ilu {

constexpr int LFA_PERMS = 24;       // vertex permutations of a tetrahedron
constexpr int LFA_REC = 24;         // per (tet, permutation): A[15], L[7], D, converged
constexpr int LFA_MAX_ITERS = 20000;

// verts: device, tetrahedron i's vertices [4][3] at verts + i * vstride
// (doubles); rec: device [ntets * 24][LFA_REC]
void launch_lfa_stencils(const double* verts, int64_t vstride, int ntets, double* rec, hipStream_t st);
// mu: device [ntets * 24]; samples frequencies per direction
void launch_lfa_symbols(const double* rec, int ntets, int samples, double* mu, hipStream_t st);
// best: device [ntets], per tetrahedron the first k with the smallest mu
void launch_lfa_best(const double* mu, int ntets, int32_t* best, hipStream_t st);

}  // namespace ilu
