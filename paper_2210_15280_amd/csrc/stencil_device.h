// Stencil row of one lattice point of a refined macro-tetrahedron (Sec. 2.1),
// shared by the assembly kernel and the LFA kernel.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels_common.h"

namespace ilu {

// Slot in the 15-point stencil (listing order w,s,se,bnw,bn,bc,be,c,e,n,nw,tse,ts,tc,tw)
// of a lattice offset with components in {-1,0,1}; -1 if it is not a stencil offset.
__device__ inline int stencil_slot(int dx, int dy, int dz) {
    if (dz == -1) {
        if (dy == 0 && dx == 0) return 5;    // bc
        if (dy == 0 && dx == 1) return 6;    // be
        if (dy == 1 && dx == -1) return 3;   // bnw
        if (dy == 1 && dx == 0) return 4;    // bn
        return -1;
    }
    if (dz == 0) {
        if (dy == -1 && dx == 0) return 1;   // s
        if (dy == -1 && dx == 1) return 2;   // se
        if (dy == 0 && dx == -1) return 0;   // w
        if (dy == 0 && dx == 0) return 7;    // c
        if (dy == 0 && dx == 1) return 8;    // e
        if (dy == 1 && dx == 0) return 9;    // n
        if (dy == 1 && dx == -1) return 10;  // nw
        return -1;
    }
    if (dy == -1 && dx == 1) return 11;      // tse
    if (dy == -1 && dx == 0) return 12;      // ts
    if (dy == 0 && dx == 0) return 13;       // tc
    if (dy == 0 && dx == -1) return 14;      // tw
    return -1;
}

// Ad[15] = stencil row of lattice point (x,y,z) for the macro map
// X = v0 + J (x,y,z) / n (invn = 1/n) and the coefficient kappa(X) taken at
// micro-tet centroids: the sum over the 24 micro-tetrahedra around the point
// of their P1 element stiffness rows.  The micro-mesh is the Kuhn subdivision
// in (a,b,c) = (x, x+y, x+y+z): the simplices containing P are
// q + {0, e_s1, e_s1+e_s2, (1,1,1)} with P one of the four vertices.  No
// boundary test: every neighbour is counted.
template <typename Kappa>
__device__ __forceinline__ void stencil_row(const double* J, const double* v0, double invn, int x, int y, int z,
                                            Kappa kappa, double Ad[15]) {
    constexpr int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int s = 0; s < 15; ++s) Ad[s] = 0.0;
    const int P[3] = {x, x + y, x + y + z};
    for (int sg = 0; sg < 6; ++sg) {
        int off[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {1, 1, 1}};
        off[1][perm[sg][0]] = 1;
        off[2][perm[sg][0]] = 1;
        off[2][perm[sg][1]] = 1;
        for (int k = 0; k < 4; ++k) {
            // vertices (logical xyz) of the simplex whose k-th vertex is p
            int lx[4], ly[4], lz[4];
            for (int j = 0; j < 4; ++j) {
                const int a = P[0] - off[k][0] + off[j][0];
                const int bb = P[1] - off[k][1] + off[j][1];
                const int c = P[2] - off[k][2] + off[j][2];
                lx[j] = a;
                ly[j] = bb - a;
                lz[j] = c - bb;
            }
            // physical edge matrix E (columns X_j - X_0) = J (l_j - l_0) / n
            double E[3][3], cen[3];
            for (int r = 0; r < 3; ++r) {
                for (int cc = 0; cc < 3; ++cc) {
                    const int ex = lx[cc + 1] - lx[0], ey = ly[cc + 1] - ly[0], ez = lz[cc + 1] - lz[0];
                    E[r][cc] = (J[3 * r] * ex + J[3 * r + 1] * ey + J[3 * r + 2] * ez) * invn;
                }
                const double mx = 0.25 * (lx[0] + lx[1] + lx[2] + lx[3]);
                const double my = 0.25 * (ly[0] + ly[1] + ly[2] + ly[3]);
                const double mz = 0.25 * (lz[0] + lz[1] + lz[2] + lz[3]);
                cen[r] = v0[r] + (J[3 * r] * mx + J[3 * r + 1] * my + J[3 * r + 2] * mz) * invn;
            }
            const double c00 = E[1][1] * E[2][2] - E[1][2] * E[2][1];
            const double c01 = E[1][2] * E[2][0] - E[1][0] * E[2][2];
            const double c02 = E[1][0] * E[2][1] - E[1][1] * E[2][0];
            const double det = E[0][0] * c00 + E[0][1] * c01 + E[0][2] * c02;
            const double id = 1.0 / det;
            // rows of E^{-1} are the gradients of lambda_1..3
            double g[4][3];
            g[1][0] = c00 * id;
            g[1][1] = (E[0][2] * E[2][1] - E[0][1] * E[2][2]) * id;
            g[1][2] = (E[0][1] * E[1][2] - E[0][2] * E[1][1]) * id;
            g[2][0] = c01 * id;
            g[2][1] = (E[0][0] * E[2][2] - E[0][2] * E[2][0]) * id;
            g[2][2] = (E[0][2] * E[1][0] - E[0][0] * E[1][2]) * id;
            g[3][0] = c02 * id;
            g[3][1] = (E[0][1] * E[2][0] - E[0][0] * E[2][1]) * id;
            g[3][2] = (E[0][0] * E[1][1] - E[0][1] * E[1][0]) * id;
            for (int r = 0; r < 3; ++r) g[0][r] = -(g[1][r] + g[2][r] + g[3][r]);
            const double scale = kappa(cen[0], cen[1], cen[2]) * fabs(det) / 6.0;
            for (int j = 0; j < 4; ++j) {
                const double kij = scale * (g[k][0] * g[j][0] + g[k][1] * g[j][1] + g[k][2] * g[j][2]);
                const int sl = stencil_slot(lx[j] - lx[k], ly[j] - ly[k], lz[j] - lz[k]);
                Ad[sl] += kij;
            }
        }
    }
}

}  // namespace ilu
