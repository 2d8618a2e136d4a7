// Stencil row of one lattice point of a refined macro-tetrahedron (Sec. 2.1),
// shared by the assembly kernel and the LFA kernel.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels_common.h"

namespace ilu {

// Slot in the 15-point stencil (listing order w,s,se,bnw,bn,bc,be,c,e,n,nw,tse,ts,tc,tw)
// of a lattice offset with components in {-1,0,1}; -1 if it is not a stencil offset.
__host__ __device__ constexpr int stencil_slot(int dx, int dy, int dz) {
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

// The 24 micro-tetrahedra around a lattice point P.  The micro-mesh is the
// Kuhn subdivision in (a,b,c) = (x, x+y, x+y+z): the simplices of the cell
// with corner q are q + {0, e_s1, e_s1+e_s2, (1,1,1)} for the six orders
// (s1, s2, s3) of the axes, and P is one of the four vertices (index k).
// Micro-tetrahedron sg * 4 + k: its logical (x,y,z) edge vectors l_j - l_0
// (j = 1..3), four times its centroid minus P, the index k of P and the
// stencil slot of l_j - l_k for j = 0..3.  Only these integers depend on the
// micro-tetrahedron; everything else follows from the macro map.
struct MicroTet {
    int d[3][3];
    int c4[3];
    int k;
    int slot[4];
};

__host__ __device__ constexpr MicroTet micro_tet(int sg, int k) {
    const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int off[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {1, 1, 1}};
    off[1][perm[sg][0]] = 1;
    off[2][perm[sg][0]] = 1;
    off[2][perm[sg][1]] = 1;
    // logical offsets of the vertices from P: (da, db - da, dc - db)
    int l[4][3] = {};
    for (int j = 0; j < 4; ++j) {
        const int da = off[j][0] - off[k][0], db = off[j][1] - off[k][1], dc = off[j][2] - off[k][2];
        l[j][0] = da;
        l[j][1] = db - da;
        l[j][2] = dc - db;
    }
    MicroTet m{};
    for (int j = 1; j < 4; ++j)
        for (int r = 0; r < 3; ++r) m.d[j - 1][r] = l[j][r] - l[0][r];
    for (int r = 0; r < 3; ++r) m.c4[r] = l[0][r] + l[1][r] + l[2][r] + l[3][r];
    m.k = k;
    for (int j = 0; j < 4; ++j) m.slot[j] = stencil_slot(l[j][0] - l[k][0], l[j][1] - l[k][1], l[j][2] - l[k][2]);
    return m;
}

#define ILU_MICRO_ROW(sg) micro_tet(sg, 0), micro_tet(sg, 1), micro_tet(sg, 2), micro_tet(sg, 3)
__constant__ constexpr MicroTet kMicroTets[24] = {ILU_MICRO_ROW(0), ILU_MICRO_ROW(1), ILU_MICRO_ROW(2),
                                                  ILU_MICRO_ROW(3), ILU_MICRO_ROW(4), ILU_MICRO_ROW(5)};
#undef ILU_MICRO_ROW

// Ad[slot_j] += kij[j] for micro-tetrahedron Q, with the slots as constants
// (a runtime index would put Ad in scratch memory).
template <int Q>
__device__ __forceinline__ void add_micro_row(double (&Ad)[15], const double (&kij)[4]) {
    constexpr MicroTet m = micro_tet(Q / 4, Q % 4);
    Ad[m.slot[0]] += kij[0];
    Ad[m.slot[1]] += kij[1];
    Ad[m.slot[2]] += kij[2];
    Ad[m.slot[3]] += kij[3];
}

// Ad[15] = stencil row of lattice point (x,y,z) for the macro map
// X = v0 + J (x,y,z) / n (invn = 1/n) and the coefficient kappa(X) taken at
// micro-tet centroids: the sum over the 24 micro-tetrahedra around the point
// of their P1 element stiffness rows (in the order sg, then k, then j).  No
// boundary test: every neighbour is counted.
template <typename Kappa>
__device__ __forceinline__ void stencil_row(const double* J, const double* v0, double invn, int x, int y, int z,
                                            Kappa kappa, double (&Ad)[15]) {
#pragma unroll
    for (int s = 0; s < 15; ++s) Ad[s] = 0.0;
#pragma unroll 1
    for (int q = 0; q < 24; ++q) {
        const MicroTet& m = kMicroTets[q];
        // physical edge matrix E (columns X_j - X_0) = J (l_j - l_0) / n
        double E[3][3], cen[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
                E[r][cc] = (J[3 * r] * m.d[cc][0] + J[3 * r + 1] * m.d[cc][1] + J[3 * r + 2] * m.d[cc][2]) * invn;
            const double mx = 0.25 * (4 * x + m.c4[0]), my = 0.25 * (4 * y + m.c4[1]), mz = 0.25 * (4 * z + m.c4[2]);
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
#pragma unroll
        for (int r = 0; r < 3; ++r) g[0][r] = -(g[1][r] + g[2][r] + g[3][r]);
        const double scale = kappa(cen[0], cen[1], cen[2]) * fabs(det) / 6.0;
        // the vertex of P (uniform over the wavefront: a select, not an index)
        double gk[3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
            gk[r] = m.k == 0 ? g[0][r] : m.k == 1 ? g[1][r] : m.k == 2 ? g[2][r] : g[3][r];
        double kij[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) kij[j] = scale * (gk[0] * g[j][0] + gk[1] * g[j][1] + gk[2] * g[j][2]);
        switch (q) {
#define ILU_MICRO_CASE(Q) \
    case Q: add_micro_row<Q>(Ad, kij); break;
            ILU_MICRO_CASE(0) ILU_MICRO_CASE(1) ILU_MICRO_CASE(2) ILU_MICRO_CASE(3) ILU_MICRO_CASE(4)
            ILU_MICRO_CASE(5) ILU_MICRO_CASE(6) ILU_MICRO_CASE(7) ILU_MICRO_CASE(8) ILU_MICRO_CASE(9)
            ILU_MICRO_CASE(10) ILU_MICRO_CASE(11) ILU_MICRO_CASE(12) ILU_MICRO_CASE(13) ILU_MICRO_CASE(14)
            ILU_MICRO_CASE(15) ILU_MICRO_CASE(16) ILU_MICRO_CASE(17) ILU_MICRO_CASE(18) ILU_MICRO_CASE(19)
            ILU_MICRO_CASE(20) ILU_MICRO_CASE(21) ILU_MICRO_CASE(22) ILU_MICRO_CASE(23)
#undef ILU_MICRO_CASE
        }
    }
}

}  // namespace ilu
