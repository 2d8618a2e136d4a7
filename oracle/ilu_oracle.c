/*
 * ilu_oracle.c -- plain, slow, CPU FP64 reference for the matrix-free ILU(0)
 * smoother of Drzisga, Wagner, Wohlmuth, "A matrix-free ILU realization based
 * on surrogates" (arXiv:2210.15280).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or constant with the
 * HIP library.  Build: gcc -O2 -ffp-contract=off -fPIC -shared.
 *
 * Contents (paper section in brackets):
 *   lattice / DOF numbering            [Sec. 2.1, logical grid coordinates and
 *                                       the lexicographic ordering]
 *   micro-mesh, P1 element stiffness,  [Sec. 2.1, bilinear form a(u,v) and the
 *   assembly of R_t A R_t^T,            stencil notation A^p_d]
 *   stencil rows of single points
 *   ILU(0), definition (IKJ on CSR)    [Sec. 3, (L D L^T)_ij = A_ij on S_A]
 *   ILU(0), stencil recurrences        [Sec. 3, eq. (matrix-equations); Alg. 1]
 *   smoothing step, matrix form        [Sec. 2.1 Richardson smoother with
 *                                       C_t,sym = L_t D_t L_t^T]
 *   smoothing step, stencil form       [Alg. 2, variant V2]
 *   mixed-precision smoothing step     [FP64 residual, FP32 sweeps]
 *
 * Readings of points the paper leaves open (the same list is in the design
 * notes): micro vertex X(x,y,z) = v1 + (x d1 + y d2 + z d3)/2^L; the micro-mesh
 * is the Freudenthal-Kuhn subdivision whose edge set is the stencil direction
 * set D minus c; variable coefficients use the one-point centroid rule;
 * entries A^p_d with p+d on the macro boundary are dropped (homogeneous
 * Dirichlet, restriction R_t); the sparsity pattern is the structural
 * 15-point pattern.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Stencil directions in the paper's listing order (Sec. 2.1):
 * D = {w, s, se, bnw, bn, bc, be, c, e, n, nw, tse, ts, tc, tw};
 * the first seven form the lower set D_l, index 7 is the centre c and
 * index 8+k is the negative of lower direction k. */
static const int DIR[15][3] = {
    {-1, 0, 0}, {0, -1, 0}, {1, -1, 0}, {-1, 1, -1}, {0, 1, -1}, {0, 0, -1}, {1, 0, -1},
    {0, 0, 0},
    {1, 0, 0}, {0, 1, 0}, {-1, 1, 0}, {1, -1, 1}, {0, -1, 1}, {0, 0, 1}, {-1, 0, 1}};
enum { NDIR = 15, NLOW = 7, CENTRE = 7 };

static int slot_of(int dx, int dy, int dz) {
    for (int s = 0; s < NDIR; ++s)
        if (DIR[s][0] == dx && DIR[s][1] == dy && DIR[s][2] == dz) return s;
    return -1;
}

static int lower_slot_of(int dx, int dy, int dz) {
    int s = slot_of(dx, dy, dz);
    return (s >= 0 && s < NLOW) ? s : -1;
}

/* ---------------------------------------------------------------- lattice */

/* Interior points: x,y,z >= 1 and x+y+z <= n-1 with n = 2^L (Sec. 2.1).
 * Lexicographic order: z slowest, then y, then x. */
int64_t oracle_num_interior(int level) {
    int64_t n = (int64_t)1 << level;
    return (n - 1) * (n - 2) * (n - 3) / 6;
}

static int64_t layer_offset(int64_t n, int64_t z) {
    /* number of interior points with z' < z: layer z' holds m(m-1)/2 points,
     * m = n-1-z' */
    int64_t off = 0;
    for (int64_t zz = 1; zz < z; ++zz) {
        int64_t m = n - 1 - zz;
        off += m * (m - 1) / 2;
    }
    return off;
}

typedef struct {
    int64_t n;
    int64_t *zoff; /* zoff[z] = index of the first interior point of layer z */
} lattice_t;

static int lattice_init(lattice_t *lt, int level) {
    lt->n = (int64_t)1 << level;
    lt->zoff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(lt->n + 1));
    if (!lt->zoff) return -1;
    for (int64_t z = 0; z <= lt->n; ++z) lt->zoff[z] = z >= 1 ? layer_offset(lt->n, z) : 0;
    return 0;
}

static void lattice_free(lattice_t *lt) { free(lt->zoff); }

static int is_interior(int64_t n, int64_t x, int64_t y, int64_t z) {
    return x >= 1 && y >= 1 && z >= 1 && x + y + z <= n - 1;
}

static int64_t interior_index(const lattice_t *lt, int64_t x, int64_t y, int64_t z) {
    if (!is_interior(lt->n, x, y, z)) return -1;
    int64_t m = lt->n - 1 - z;
    return lt->zoff[z] + (y - 1) * m - (y - 1) * y / 2 + (x - 1);
}

/* Coordinates of all interior points in lexicographic order, xyz[3*i+k]. */
int oracle_interior_points(int level, int32_t *xyz) {
    int64_t n = (int64_t)1 << level, i = 0;
    for (int64_t z = 1; z <= n - 3; ++z)
        for (int64_t y = 1; y <= n - 2 - z; ++y)
            for (int64_t x = 1; x <= n - 1 - z - y; ++x) {
                xyz[3 * i] = (int32_t)x;
                xyz[3 * i + 1] = (int32_t)y;
                xyz[3 * i + 2] = (int32_t)z;
                ++i;
            }
    return 0;
}

/* Interior index of every (x,y,z) given as triples, -1 if not interior. */
int oracle_index_of(int level, int64_t count, const int32_t *xyz, int64_t *out) {
    lattice_t lt;
    if (lattice_init(&lt, level)) return -1;
    for (int64_t i = 0; i < count; ++i)
        out[i] = interior_index(&lt, xyz[3 * i], xyz[3 * i + 1], xyz[3 * i + 2]);
    lattice_free(&lt);
    return 0;
}

/* ------------------------------------------------------------- geometry */

/* Scalar coefficient kappa at a physical point (Sec. 2.1, K = kappa Id). */
static double kappa_at(int kind, const double *p, const double *X) {
    const double two_pi = 6.283185307179586476925286766559;
    switch (kind) {
    case 0: return p[0];
    case 1: return p[0] + p[1] * sin(two_pi * p[2] * X[0]) * sin(two_pi * p[2] * X[1]) *
                              sin(two_pi * p[2] * X[2]);
    case 2: return exp(p[0] * sin(two_pi * p[2] * X[0]) * cos(two_pi * p[2] * X[1]));
    case 3: {
        int i = (int)p[2];
        return p[0] + p[1] * (pow(X[0], i) + pow(X[1], i) + pow(X[2], i));
    }
    default: return NAN;
    }
}

/* Micro vertex position: v1 + (x d1 + y d2 + z d3) / n with d_i = v_{i+1} - v1. */
static void micro_position(const double *v, int64_t n, int64_t x, int64_t y, int64_t z, double *X) {
    for (int k = 0; k < 3; ++k) {
        double d1 = v[3 + k] - v[k], d2 = v[6 + k] - v[k], d3 = v[9 + k] - v[k];
        X[k] = v[k] + ((double)x * d1 + (double)y * d2 + (double)z * d3) / (double)n;
    }
}

/* P1 element stiffness K_ij = kappa |T| grad(lambda_i) . grad(lambda_j) for a
 * tetrahedron with physical vertices P[4][3].  The barycentric gradients are
 * the rows of E^{-1}, E = [P1-P0, P2-P0, P3-P0] (columns), and
 * grad(lambda_0) = -(sum of the others).  Returns the signed det E. */
double oracle_element_stiffness(const double *P, double kappa, double *K) {
    double E[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) E[r][c] = P[3 * (c + 1) + r] - P[r];
    double det = E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1]) -
                 E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0]) +
                 E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
    /* inverse by cofactors: inv[i][j] = cof[j][i] / det */
    double inv[3][3];
    inv[0][0] = (E[1][1] * E[2][2] - E[1][2] * E[2][1]) / det;
    inv[0][1] = (E[0][2] * E[2][1] - E[0][1] * E[2][2]) / det;
    inv[0][2] = (E[0][1] * E[1][2] - E[0][2] * E[1][1]) / det;
    inv[1][0] = (E[1][2] * E[2][0] - E[1][0] * E[2][2]) / det;
    inv[1][1] = (E[0][0] * E[2][2] - E[0][2] * E[2][0]) / det;
    inv[1][2] = (E[0][2] * E[1][0] - E[0][0] * E[1][2]) / det;
    inv[2][0] = (E[1][0] * E[2][1] - E[1][1] * E[2][0]) / det;
    inv[2][1] = (E[0][1] * E[2][0] - E[0][0] * E[2][1]) / det;
    inv[2][2] = (E[0][0] * E[1][1] - E[0][1] * E[1][0]) / det;
    double g[4][3];
    for (int k = 0; k < 3; ++k) {
        g[1][k] = inv[0][k];
        g[2][k] = inv[1][k];
        g[3][k] = inv[2][k];
        g[0][k] = -(g[1][k] + g[2][k] + g[3][k]);
    }
    double vol = fabs(det) / 6.0;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
            K[4 * i + j] = kappa * vol * (g[i][0] * g[j][0] + g[i][1] * g[j][1] + g[i][2] * g[j][2]);
    return det;
}

/* Assembly of the restricted stiffness matrix R_t A R_t^T in stencil form.
 *
 * Micro-mesh: in the coordinates (a,b,c) = (x, x+y, x+y+z) the logical
 * tetrahedron is {0 <= a <= b <= c <= n}; every unit cube q + [0,1]^3 splits
 * into the six Kuhn simplices {q, q+e_s1, q+e_s1+e_s2, q+(1,1,1)}, and the
 * ones lying in the region form the micro-mesh (n^3 micro-tetrahedra, edge
 * vectors = D minus c).
 *
 * Output (N x 15, listing order of D):
 *   A[15 i + s]   = full stencil weight A^p_s (also for boundary neighbours)
 *   col[15 i + s] = interior index of p + d_s, or -1 if p + d_s is on the
 *                   macro boundary (the restricted matrix drops it).
 * Returns the number of micro-tetrahedra visited, or -1 on error. */
int64_t oracle_assemble(const double *verts, int level, int kind, const double *params,
                        double *A, int64_t *col) {
    lattice_t lt;
    if (lattice_init(&lt, level)) return -1;
    int64_t n = lt.n, N = oracle_num_interior(level);
    memset(A, 0, sizeof(double) * (size_t)(N * NDIR));
    for (int64_t i = 0; i < N * NDIR; ++i) col[i] = -1;
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int64_t ntets = 0;
    for (int64_t qa = 0; qa < n; ++qa)
        for (int64_t qb = 0; qb < n; ++qb)
            for (int64_t qc = 0; qc < n; ++qc)
                for (int s = 0; s < 6; ++s) {
                    int64_t abc[4][3];
                    abc[0][0] = qa; abc[0][1] = qb; abc[0][2] = qc;
                    for (int k = 1; k < 4; ++k) {
                        for (int m = 0; m < 3; ++m) abc[k][m] = abc[k - 1][m];
                        if (k < 3) abc[k][perm[s][k - 1]] += 1;
                    }
                    abc[3][0] = qa + 1; abc[3][1] = qb + 1; abc[3][2] = qc + 1;
                    int inside = 1;
                    for (int k = 0; k < 4 && inside; ++k)
                        inside = 0 <= abc[k][0] && abc[k][0] <= abc[k][1] && abc[k][1] <= abc[k][2] &&
                                 abc[k][2] <= n;
                    if (!inside) continue;
                    ++ntets;
                    int64_t xyz[4][3];
                    double P[12], cen[3] = {0, 0, 0};
                    for (int k = 0; k < 4; ++k) {
                        xyz[k][0] = abc[k][0];
                        xyz[k][1] = abc[k][1] - abc[k][0];
                        xyz[k][2] = abc[k][2] - abc[k][1];
                        micro_position(verts, n, xyz[k][0], xyz[k][1], xyz[k][2], P + 3 * k);
                        for (int m = 0; m < 3; ++m) cen[m] += 0.25 * P[3 * k + m];
                    }
                    double K[16];
                    oracle_element_stiffness(P, kappa_at(kind, params, cen), K);
                    for (int i = 0; i < 4; ++i) {
                        int64_t ri = interior_index(&lt, xyz[i][0], xyz[i][1], xyz[i][2]);
                        if (ri < 0) continue;
                        for (int j = 0; j < 4; ++j) {
                            int sl = slot_of((int)(xyz[j][0] - xyz[i][0]), (int)(xyz[j][1] - xyz[i][1]),
                                             (int)(xyz[j][2] - xyz[i][2]));
                            if (sl < 0) { lattice_free(&lt); return -1; }
                            A[NDIR * ri + sl] += K[4 * i + j];
                            col[NDIR * ri + sl] =
                                interior_index(&lt, xyz[j][0], xyz[j][1], xyz[j][2]);
                        }
                    }
                }
    lattice_free(&lt);
    return ntets;
}

/* Stencil rows A^p_d (d in listing order) of `count` given interior points,
 * each summed directly over the micro-tets incident to the point (Sec. 2.1,
 * the same element matrices as oracle_assemble, one point at a time, so it
 * serves lattices too large to assemble whole).  Point p is vertex k of the
 * Kuhn tetrahedron (q, sigma) exactly when q = p - (first k unit steps of
 * sigma) in the (a, b, c) coordinates; entries whose neighbour lies on the
 * macro boundary are 0.  Returns 0, or -1 for a point that is not interior. */
int oracle_stencil_at(const double *verts, int level, int kind, const double *params, int64_t count,
                      const int32_t *xyz, double *A_out) {
    const int64_t n = (int64_t)1 << level;
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    for (int64_t i = 0; i < count; ++i) {
        double *row = A_out + NDIR * i;
        for (int s = 0; s < NDIR; ++s) row[s] = 0.0;
        const int64_t px = xyz[3 * i], py = xyz[3 * i + 1], pz = xyz[3 * i + 2];
        if (!is_interior(n, px, py, pz)) return -1;
        const int64_t p_abc[3] = {px, px + py, px + py + pz};
        for (int s = 0; s < 6; ++s)
            for (int k = 0; k < 4; ++k) {
                int64_t abc[4][3];
                for (int m = 0; m < 3; ++m) abc[0][m] = p_abc[m];
                for (int m = 0; m < k; ++m) abc[0][perm[s][m]] -= 1;
                int ok = 1;
                for (int m = 0; m < 3; ++m) ok = ok && abc[0][m] >= 0 && abc[0][m] <= n - 1;
                if (!ok) continue;
                for (int v = 1; v < 4; ++v) {
                    for (int m = 0; m < 3; ++m) abc[v][m] = abc[v - 1][m];
                    if (v < 3) abc[v][perm[s][v - 1]] += 1;
                    else for (int m = 0; m < 3; ++m) abc[v][m] = abc[0][m] + 1;
                }
                for (int v = 0; v < 4 && ok; ++v)
                    ok = 0 <= abc[v][0] && abc[v][0] <= abc[v][1] && abc[v][1] <= abc[v][2] && abc[v][2] <= n;
                if (!ok) continue;
                int64_t vx[4][3];
                double P[12], cen[3] = {0, 0, 0};
                for (int v = 0; v < 4; ++v) {
                    vx[v][0] = abc[v][0];
                    vx[v][1] = abc[v][1] - abc[v][0];
                    vx[v][2] = abc[v][2] - abc[v][1];
                    micro_position(verts, n, vx[v][0], vx[v][1], vx[v][2], P + 3 * v);
                    for (int m = 0; m < 3; ++m) cen[m] += 0.25 * P[3 * v + m];
                }
                double K[16];
                oracle_element_stiffness(P, kappa_at(kind, params, cen), K);
                for (int j = 0; j < 4; ++j) {
                    if (!is_interior(n, vx[j][0], vx[j][1], vx[j][2])) continue;
                    const int sl = slot_of((int)(vx[j][0] - px), (int)(vx[j][1] - py), (int)(vx[j][2] - pz));
                    if (sl < 0) return -1;
                    row[sl] += K[4 * k + j];
                }
            }
    }
    return 0;
}

/* y = (R_t A R_t^T) x on the interior (Sec. 2.1 stencil matvec). */
void oracle_apply(int64_t N, const double *A, const int64_t *col, const double *x, double *y) {
    for (int64_t i = 0; i < N; ++i) {
        double acc = 0.0;
        for (int s = 0; s < NDIR; ++s) {
            int64_t j = col[NDIR * i + s];
            if (j >= 0) acc += A[NDIR * i + s] * x[j];
        }
        y[i] = acc;
    }
}

/* ----------------------------------------------------- ILU(0), definition */

/* Textbook ILU(0) in IKJ order on a CSR matrix with sorted column indices,
 * in place (Saad, Iterative Methods for Sparse Linear Systems, Alg. 10.4):
 * for i, for k < i in row i: a_ik /= a_kk; for j > k in row i with (k,j) in
 * the pattern: a_ij -= a_ik a_kj.  Afterwards the strict lower part is L
 * (unit diagonal implied) and the upper part incl. diagonal is U.
 * Returns 0, or 1 + (row) if a zero pivot is met. */
int64_t oracle_ilu0_csr_inplace(int64_t N, const int64_t *rowptr, const int64_t *colind, double *val) {
    int64_t *diag = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    if (!diag) return -1;
    for (int64_t i = 0; i < N; ++i) {
        diag[i] = -1;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
            if (colind[e] == i) diag[i] = e;
        if (diag[i] < 0) { free(diag); return 1 + i; }
    }
    for (int64_t i = 0; i < N; ++i) {
        for (int64_t e = rowptr[i]; e < rowptr[i + 1] && colind[e] < i; ++e) {
            int64_t k = colind[e];
            double pivot = val[diag[k]];
            if (pivot == 0.0) { free(diag); return 1 + k; }
            val[e] /= pivot;
            for (int64_t f = e + 1; f < rowptr[i + 1]; ++f) {
                int64_t j = colind[f];
                for (int64_t g = diag[k] + 1; g < rowptr[k + 1]; ++g)
                    if (colind[g] == j) { val[f] -= val[e] * val[g]; break; }
            }
        }
    }
    free(diag);
    return 0;
}

/* Restricted matrix in CSR (sorted columns) from the stencil form. */
static int stencil_to_csr(int64_t N, const double *A, const int64_t *col, int64_t **rp, int64_t **ci,
                          double **va) {
    int64_t nnz = 0;
    for (int64_t i = 0; i < N * NDIR; ++i) nnz += col[i] >= 0;
    *rp = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N + 1));
    *ci = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
    *va = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    if (!*rp || !*ci || !*va) return -1;
    int64_t e = 0;
    (*rp)[0] = 0;
    for (int64_t i = 0; i < N; ++i) {
        int64_t start = e;
        for (int s = 0; s < NDIR; ++s) {
            int64_t j = col[NDIR * i + s];
            if (j < 0) continue;
            /* insertion sort by column */
            int64_t f = e++;
            while (f > start && (*ci)[f - 1] > j) {
                (*ci)[f] = (*ci)[f - 1];
                (*va)[f] = (*va)[f - 1];
                --f;
            }
            (*ci)[f] = j;
            (*va)[f] = A[NDIR * i + s];
        }
        (*rp)[i + 1] = e;
    }
    return 0;
}

/* ILU(0) of the restricted matrix by the definition.  Returns L (N x 7, lower
 * slots of D; 0 where p+d is not interior), U (N x 7, upper slots 8..14) and
 * D = diag(U).  Returns 0 or the IKJ error code. */
int64_t oracle_ilu0_csr(int64_t N, const double *A, const int64_t *col, double *L, double *U, double *D) {
    int64_t *rp, *ci;
    double *va;
    if (stencil_to_csr(N, A, col, &rp, &ci, &va)) return -1;
    int64_t rc = oracle_ilu0_csr_inplace(N, rp, ci, va);
    if (rc == 0) {
        for (int64_t i = 0; i < N; ++i) {
            for (int s = 0; s < NLOW; ++s) { L[NLOW * i + s] = 0.0; U[NLOW * i + s] = 0.0; }
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
                int64_t j = ci[e];
                for (int s = 0; s < NDIR; ++s) {
                    if (col[NDIR * i + s] != j) continue;
                    if (s < NLOW) L[NLOW * i + s] = va[e];
                    else if (s == CENTRE) D[i] = va[e];
                    else U[NLOW * i + (s - 8)] = va[e];
                }
            }
        }
    }
    free(rp); free(ci); free(va);
    return rc;
}

/* ----------------------------------------------- ILU(0), stencil equations */

/* The stencil equations of Sec. 3 (eq. matrix-equations), solved point by
 * point in lexicographic order, in the order bc, s, bnw, be, w, bn, se and
 * then c, exactly as Alg. 1 does with its two face layers (here the whole
 * lattice is stored, which changes no arithmetic):
 *   A^p_d = sum_{dt in D_l u {c}} L^p_dt D^{p+dt} L^{p+d}_{dt-d},
 *   A^p_c = D^p + sum_{dt in D_l} (L^p_dt)^2 D^{p+dt}.
 * Terms whose point is not interior vanish (L = 0 there; the paper's
 * beta_c = 1 initialisation only guards the divisions).
 * Returns 0, or 1 + index of the first point with D^p <= 0. */
int64_t oracle_ilu0_stencil(int level, const double *A, const int64_t *col, double *L, double *D) {
    static const int order[NLOW] = {5, 1, 3, 6, 0, 4, 2}; /* bc s bnw be w bn se */
    int64_t N = oracle_num_interior(level);
    int64_t bad = 0;
    for (int64_t i = 0; i < N; ++i) {
        for (int s = 0; s < NLOW; ++s) L[NLOW * i + s] = 0.0;
        for (int oi = 0; oi < NLOW; ++oi) {
            int d = order[oi];
            int64_t q = col[NDIR * i + d]; /* p + d */
            if (q < 0) continue;
            double acc = A[NDIR * i + d];
            for (int dt = 0; dt < NLOW; ++dt) {
                if (dt == d) continue;
                int64_t r = col[NDIR * i + dt]; /* p + dt */
                if (r < 0) continue;
                int e = lower_slot_of(DIR[dt][0] - DIR[d][0], DIR[dt][1] - DIR[d][1], DIR[dt][2] - DIR[d][2]);
                if (e < 0) continue;
                acc -= L[NLOW * i + dt] * D[r] * L[NLOW * q + e];
            }
            L[NLOW * i + d] = acc / D[q];
        }
        double dc = A[NDIR * i + CENTRE];
        for (int dt = 0; dt < NLOW; ++dt) {
            int64_t r = col[NDIR * i + dt];
            if (r < 0) continue;
            dc -= L[NLOW * i + dt] * L[NLOW * i + dt] * D[r];
        }
        D[i] = dc;
        if (!(dc > 0.0) && bad == 0) bad = 1 + i;
    }
    return bad;
}

/* ------------------------------------------------------- smoothing steps */

static double norm2(int64_t N, const double *v) {
    double s = 0.0;
    for (int64_t i = 0; i < N; ++i) s += v[i] * v[i];
    return sqrt(s);
}

/* Smoothing step by the definition (Sec. 2.1 Richardson smoother):
 *   x <- x + (L D L^T)^{-1} (b - A x)
 * r = b - A x by CSR rows; L w = r by forward substitution (row-oriented);
 * (D L^T) z = w by backward substitution in column-oriented form.
 * relres[k] = ||b - A x_k|| / ||b|| for k = 0..nsweeps (may be NULL). */
int oracle_smooth_csr(int64_t N, const double *A, const int64_t *col, const double *L, const double *D,
                      const double *b, double *x, int nsweeps, double *relres) {
    int64_t *rp, *ci;
    double *va;
    if (stencil_to_csr(N, A, col, &rp, &ci, &va)) return -1;
    double *w = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double *acc = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double bn = norm2(N, b);
    for (int k = 0; k <= nsweeps; ++k) {
        for (int64_t i = 0; i < N; ++i) {
            double r = b[i];
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) r -= va[e] * x[ci[e]];
            w[i] = r;
        }
        if (relres) relres[k] = norm2(N, w) / (bn > 0 ? bn : 1.0);
        if (k == nsweeps) break;
        for (int64_t i = 0; i < N; ++i) {
            double s = w[i];
            for (int t = 0; t < NLOW; ++t) {
                int64_t j = col[NDIR * i + t];
                if (j >= 0) s -= L[NLOW * i + t] * w[j];
            }
            w[i] = s;
        }
        for (int64_t i = 0; i < N; ++i) acc[i] = 0.0;
        for (int64_t i = N - 1; i >= 0; --i) {
            double z = w[i] / D[i] - acc[i];
            w[i] = z;
            for (int t = 0; t < NLOW; ++t) {
                int64_t j = col[NDIR * i + t];
                if (j >= 0) acc[j] += L[NLOW * i + t] * z;
            }
        }
        for (int64_t i = 0; i < N; ++i) x[i] += w[i];
    }
    free(w); free(acc); free(rp); free(ci); free(va);
    return 0;
}

/* Smoothing step in the stencil form of Alg. 2, variant V2: pass 1 fuses the
 * residual with the forward substitution, pass 2 (reverse order) fuses the
 * D^{-1} scaling, the backward substitution with L^{p-d}_d and the update.
 * Weights whose neighbour is not interior are taken as 0 (V2).  Lw is the
 * per-point lower stencil (N x 7), Dinv the per-point inverse pivot. */
int oracle_smooth_stencil(int64_t N, const double *A, const int64_t *col, const double *Lw,
                          const double *Dinv, const double *b, double *x, int nsweeps, double *relres) {
    double *w = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double bn = norm2(N, b), rr = 0.0;
    for (int k = 0; k <= nsweeps; ++k) {
        rr = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            double r = b[i];
            for (int s = 0; s < NDIR; ++s) {
                int64_t j = col[NDIR * i + s];
                if (j >= 0) r -= A[NDIR * i + s] * x[j];
            }
            rr += r * r;
            for (int s = 0; s < NLOW; ++s) {
                int64_t j = col[NDIR * i + s];
                if (j >= 0) r -= Lw[NLOW * i + s] * w[j];
            }
            w[i] = r;
        }
        if (relres) relres[k] = sqrt(rr) / (bn > 0 ? bn : 1.0);
        if (k == nsweeps) break;
        for (int64_t i = N - 1; i >= 0; --i) {
            double v = w[i] * Dinv[i];
            for (int s = 0; s < NLOW; ++s) {
                int64_t j = col[NDIR * i + 8 + s]; /* p - d_s */
                if (j >= 0) v -= Lw[NLOW * j + s] * w[j];
            }
            w[i] = v;
            x[i] += v;
        }
    }
    free(w);
    return 0;
}

/* Mixed-precision smoothing step: the residual b - A x is formed in FP64 and
 * rounded to FP32, both substitutions run in FP32 with FP32 weights, and the
 * correction is added to x in FP64. */
int oracle_smooth_stencil_f32(int64_t N, const double *A, const int64_t *col, const float *Lw,
                              const float *Dinv, const double *b, double *x, int nsweeps, double *relres) {
    float *w = (float *)malloc(sizeof(float) * (size_t)(N > 0 ? N : 1));
    double bn = norm2(N, b);
    for (int k = 0; k <= nsweeps; ++k) {
        double rr = 0.0;
        for (int64_t i = 0; i < N; ++i) {
            double r = b[i];
            for (int s = 0; s < NDIR; ++s) {
                int64_t j = col[NDIR * i + s];
                if (j >= 0) r -= A[NDIR * i + s] * x[j];
            }
            rr += r * r;
            float v = (float)r;
            for (int s = 0; s < NLOW; ++s) {
                int64_t j = col[NDIR * i + s];
                if (j >= 0) v -= Lw[NLOW * i + s] * w[j];
            }
            w[i] = v;
        }
        if (relres) relres[k] = sqrt(rr) / (bn > 0 ? bn : 1.0);
        if (k == nsweeps) break;
        for (int64_t i = N - 1; i >= 0; --i) {
            float v = w[i] * Dinv[i];
            for (int s = 0; s < NLOW; ++s) {
                int64_t j = col[NDIR * i + 8 + s];
                if (j >= 0) v -= Lw[NLOW * j + s] * w[j];
            }
            w[i] = v;
            x[i] += (double)v;
        }
    }
    free(w);
    return 0;
}
