"""CPU FP64 oracle for the matrix-free ILU(0) smoother (arXiv:2210.15280).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product library.  The heavy loops
live in plain C (ilu_oracle.c, built with -ffp-contract=off); the surrogate
least-squares fit uses numpy/scipy library primitives.

Functions and the passage they follow:
  interior_points, index_of   Sec. 2.1 logical coordinates, lexicographic order
  assemble, apply              Sec. 2.1 bilinear form and stencil matvec
  stencil_at                   Sec. 2.1 stencil rows of single points
  ilu0                         Sec. 3 definition of ILU(0) (IKJ on CSR)
  ilu0_stencil                 Sec. 3 stencil equations / Alg. 1
  smooth                       Sec. 2.1 Richardson smoother with C = L D L^T
  smooth_stencil(_f32)         Alg. 2 (variant V2), FP64 / FP32-mixed
  Problem.boundary_points,     Sec. 4.1 boundary variant V1: boundary points and their
    Problem.v1_weights         stored exact factors in place of the surrogate
  sample_set, fit_surrogate    Sec. 4.1 sample sets S_d and LSQ fit
  eval_surrogate               Sec. 4.1 surrogate polynomials
  fit/eval_operator_surrogate  Sec. 4.2 surrogate for the operator A itself
  asymptotic_stencil           Sec. 3 Gauss-Seidel iteration of the stencil equations
  contraction_factor           Sec. 4.2 asymptotic rate by power iteration, applied to
                               the smoother's error propagation I - C^{-1} A
  Problem.sgs_factors          Sec. 2.1 symmetric Gauss-Seidel preconditioner in L D L^T form
  pcg                          Sec. 4.2 CG experiment: CG preconditioned by C^{-1}
  lfa_orientation              Sec. 3.1 (strategy on macro-elements): LFA smoothing factor of
                               the asymptotic ILU stencil for each vertex permutation
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from math import comb

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ilu_oracle.c")
_LIB = os.path.join(_HERE, "libilu_oracle.so")

# Paper listing order of D (Sec. 2.1); the first 7 are D_l, 7 is c, 8+k = -D_l[k].
DIRS = np.array([(-1, 0, 0), (0, -1, 0), (1, -1, 0), (-1, 1, -1), (0, 1, -1), (0, 0, -1), (1, 0, -1),
                 (0, 0, 0),
                 (1, 0, 0), (0, 1, 0), (-1, 1, 0), (1, -1, 1), (0, -1, 1), (0, 0, 1), (-1, 0, 1)])
DIR_NAMES = ("w", "s", "se", "bnw", "bn", "bc", "be", "c", "e", "n", "nw", "tse", "ts", "tc", "tw")
NLOW = 7
CENTRE = 7


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        i64, i32, dbl, p = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        lib.oracle_num_interior.restype = i64
        lib.oracle_num_interior.argtypes = [i32]
        lib.oracle_interior_points.argtypes = [i32, p]
        lib.oracle_index_of.argtypes = [i32, i64, p, p]
        lib.oracle_element_stiffness.restype = dbl
        lib.oracle_element_stiffness.argtypes = [p, dbl, p]
        lib.oracle_assemble.restype = i64
        lib.oracle_assemble.argtypes = [p, i32, i32, p, p, p]
        lib.oracle_apply.argtypes = [i64, p, p, p, p]
        lib.oracle_stencil_at.restype = i32
        lib.oracle_stencil_at.argtypes = [p, i32, i32, p, i64, p, p]
        lib.oracle_ilu0_csr_inplace.restype = i64
        lib.oracle_ilu0_csr_inplace.argtypes = [i64, p, p, p]
        lib.oracle_ilu0_csr.restype = i64
        lib.oracle_ilu0_csr.argtypes = [i64, p, p, p, p, p]
        lib.oracle_ilu0_stencil.restype = i64
        lib.oracle_ilu0_stencil.argtypes = [i32, p, p, p, p]
        lib.oracle_smooth_csr.argtypes = [i64, p, p, p, p, p, p, i32, p]
        lib.oracle_smooth_stencil.argtypes = [i64, p, p, p, p, p, p, i32, p]
        lib.oracle_smooth_stencil_f32.argtypes = [i64, p, p, p, p, p, p, i32, p]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


def num_interior(level: int) -> int:
    return comb((1 << level) - 1, 3)


def interior_points(level: int) -> np.ndarray:
    """(N,3) int32 interior coordinates in lexicographic order (z, then y, then x)."""
    out = np.zeros((num_interior(level), 3), dtype=np.int32)
    _L().oracle_interior_points(level, _ptr(out))
    return out


def index_of(level: int, xyz) -> np.ndarray:
    xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.int32).reshape(-1, 3))
    out = np.zeros(len(xyz), dtype=np.int64)
    _L().oracle_index_of(level, len(xyz), _ptr(xyz), _ptr(out))
    return out


def element_stiffness(P, kappa: float = 1.0):
    P = np.ascontiguousarray(np.asarray(P, dtype=np.float64).reshape(12))
    K = np.zeros(16)
    det = _L().oracle_element_stiffness(_ptr(P), float(kappa), _ptr(K))
    return K.reshape(4, 4), det


def stencil_at(tet, xyz) -> np.ndarray:
    """(k,15) stencil rows A^p_d of the given interior points of `tet`, summed
    point by point over the incident micro-tets (Sec. 2.1); boundary
    neighbours give 0."""
    xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.int32).reshape(-1, 3))
    verts = np.ascontiguousarray(np.asarray(tet.verts, dtype=np.float64).reshape(12))
    cp = tuple(tet.coeff_params)
    params = np.ascontiguousarray(np.asarray(cp + (0.0,) * (4 - len(cp)), dtype=np.float64))
    out = np.zeros((len(xyz), 15))
    if _L().oracle_stencil_at(_ptr(verts), int(tet.level), int(tet.coeff_kind), _ptr(params), len(xyz),
                              _ptr(xyz), _ptr(out)) != 0:
        raise ValueError("point not interior")
    return out


def random_interior(level: int, count: int, seed: int) -> np.ndarray:
    """`count` distinct uniformly drawn interior points (rejection sampling)."""
    n = 1 << level
    rng = np.random.default_rng(seed)
    pts = set()
    while len(pts) < count:
        c = rng.integers(1, n - 2, size=(4 * count, 3), endpoint=True)
        c = c[c.sum(1) <= n - 1]
        for p in map(tuple, c):
            pts.add(p)
            if len(pts) == count:
                break
    return np.array(sorted(pts), dtype=np.int32)


class Problem:
    """Assembled restricted operator of one macro-tetrahedron (stencil form)."""

    def __init__(self, verts, level: int, coeff_kind: int = 0, coeff_params=(1.0, 0, 0, 0)):
        self.verts = np.ascontiguousarray(np.asarray(verts, dtype=np.float64).reshape(12))
        self.level = int(level)
        self.n = 1 << level
        self.N = num_interior(level)
        self.coeff_kind = int(coeff_kind)
        self.params = np.ascontiguousarray(np.asarray(tuple(coeff_params) + (0.0,) * (4 - len(coeff_params)),
                                                      dtype=np.float64))
        self.A = np.zeros((self.N, 15))
        self.col = np.zeros((self.N, 15), dtype=np.int64)
        self.ntets = _L().oracle_assemble(_ptr(self.verts), self.level, self.coeff_kind, _ptr(self.params),
                                          _ptr(self.A), _ptr(self.col))
        if self.ntets < 0:
            raise RuntimeError("assembly failed")

    @classmethod
    def from_tet(cls, tet):
        return cls(tet.verts, tet.level, tet.coeff_kind, tet.coeff_params)

    def _op(self, A):
        return self.A if A is None else np.ascontiguousarray(A, dtype=np.float64).reshape(self.N, 15)

    def apply(self, x, A=None):
        """y = A x (or with the stencil array A given in the same layout, e.g. a surrogate operator)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros(self.N)
        _L().oracle_apply(self.N, _ptr(self._op(A)), _ptr(self.col), _ptr(x), _ptr(y))
        return y

    def csr(self):
        """Restricted matrix as a scipy CSR matrix (structural pattern kept)."""
        import scipy.sparse as sp
        m = self.col >= 0
        rows = np.repeat(np.arange(self.N), 15).reshape(self.N, 15)[m]
        A = sp.csr_matrix((self.A[m], (rows, self.col[m])), shape=(self.N, self.N))
        A.sort_indices()
        return A

    # -------------------------------------------------------------- ILU(0)
    def ilu0(self):
        """ILU(0) by the definition: returns (L (N,7), U (N,7 upper), D (N,))."""
        L = np.zeros((self.N, 7)); U = np.zeros((self.N, 7)); D = np.zeros(self.N)
        rc = _L().oracle_ilu0_csr(self.N, _ptr(self.A), _ptr(self.col), _ptr(L), _ptr(U), _ptr(D))
        if rc != 0:
            raise ArithmeticError("ILU(0) zero pivot (code %d)" % rc)
        return L, U, D

    def ilu0_stencil(self):
        """ILU(0) from the stencil equations (Alg. 1 order): (L (N,7), D (N,), breakdown)."""
        L = np.zeros((self.N, 7)); D = np.zeros(self.N)
        bad = _L().oracle_ilu0_stencil(self.level, _ptr(self.A), _ptr(self.col), _ptr(L), _ptr(D))
        return L, D, int(bad)

    # ------------------------------------------------------ smoothing steps
    def smooth(self, L, D, b, x0=None, nsweeps=1):
        """x <- x + (L D L^T)^{-1}(b - A x), nsweeps times (matrix form).  Returns (x, relres)."""
        x = np.zeros(self.N) if x0 is None else np.array(x0, dtype=np.float64)
        rel = np.zeros(nsweeps + 1)
        _L().oracle_smooth_csr(self.N, _ptr(self.A), _ptr(self.col), _ptr(np.ascontiguousarray(L)),
                               _ptr(np.ascontiguousarray(D)), _ptr(np.ascontiguousarray(b, dtype=np.float64)),
                               _ptr(x), int(nsweeps), _ptr(rel))
        return x, rel

    def smooth_stencil(self, Lw, Dinv, b, x0=None, nsweeps=1, A=None):
        """Alg. 2 (V2) with per-point weights Lw (N,7) and Dinv (N,); the residual
        uses A (default: the assembled operator).  Returns (x, relres)."""
        x = np.zeros(self.N) if x0 is None else np.array(x0, dtype=np.float64)
        rel = np.zeros(nsweeps + 1)
        _L().oracle_smooth_stencil(self.N, _ptr(self._op(A)), _ptr(self.col),
                                   _ptr(np.ascontiguousarray(Lw, dtype=np.float64)),
                                   _ptr(np.ascontiguousarray(Dinv, dtype=np.float64)),
                                   _ptr(np.ascontiguousarray(b, dtype=np.float64)), _ptr(x), int(nsweeps),
                                   _ptr(rel))
        return x, rel

    def smooth_stencil_f32(self, Lw, Dinv, b, x0=None, nsweeps=1, A=None):
        """Alg. 2 with FP64 residual, FP32 weights and substitutions, FP64 update."""
        x = np.zeros(self.N) if x0 is None else np.array(x0, dtype=np.float64)
        rel = np.zeros(nsweeps + 1)
        _L().oracle_smooth_stencil_f32(self.N, _ptr(self._op(A)), _ptr(self.col),
                                       _ptr(np.ascontiguousarray(Lw, dtype=np.float32)),
                                       _ptr(np.ascontiguousarray(Dinv, dtype=np.float32)),
                                       _ptr(np.ascontiguousarray(b, dtype=np.float64)), _ptr(x), int(nsweeps),
                                       _ptr(rel))
        return x, rel


    def boundary_points(self):
        """Mask (N,) of the boundary points of Sec. 4.1: interior points with at
        least one of the 14 stencil neighbours on the macro boundary."""
        return np.any(np.delete(self.col, CENTRE, axis=1) < 0, axis=1)

    def v1_weights(self, Lw, Dinv, L, D):
        """Boundary variant V1 (Sec. 4.1, the substitution algorithm with the
        boundary layer): the exact factors L^p_d and 1/D^p of every boundary
        point p replace its surrogate values.  The forward substitution at p
        reads L^p_d, the backward substitution reads 1/D^p at p and L^p_d at
        p + d, so replacing the per-point weights covers every use.  Returns
        (Lw1 (N,7), Dinv1 (N,))."""
        m = self.boundary_points()
        Lw1 = np.array(Lw, dtype=np.float64)
        Dinv1 = np.array(Dinv, dtype=np.float64)
        Lw1[m] = L[m]
        Dinv1[m] = 1.0 / D[m]
        return Lw1, Dinv1

    def sgs_factors(self):
        """Symmetric Gauss-Seidel (Sec. 2.1): C = (D_A + L_A) D_A^{-1} (D_A + L_A)^T
        with D_A, L_A the diagonal and strictly lower part of A, written as
        unit-lower L times D times L^T: L^p_d = A^p_d / A^{p+d}_c, D^p = A^p_c.
        Returns (L (N,7), D (N,)) in the layout of ilu0."""
        L = np.zeros((self.N, NLOW))
        for d in range(NLOW):
            j = self.col[:, d]
            m = j >= 0
            L[m, d] = self.A[m, d] / self.A[j[m], CENTRE]
        return L, self.A[:, CENTRE].copy()

    def precond(self, Lw, Dinv, f32: bool = False):
        """z = C^{-1} r as one smoothing step from zero with right-hand side r
        (Alg. 2; FP32 substitutions after rounding r when f32)."""
        if f32:
            L32, D32 = np.asarray(Lw, dtype=np.float32), np.asarray(Dinv, dtype=np.float32)
            return lambda r: self.smooth_stencil_f32(L32, D32, r, None, 1)[0]
        return lambda r: self.smooth_stencil(Lw, Dinv, r, None, 1)[0]


def pcg(problem: "Problem", precond, b, x0=None, maxit: int = 1000, rel_tol: float = 0.0, abs_tol: float = 0.0):
    """Preconditioned conjugate gradients (Hestenes-Stiefel) for A x = b with
    z = precond(r) ~ C^{-1} r, the use of the ILU as a CG preconditioner in
    Sec. 4.2.  Stops at the first k with ||r_k|| <= max(rel_tol ||b||, abs_tol)
    for the recursively updated residual.  Returns (x, iterations, ||r_k|| per
    iteration starting with k = 0, converged)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    tol = max(rel_tol * np.linalg.norm(b), abs_tol)
    r = b - problem.apply(x)
    hist = [np.linalg.norm(r)]
    if hist[-1] <= tol:
        return x, 0, hist, True
    z = precond(r)
    p = z.copy()
    rz = r @ z
    for k in range(1, maxit + 1):
        q = problem.apply(p)
        alpha = rz / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        hist.append(np.linalg.norm(r))
        if hist[-1] <= tol:
            return x, k, hist, True
        z = precond(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxit, hist, False


def ilu0_csr_inplace(rowptr, colind, val):
    """Generic IKJ ILU(0) on any CSR matrix with sorted columns (in place)."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    colind = np.ascontiguousarray(colind, dtype=np.int64)
    val = np.ascontiguousarray(val, dtype=np.float64).copy()
    rc = _L().oracle_ilu0_csr_inplace(len(rowptr) - 1, _ptr(rowptr), _ptr(colind), _ptr(val))
    if rc != 0:
        raise ArithmeticError("zero pivot")
    return val


# ---------------------------------------------------------------- surrogates

def sample_shift(d) -> np.ndarray:
    """Offset of S_d: 1 - min(d, 0) componentwise (Sec. 4.1, reading of the
    garbled shift; puts the first sample where p + d is interior)."""
    d = np.asarray(d)
    return 1 - np.minimum(d, 0)


def sample_side(level: int, d, stride: int) -> int:
    """Side M of the lattice simplex {k >= 0, sum k <= M} that S_d maps to."""
    n = 1 << level
    d = np.asarray(d)
    room = n - 1 - max(0, int(d.sum())) - int(sample_shift(d).sum())
    return room // stride if room >= 0 else -1


def effective_stride(level: int, degree, stride: int) -> int:
    """Largest s in {stride, stride/2, ..., 1} for which every S_d is unisolvent
    for P_{dx,dy,dz} (a lattice simplex of side M is unisolvent iff
    M >= dx + dy + dz); 0 if none is."""
    dg = (degree,) * 3 if np.isscalar(degree) else tuple(degree)
    need = sum(dg)
    s = stride
    while s >= 1:
        if all(sample_side(level, DIRS[t], s) >= need for t in list(range(NLOW)) + [CENTRE]):
            return s
        s //= 2
    return 0


def sample_set(level: int, slot: int, stride: int) -> np.ndarray:
    """Interior indices of S_d: p interior, p = shift_d (mod stride), p + d interior."""
    pts = interior_points(level).astype(np.int64)
    d = DIRS[slot]
    sh = sample_shift(d)
    m = np.all((pts - sh) % stride == 0, axis=1)
    q = pts + d
    n = 1 << level
    m &= np.all(q >= 1, axis=1) & (q.sum(axis=1) <= n - 1)
    return np.nonzero(m)[0]


def legendre_tensor_matrix(Xhat: np.ndarray, degree) -> np.ndarray:
    """Columns P_i(2x-1) P_j(2y-1) P_k(2z-1), column index (k (dy+1) + j)(dx+1) + i."""
    from numpy.polynomial import legendre as lg
    dx, dy, dz = (degree,) * 3 if np.isscalar(degree) else degree
    px = lg.legvander(2 * Xhat[:, 0] - 1, dx)
    py = lg.legvander(2 * Xhat[:, 1] - 1, dy)
    pz = lg.legvander(2 * Xhat[:, 2] - 1, dz)
    return (pz[:, :, None, None] * py[:, None, :, None] * px[:, None, None, :]).reshape(len(Xhat), -1)


def monomial_tensor_matrix(Xhat: np.ndarray, degree) -> np.ndarray:
    """Columns x^i y^j z^k (the paper's basis), same column order."""
    dx, dy, dz = (degree,) * 3 if np.isscalar(degree) else degree
    px = np.vander(Xhat[:, 0], dx + 1, increasing=True)
    py = np.vander(Xhat[:, 1], dy + 1, increasing=True)
    pz = np.vander(Xhat[:, 2], dz + 1, increasing=True)
    return (pz[:, :, None, None] * py[:, None, :, None] * px[:, None, None, :]).reshape(len(Xhat), -1)


def lsq(V: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Least squares by column-pivoted Householder QR (LAPACK geqp3)."""
    import scipy.linalg as sla
    Q, R, piv = sla.qr(V, mode="economic", pivoting=True)
    c = np.zeros(V.shape[1])
    c[piv] = sla.solve_triangular(R, Q.T @ y)
    return c


def fit_surrogate(level: int, L: np.ndarray, D: np.ndarray, degree, stride: int, basis: str = "legendre"):
    """One polynomial per d in D_l (fit to L^p_d) and one for c (fit to 1/D^p),
    each on its sample set S_d with coordinates X^ = (x,y,z)/2^L (Sec. 4.1 and
    the sampling step of Alg. 1).  Returns coeffs (8, K): rows 0..6 = D_l, 7 = c."""
    pts = interior_points(level).astype(np.float64) / (1 << level)
    mat = legendre_tensor_matrix if basis == "legendre" else monomial_tensor_matrix
    out = []
    for t in list(range(NLOW)) + [CENTRE]:
        idx = sample_set(level, t, stride)
        y = L[idx, t] if t < NLOW else 1.0 / D[idx]
        out.append(lsq(mat(pts[idx], degree), y))
    return np.array(out)


def eval_surrogate(level: int, coeffs: np.ndarray, degree, basis: str = "legendre"):
    """Surrogate weights at every interior point: Lw (N,7) and Dinv (N,).
    V2 zeroing of weights whose neighbour is not interior happens inside the
    sweep (it multiplies a boundary value that is never read)."""
    pts = interior_points(level).astype(np.float64) / (1 << level)
    mat = legendre_tensor_matrix if basis == "legendre" else monomial_tensor_matrix
    vals = mat(pts, degree) @ coeffs.T
    return np.ascontiguousarray(vals[:, :NLOW]), np.ascontiguousarray(vals[:, NLOW])


def fit_operator_surrogate(level: int, A: np.ndarray, degree, stride: int, basis: str = "legendre"):
    """Surrogate for the operator (Sec. 4.2 approximates A by surrogate
    polynomials as well): one polynomial per d in D_l fit to A^p_d and one
    for c fit to A^p_c, on the sample sets S_d of the ILU fit (p + d interior,
    so the dropped boundary entries are never samples).  A is the (N,15)
    stencil array.  Returns coeffs (8, K): rows 0..6 = D_l, 7 = c."""
    pts = interior_points(level).astype(np.float64) / (1 << level)
    mat = legendre_tensor_matrix if basis == "legendre" else monomial_tensor_matrix
    out = []
    for t in list(range(NLOW)) + [CENTRE]:
        idx = sample_set(level, t, stride)
        out.append(lsq(mat(pts[idx], degree), A[idx, t]))
    return np.array(out)


def eval_operator_surrogate(level: int, coeffs: np.ndarray, degree, basis: str = "legendre") -> np.ndarray:
    """The surrogate stencil in the (N,15) layout: lower weights from their
    polynomials at p, the upper weight of direction -d_k as the lower
    polynomial k at p - d_k (A^p_{-d} = A^{p-d}_d, so the surrogate stays
    symmetric), and the centre from the zero row sums of the unrestricted
    operator, A_c = -(sum of the 14 neighbour weights), because
    a(phi_p, 1) = 0 for every coefficient (Sec. 2.1).  The fitted centre
    polynomial (row 7) is not used: a fitted centre breaks the row sums by
    the fit error, which is far larger than the O(h^3) smallest eigenvalues
    of A and makes the iteration diverge at fine levels.  Entries whose
    neighbour is not interior multiply nothing (they still enter the centre)."""
    pts = interior_points(level).astype(np.float64)
    n = 1 << level
    mat = legendre_tensor_matrix if basis == "legendre" else monomial_tensor_matrix
    out = np.zeros((len(pts), 15))
    vals = mat(pts / n, degree) @ coeffs.T
    out[:, :NLOW] = vals[:, :NLOW]
    for k in range(NLOW):
        out[:, 8 + k] = mat((pts - DIRS[k]) / n, degree) @ coeffs[k]
    out[:, CENTRE] = -(out[:, :NLOW].sum(axis=1) + out[:, 8:].sum(axis=1))
    return out


def surrogate_error(level: int, L, D, Lw, Dinv):
    """Per-direction relative discrete L2 error and max-abs error over the
    points whose neighbour p + d is interior (for c: all points, on 1/D)."""
    n = 1 << level
    pts = interior_points(level).astype(np.int64)
    rel, mx = [], []
    for t in range(NLOW):
        q = pts + DIRS[t]
        m = np.all(q >= 1, axis=1) & (q.sum(axis=1) <= n - 1)
        e = Lw[m, t] - L[m, t]
        rel.append(np.linalg.norm(e) / max(np.linalg.norm(L[m, t]), 1e-300))
        mx.append(np.abs(e).max() if e.size else 0.0)
    e = Dinv - 1.0 / D
    rel.append(np.linalg.norm(e) / np.linalg.norm(1.0 / D))
    mx.append(np.abs(e).max())
    return np.array(rel), np.array(mx)


# --------------------------------------------------------------- asymptotics

def asymptotic_stencil(Ad, iters: int = 20000, tol: float = 1e-15):
    """Gauss-Seidel iteration of the stencil equations with a constant stencil
    A_d (Sec. 3): start from L_c = D_c = 1 and L_d = 0, sweep the equations in
    the order bc, s, bnw, be, w, bn, se, c, with every neighbour value equal
    to the current iterate.  Returns (L (7,), D)."""
    Ad = np.asarray(Ad, dtype=np.float64)
    L = np.zeros(7)
    D = 1.0
    lower = {tuple(DIRS[t]): t for t in range(NLOW)}
    order = (5, 1, 3, 6, 0, 4, 2)
    for _ in range(iters):
        Lold, Dold = L.copy(), D
        for d in order:
            acc = Ad[d]
            for dt in range(NLOW):
                if dt == d:
                    continue
                e = lower.get(tuple(DIRS[dt] - DIRS[d]))
                if e is not None:
                    acc -= L[dt] * D * L[e]
            L[d] = acc / D
        D = Ad[CENTRE] - D * np.sum(L * L)
        if np.max(np.abs(L - Lold)) < tol and abs(D - Dold) < tol * abs(D):
            break
    return L, D


# ------------------------------------------------------------- contraction

def contraction_factor(problem: "Problem", step, x0, steps: int = 20):
    """Asymptotic contraction of one smoother by power iteration (the rate
    definition of the numerical results in Sec. 4.2, applied to the smoothing
    step itself): with b = 0 a step maps the error e to (I - C^{-1} A) e.
    Start from x0, apply `steps` steps, normalising after each.

    `step(y)` must return one smoothing step of y with zero right-hand side.
    Returns (rho, rho_res): rho = ||x_k||_2 / ||x_{k-1}||_2 of the last step,
    rho_res = (||A x_k||_2 / ||A x_0||_2)^(1/k) of the unnormalised iteration."""
    y = np.array(x0, dtype=np.float64)
    y /= np.linalg.norm(y)
    ra = np.linalg.norm(problem.apply(y))
    rho, logsum = float("nan"), 0.0
    for _ in range(steps):
        z = step(y)
        nz = np.linalg.norm(z)
        rz = np.linalg.norm(problem.apply(z))
        rho = nz                     # ||y|| = 1
        logsum += np.log(rz / ra)
        y = z / nz
        ra = rz / nz
    return rho, float(np.exp(logsum / steps))


# ------------------------------------------------------------------ LFA

def constant_stencil(verts) -> np.ndarray:
    """The 15 stencil weights A_d (listing order of D) for kappa = 1 at an
    interior point whose neighbours are all interior (level 4, point (4,4,4)):
    with an affine macro map and a constant coefficient every such point has
    the same stencil (Sec. 3.1, strategy on macro-elements)."""
    class _T:
        pass
    t = _T()
    t.verts, t.level, t.coeff_kind, t.coeff_params = verts, 4, 0, (1.0, 0.0, 0.0, 0.0)
    return stencil_at(t, [[4, 4, 4]])[0]


def lfa_frequencies(samples: int = 16) -> np.ndarray:
    """Theta_osc = (-pi, pi)^3 minus (-pi/2, pi/2)^3 sampled on a uniform grid
    of `samples` cell centres per direction (reading of the sampling rule):
    theta_j = -pi + (2 j + 1) pi / samples, kept if some |theta_i| >= pi/2."""
    th = -np.pi + (2 * np.arange(samples) + 1) * np.pi / samples
    T = np.stack(np.meshgrid(th, th, th, indexing="ij"), -1).reshape(-1, 3)
    return T[np.abs(T).max(axis=1) >= np.pi / 2]


def smoothing_factor(A, L, D, thetas) -> float:
    """mu = max over thetas of |(L D conj(L) - A) / (L D conj(L))| with the
    symbols L(theta) = 1 + sum_{d in D_l} L_d e^{i d.theta}, D(theta) = D and
    A(theta) = sum_{d in D} A_d e^{i d.theta} (Sec. 3)."""
    Ls = 1.0 + sum(L[d] * np.exp(1j * (thetas @ DIRS[d])) for d in range(NLOW))
    As = sum(A[d] * np.exp(1j * (thetas @ DIRS[d])) for d in range(15))
    C = Ls * D * np.conj(Ls)
    return float(np.abs((C - As) / C).max())


def permutations():
    """The 24 vertex permutations s = (s1 s2 s3 s4) in lexicographic order."""
    import itertools
    return [tuple(p) for p in itertools.permutations((1, 2, 3, 4))]


def permute_vertices(verts, s):
    """Reading of the permutation notation: original vertex i becomes vertex
    s_i of the permuted tetrahedron."""
    v = np.asarray(verts, dtype=np.float64).reshape(4, 3)
    out = np.empty_like(v)
    for i, si in enumerate(s):
        out[si - 1] = v[i]
    return out


def lfa_orientation(verts, samples: int = 16):
    """Smoothing factor mu of the asymptotic ILU stencil (LFA) for each of the
    24 vertex permutations of one macro-tetrahedron, and the index of the
    smallest (Sec. 3.1, strategy on macro-elements).  Returns (mu (24,), best)."""
    th = lfa_frequencies(samples)
    mu = []
    for s in permutations():
        A = constant_stencil(permute_vertices(verts, s))
        L, D = asymptotic_stencil(A)
        mu.append(smoothing_factor(A, L, D, th))
    mu = np.array(mu)
    return mu, int(np.argmin(mu))
