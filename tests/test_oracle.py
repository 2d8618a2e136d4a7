"""Pins for the CPU oracle: every check compares the oracle with something
other than itself -- a closed form, an invariant of the P1 bilinear form, an
independent library routine (dense Cholesky, QR), a brute-force count, or a
value printed in the paper.  No GPU needed."""
from math import comb

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W

# --------------------------------------------------------------------------- lattice


@pytest.mark.parametrize("level", [2, 3, 4, 5, 6])
def test_interior_count_and_numbering(level):
    # G-interior = {x,y,z >= 1, x+y+z < 2^L} (Sec. 2.1); brute-force enumeration
    n = 1 << level
    brute = [(x, y, z) for z in range(n + 1) for y in range(n + 1) for x in range(n + 1)
             if x >= 1 and y >= 1 and z >= 1 and x + y + z < n]
    assert O.num_interior(level) == len(brute) == comb(n - 1, 3)
    pts = O.interior_points(level)
    # lexicographic: z slowest, then y, then x (Sec. 2.1 ordering)
    assert [tuple(p) for p in pts] == sorted(brute, key=lambda p: (p[2], p[1], p[0]))
    assert np.array_equal(O.index_of(level, pts), np.arange(len(pts)))
    assert np.all(O.index_of(level, [[0, 1, 1], [1, 1, n - 2], [1, 0, 1]]) == [-1, -1, -1])


def test_interior_counts_of_the_workloads():
    assert O.num_interior(4) == 455
    assert O.num_interior(7) == 333_375
    assert O.num_interior(8) == 2_731_135
    assert O.num_interior(9) == 22_108_415
    # hyperplanes t = x + 2y + 3z over the interior: 3n - 11 of them
    for level in (3, 4, 5):
        pts = O.interior_points(level)
        t = pts[:, 0] + 2 * pts[:, 1] + 3 * pts[:, 2]
        assert len(np.unique(t)) == 3 * (1 << level) - 11


# ------------------------------------------------------------------------ micro-mesh


@pytest.mark.parametrize("level", [2, 3, 4])
def test_micro_mesh_has_8_to_the_L_tets(level):
    # uniform 8-subdivision, L times (Sec. 2.1, Bey refinement)
    assert O.Problem(W.REFERENCE_TET, level).ntets == 8 ** level


def test_element_stiffness_against_face_normal_formula():
    # independent formula: K_ij = (n_i . n_j) / (9 |T|) with n_i the area-weighted
    # outward normal of the face opposite vertex i (|n_i| = face area)
    rng = np.random.default_rng(7)
    for _ in range(20):
        P = rng.uniform(-1, 1, size=(4, 3))
        K, det = O.element_stiffness(P, 2.5)
        vol = abs(np.linalg.det(P[1:] - P[0])) / 6
        nrm = []
        for i in range(4):
            a, b, c = [P[j] for j in range(4) if j != i]
            nv = 0.5 * np.cross(b - a, c - a)
            if np.dot(nv, P[i] - a) > 0:
                nv = -nv
            nrm.append(nv)
        K2 = np.array([[2.5 * np.dot(nrm[i], nrm[j]) / (9 * vol) for j in range(4)] for i in range(4)])
        np.testing.assert_allclose(K, K2, rtol=1e-12, atol=1e-12 * np.abs(K2).max())


# ------------------------------------------------------------------------- assembly

# Closed form, derived by hand for the reference tetrahedron with kappa = 1:
# in (a,b,c) = (x, x+y, x+y+z) the form is (1/n) int grad(u)^T G grad(v) with
# G = [[1,1,1],[1,2,2],[1,2,3]] on the Kuhn lattice; e.g. the main diagonal
# (xyz-direction e) lies in all six Kuhn simplices of one cube and gets
# -2(G12+G13+G23)/(6n) = -4h/3.  In units of h/3 (h = 2^-L):
REFERENCE_STENCIL = dict(w=-4, s=-2, se=-1, bnw=1, bn=-1, bc=-4, be=1, c=20,
                         e=-4, n=-2, nw=-1, tse=1, ts=-1, tc=-4, tw=1)


@pytest.mark.parametrize("level", [3, 4, 5])
def test_reference_tet_closed_form(level):
    P = O.Problem(W.REFERENCE_TET, level)
    h = 1.0 / P.n
    want = np.array([REFERENCE_STENCIL[nm] for nm in O.DIR_NAMES]) * h / 3
    # every interior point has the full translation-invariant stencil
    np.testing.assert_allclose(P.A, np.broadcast_to(want, P.A.shape), rtol=0, atol=1e-15)


def _jittered(level, kind, params, seed=11):
    t = W.make_tet(seed, level, kind, params, jitter=0.15)
    return t, O.Problem.from_tet(t)


@pytest.mark.parametrize("coeff", [W.KAPPA_SIN, W.KAPPA_EXP, (W.COEFF_POLY, (1.0, 10.0, 3.0, 0.0))])
def test_row_sums_vanish_and_symmetry(coeff):
    # a(phi_i, 1) = 0 for every kappa: the full stencil sums to 0 at every interior point
    t, P = _jittered(4, *coeff)
    assert np.abs(P.A.sum(axis=1)).max() < 1e-14 * np.abs(P.A).max()
    # A^p_d = A^{p+d}_{-d} (symmetric bilinear form)
    for s in range(7):
        j = P.col[:, 8 + s]
        m = j >= 0
        np.testing.assert_allclose(P.A[m, 8 + s], P.A[j[m], s], rtol=1e-13, atol=1e-16)
    # diagonal positive
    assert np.all(P.A[:, 7] > 0)


@pytest.mark.parametrize("level", [3, 4])
def test_stencil_at_equals_assembly(level):
    # point-by-point stencil rows (sum over the 24 incident micro-tets) equal
    # the rows of the whole-lattice assembly, boundary neighbours dropped
    t, P = _jittered(level, *W.KAPPA_EXP, seed=21)
    A = O.stencil_at(t, O.interior_points(level))
    want = np.where(P.col >= 0, P.A, 0.0)
    assert np.abs(A - want).max() <= 1e-14 * np.abs(want).max()


def test_stencil_at_closed_form_and_row_sums_at_level9():
    # a lattice too large to assemble whole: deep interior points of the
    # reference tet have the closed-form stencil; on a jittered tet with a
    # variable coefficient the rows of points away from the boundary sum to 0
    n = 512
    ref = W.Tet(W.REFERENCE_TET, 9, W.COEFF_CONST, (1.0, 0, 0, 0), 0)
    pts = np.array([[100, 100, 100], [3, 4, 5], [200, 150, 140], [1, 1, 509 - 300]], dtype=np.int32)
    deep = pts[np.all(pts >= 2, axis=1) & (pts.sum(axis=1) <= n - 3)]
    want = np.array([REFERENCE_STENCIL[nm] for nm in O.DIR_NAMES]) / (3 * n)
    np.testing.assert_allclose(O.stencil_at(ref, deep), np.broadcast_to(want, (len(deep), 15)), rtol=0, atol=1e-15)
    t = W.make_tet(5, 9, *W.KAPPA_EXP, jitter=0.15)
    sample = O.random_interior(9, 400, seed=3)
    away = sample[np.all(sample >= 2, axis=1) & (sample.sum(axis=1) <= n - 3)]
    A = O.stencil_at(t, away)
    assert np.abs(A.sum(axis=1)).max() <= 1e-13 * np.abs(A).max()
    assert np.all(A[:, 7] > 0)


def test_second_moment_identity():
    # P1 reproduces quadratics in the weak sense on a translation-invariant
    # lattice: J (sum_d A_d d d^T) J^T = -2 h |det J| I  (kappa = 1, any affine tet)
    t, P = _jittered(5, W.COEFF_CONST, (1.0,), seed=3)
    v = np.array(t.verts)
    J = (v[1:] - v[0]).T
    h = 1.0 / P.n
    for p in ([8, 8, 8], [3, 5, 7], [10, 4, 2]):
        i = O.index_of(5, [p])[0]
        M = sum(P.A[i, s] * np.outer(O.DIRS[s], O.DIRS[s]) for s in range(15))
        np.testing.assert_allclose(J @ M @ J.T, -2 * h * abs(np.linalg.det(J)) * np.eye(3), atol=1e-13)


def test_stiffness_scales_with_h():
    # A_d ~ Theta(h) (Remark in Sec. 3): halving h halves the stencil
    a4 = O.Problem(W.REFERENCE_TET, 4).A[100]
    a5 = O.Problem(W.REFERENCE_TET, 5).A[100]
    np.testing.assert_allclose(a5, a4 / 2, rtol=1e-13)


# ---------------------------------------------------------------------------- ILU(0)


def _factor_matrices(P, L, D):
    m = P.col[:, :7] >= 0
    rows = np.repeat(np.arange(P.N), 7).reshape(P.N, 7)[m]
    Lm = sp.csr_matrix((L[m], (rows, P.col[:, :7][m])), shape=(P.N, P.N)) + sp.identity(P.N)
    return Lm, sp.diags(D)


@pytest.mark.parametrize("level,coeff", [(3, W.KAPPA_SIN), (4, W.KAPPA_SIN), (5, W.KAPPA_EXP)])
def test_ilu_definition_on_pattern(level, coeff):
    # (L D L^T)_ij = A_ij for (i,j) in S_A (Sec. 3)
    t, P = _jittered(level, *coeff)
    L, U, D = P.ilu0()
    Lm, Dm = _factor_matrices(P, L, D)
    C = (Lm @ Dm @ Lm.T).tocsr()
    A = P.csr()
    m = P.col >= 0
    rows = np.repeat(np.arange(P.N), 15).reshape(P.N, 15)[m]
    cvals = np.asarray(C[rows, P.col[m]]).ravel()
    np.testing.assert_allclose(cvals, np.asarray(A[rows, P.col[m]]).ravel(), rtol=0,
                               atol=1e-13 * np.abs(P.A).max())
    # U = D L^T
    for s in range(7):
        j = P.col[:, 8 + s]
        mm = j >= 0
        np.testing.assert_allclose(U[mm, s], D[mm] * L[j[mm], s], rtol=1e-13, atol=1e-300)


@pytest.mark.parametrize("level,coeff", [(4, W.KAPPA_SIN), (5, (W.COEFF_POLY, (1.0, 10.0, 2.0, 0.0)))])
def test_stencil_recurrences_equal_definition(level, coeff):
    # Alg. 1 / eq. (matrix-equations) reproduce the IKJ ILU(0)
    t, P = _jittered(level, *coeff)
    L, U, D = P.ilu0()
    L2, D2, bad = P.ilu0_stencil()
    assert bad == 0
    np.testing.assert_allclose(L2, L, rtol=0, atol=1e-13)
    np.testing.assert_allclose(D2, D, rtol=1e-13)


def test_full_pattern_ilu_is_dense_cholesky():
    # ILU(0) with a full pattern drops nothing, so it is the exact LDL^T = Cholesky
    t, P = _jittered(3, *W.KAPPA_SIN)
    A = P.csr().toarray()
    N = P.N
    rowptr = np.arange(0, N * N + 1, N)
    colind = np.tile(np.arange(N), N)
    LU = O.ilu0_csr_inplace(rowptr, colind, A.ravel()).reshape(N, N)
    R = np.linalg.cholesky(A)          # A = R R^T
    d = np.diag(R) ** 2
    Lx = R / np.diag(R)[None, :]
    np.testing.assert_allclose(np.tril(LU, -1), np.tril(Lx, -1), atol=1e-13)
    np.testing.assert_allclose(np.diag(LU), d, rtol=1e-13)


def test_ilu_rows_before_first_dropped_fill_are_exact():
    # rows computed before any fill has been dropped coincide with the exact factor
    t, P = _jittered(4, *W.KAPPA_SIN)
    A = P.csr().toarray()
    R = np.linalg.cholesky(A)
    Lx = R / np.diag(R)[None, :]
    pattern = A != 0
    fill = (np.abs(np.tril(Lx, -1)) > 1e-15) & ~pattern
    i0 = int(np.nonzero(fill.any(axis=1))[0].min())
    assert i0 > 0
    L, U, D = P.ilu0()
    Lm, _ = _factor_matrices(P, L, D)
    Ld = Lm.toarray()
    np.testing.assert_allclose(Ld[:i0], Lx[:i0], atol=1e-14)
    np.testing.assert_allclose(D[:i0], (np.diag(R) ** 2)[:i0], rtol=1e-13)


def test_fill_in_is_12_offsets_per_row():
    # "our fill-in consists of 12 additional nonzero entries per row" (Sec. 3 remark)
    t, P = _jittered(5, *W.KAPPA_SIN)
    L, U, D = P.ilu0()
    Lm, Dm = _factor_matrices(P, L, D)
    C = (Lm @ Dm @ Lm.T).tocsr()
    i = O.index_of(5, [[10, 10, 8]])[0]
    pts = O.interior_points(5)
    row = C.getrow(i)
    offs = {tuple(pts[j] - pts[i]) for j, v in zip(row.indices, row.data) if v != 0}
    stencil = {tuple(d) for d in O.DIRS}
    assert stencil <= offs
    assert len(offs - stencil) == 12


def test_interior_ilu_converges_to_asymptotic_stencil():
    # deep inside, the factors approach the Gauss-Seidel fixed point of the stencil
    # equations (Sec. 3); D^inf ~ h and L^inf ~ 1 (Remark), A_c = D^inf (1 + sum L^2)
    prev = None
    for level in (5, 6):
        P = O.Problem(W.REFERENCE_TET, level)
        L, U, D = P.ilu0()
        c = P.n // 4
        i = O.index_of(level, [[c, c, c]])[0]
        Li, Di = O.asymptotic_stencil(P.A[i])
        tol = 1e-6 if level == 5 else 1e-13
        np.testing.assert_allclose(L[i], Li, atol=tol)
        np.testing.assert_allclose(D[i], Di, rtol=tol)
        np.testing.assert_allclose(P.A[i, 7], Di * (1 + np.sum(Li ** 2)), rtol=1e-13)
        if prev is not None:
            np.testing.assert_allclose(Li, prev[0], atol=1e-12)
            np.testing.assert_allclose(Di, prev[1] / 2, rtol=1e-12)
        prev = (Li, Di)


def test_breakdown_is_reported():
    # a coefficient that is negative on part of the tet destroys positivity of pivots
    t = W.make_tet(1, 4, W.COEFF_SINPROD, (0.0, 1.0, 1.0, 0.0))
    P = O.Problem.from_tet(t)
    L, D, bad = P.ilu0_stencil()
    assert bad > 0


# ---------------------------------------------------------------------- smoothing


@pytest.mark.parametrize("level", [3, 4])
def test_smoothing_step_solves_with_ldlt(level):
    # x1 - x0 = (L D L^T)^{-1} (b - A x0): verified by products only
    t, P = _jittered(level, *W.KAPPA_SIN)
    L, U, D = P.ilu0()
    rng = np.random.default_rng(1)
    b = rng.uniform(-1, 1, P.N)
    x0 = rng.uniform(-1, 1, P.N)
    x1, _ = P.smooth(L, D, b, x0, nsweeps=1)
    Lm, Dm = _factor_matrices(P, L, D)
    lhs = Lm @ (Dm @ (Lm.T @ (x1 - x0)))
    rhs = b - P.apply(x0)
    assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(rhs)


def test_first_step_from_zero_is_preconditioned_rhs():
    t, P = _jittered(4, *W.KAPPA_SIN)
    L, U, D = P.ilu0()
    b = t.rhs()
    x1, rel = P.smooth(L, D, b, nsweeps=1)
    Lm, Dm = _factor_matrices(P, L, D)
    assert np.linalg.norm(Lm @ (Dm @ (Lm.T @ x1)) - b) <= 1e-13 * np.linalg.norm(b)
    assert rel[0] == pytest.approx(1.0)


@pytest.mark.parametrize("level,coeff", [(4, W.KAPPA_SIN), (5, W.KAPPA_EXP)])
def test_stencil_sweep_equals_matrix_sweep(level, coeff):
    # Alg. 2 (stencil form, V2) with the exact factors = the definition
    t, P = _jittered(level, *coeff)
    L, U, D = P.ilu0()
    b = t.rhs()
    x, r = P.smooth(L, D, b, nsweeps=5)
    x2, r2 = P.smooth_stencil(L, 1.0 / D, b, nsweeps=5)
    np.testing.assert_allclose(x2, x, rtol=0, atol=1e-13 * np.abs(x).max())
    np.testing.assert_allclose(r2, r, rtol=1e-10)
    assert r[-1] < r[0] * 0.05


def test_mixed_precision_sweep_tracks_fp64():
    t, P = _jittered(4, *W.KAPPA_SIN)
    L, U, D = P.ilu0()
    b = t.rhs()
    x, r = P.smooth_stencil(L, 1.0 / D, b, nsweeps=30)
    x32, r32 = P.smooth_stencil_f32(L.astype(np.float32), (1.0 / D).astype(np.float32), b, nsweeps=30)
    # the FP64 residual keeps driving the error down past FP32 resolution
    assert r32[-1] < 1e-9
    np.testing.assert_allclose(r32[:5], r[:5], rtol=1e-4)


def _dense_unit_lower(P, Lw):
    # unit-lower L with L[p, p+d] = L^p_d for the lower directions whose
    # neighbour is interior (the V2 rule drops the others), dtype of Lw
    N = P.N
    Lm = np.eye(N, dtype=Lw.dtype)
    for d in range(O.NLOW):
        j = P.col[:, d]
        m = j >= 0
        Lm[np.nonzero(m)[0], j[m]] = Lw[m, d]
    return Lm


@pytest.mark.parametrize("level,start", [(3, "zero"), (4, "zero"), (4, "random")])
def test_fp32_emulation_is_fp32_triangular_solves(level, start):
    # The mixed-precision step (FP64 residual rounded to FP32, both
    # substitutions in FP32, FP64 update) rebuilt from dense FP32 triangular
    # solves (LAPACK strtrs through scipy; no code shared with the oracle's
    # stencil loops): the oracle's FP32 emulation agrees to a few FP32 units of
    # the correction, and it is not the FP64 step (which it would be if the
    # emulation ran the substitutions in FP64).  From x = 0 the result is
    # (double) w with w an FP32 vector, so it is exactly FP32-representable.
    import scipy.linalg as sla
    t, P = _jittered(level, *W.KAPPA_EXP)
    L, U, D = P.ilu0()
    # a surrogate stand-in: exact factors off by a smooth relative perturbation
    pts = O.interior_points(level).astype(np.float64) / (1 << level)
    pert = 1.0 + 0.05 * np.sin(7.0 * pts[:, 0] + 3.0 * pts[:, 1] - 5.0 * pts[:, 2])
    Lw32 = (L * pert[:, None]).astype(np.float32)
    Di32 = (pert / D).astype(np.float32)
    b = t.rhs()
    x0 = np.zeros(P.N) if start == "zero" else np.random.default_rng(level).uniform(-1, 1, P.N)
    r32 = (b - P.apply(x0)).astype(np.float32)
    Lm = _dense_unit_lower(P, Lw32)
    y = sla.solve_triangular(Lm, r32, lower=True, unit_diagonal=True)
    z = (Di32 * y).astype(np.float32)
    w = sla.solve_triangular(Lm, z, lower=True, trans="T", unit_diagonal=True)
    assert y.dtype == np.float32 and w.dtype == np.float32
    want = x0 + w.astype(np.float64)
    got, _ = P.smooth_stencil_f32(Lw32, Di32, b, x0=x0, nsweeps=1)
    x64, _ = P.smooth_stencil(Lw32.astype(np.float64), Di32.astype(np.float64), b, x0=x0, nsweeps=1)
    scale = np.abs(w).max()
    assert np.abs(got - want).max() <= 8 * 2.0 ** -24 * scale
    assert np.abs(got - x64).max() >= 1e-9 * np.abs(x64).max()
    if start == "zero":
        assert np.array_equal(got.astype(np.float32).astype(np.float64), got)
        assert not np.array_equal(x64.astype(np.float32).astype(np.float64), x64)


# ----------------------------------------------------------------------- surrogates


def test_sample_sets_match_definition():
    level, s = 5, 4
    pts = O.interior_points(level)
    n = 1 << level
    for t in list(range(7)) + [7]:
        d = O.DIRS[t]
        idx = set(O.sample_set(level, t, s).tolist())
        shift = 1 - np.minimum(d, 0)
        for i, p in enumerate(pts):
            q = p + d
            ok = all((p - shift) % s == 0) and all(q >= 1) and q.sum() <= n - 1
            assert (i in idx) == ok
    # the c set is the plain coarse grid 1 + s Z^3 (no shift)
    assert all(((pts[sorted(O.sample_set(level, 7, 2))] - 1) % 2 == 0).ravel())


@pytest.mark.parametrize("level,stride", [(5, 4), (6, 4), (6, 2)])
def test_sample_sets_follow_the_figure(level, stride):
    # Sec. 4.1, the sample-set figure: S_d is a stride-s sub-lattice of the
    # points whose d-neighbour is interior, placed at the first such point
    # (brute force over the lattice, no shift formula): no offset for the
    # centre, an offset from the left (x) for w, from the bottom (z) for be
    n = 1 << level
    pts = O.interior_points(level).astype(np.int64)
    for t in list(range(O.NLOW)) + [O.CENTRE]:
        d = O.DIRS[t]
        q = pts + d
        ok = np.all(q >= 1, axis=1) & (q.sum(axis=1) <= n - 1)
        first = pts[ok].min(axis=0)            # componentwise first point with p + d interior
        assert ok[np.nonzero(np.all(pts == first, axis=1))[0]].all()
        want = np.nonzero(ok & np.all((pts - first) % stride == 0, axis=1))[0]
        got = O.sample_set(level, t, stride)
        assert np.array_equal(np.sort(got), want), O.DIR_NAMES[t]
        if O.DIR_NAMES[t] == "c":
            assert tuple(first) == (1, 1, 1)
        if O.DIR_NAMES[t] == "w":
            assert tuple(first) == (2, 1, 1)
        if O.DIR_NAMES[t] == "be":
            assert tuple(first) == (1, 1, 2)


@pytest.mark.parametrize("level,stride,deg", [(5, 4, 4), (5, 2, 4), (6, 4, 4), (5, 4, 2)])
def test_unisolvence_rule_matches_rank(level, stride, deg):
    pts = O.interior_points(level).astype(float) / (1 << level)
    for t in list(range(7)) + [7]:
        idx = O.sample_set(level, t, stride)
        V = O.legendre_tensor_matrix(pts[idx], deg)
        full = np.linalg.matrix_rank(V) == V.shape[1]
        assert full == (O.sample_side(level, O.DIRS[t], stride) >= 3 * deg)
    # L5, stride 4, degree 4 is rank deficient; the rule falls back to stride 2
    assert O.effective_stride(5, 4, 4) == 2
    assert O.effective_stride(7, 4, 4) == 4


@pytest.mark.parametrize("deg", [(0, 0, 4), (1, 2, 4), (3, 1, 0), (0, 2, 0)])
@pytest.mark.parametrize("level,stride", [(4, 1), (5, 2), (5, 4), (6, 4)])
def test_unisolvence_rule_matches_rank_anisotropic(level, stride, deg):
    # tensor degrees (dg_x, dg_y, dg_z): a lattice simplex of side M is
    # unisolvent exactly when M >= dg_x + dg_y + dg_z (checked by rank)
    pts = O.interior_points(level).astype(float) / (1 << level)
    for t in list(range(7)) + [7]:
        idx = O.sample_set(level, t, stride)
        if len(idx) == 0:
            continue
        V = O.legendre_tensor_matrix(pts[idx], deg)
        full = np.linalg.matrix_rank(V) == V.shape[1]
        assert full == (O.sample_side(level, O.DIRS[t], stride) >= sum(deg))


def test_anisotropic_tensor_polynomials_are_recovered_exactly():
    # samples of a polynomial in P_{1,2,4} (monomials x^i y^j z^k, i <= 1, j <= 2,
    # k <= 4) are reproduced by the fit, and the fit of a lower tensor space
    # (0, 0, 4) cannot reproduce its x-dependence
    level, s = 6, 2
    pts = O.interior_points(level).astype(float) / (1 << level)
    x, y, z = pts.T
    f = 0.3 + x * (1 - y) ** 2 * z ** 4 - 2.0 * y * z ** 3 + 0.5 * x * y
    L = np.tile(f[:, None], (1, 7))
    D = 1.0 / (1.0 + f ** 2)
    c = O.fit_surrogate(level, L, D, (1, 2, 4), s)
    Lw, Dinv = O.eval_surrogate(level, c, (1, 2, 4))
    np.testing.assert_allclose(Lw[:, 0], f, atol=1e-11)
    c0 = O.fit_surrogate(level, L, D, (0, 0, 4), s)
    Lw0, _ = O.eval_surrogate(level, c0, (0, 0, 4))
    assert np.abs(Lw0[:, 0] - f).max() > 1e-2


def test_polynomial_samples_are_recovered_exactly():
    level, deg, s = 6, 3, 2
    pts = O.interior_points(level).astype(float) / (1 << level)
    rng = np.random.default_rng(3)
    coef = rng.normal(size=(8, (deg + 1) ** 3))
    Ltrue = O.monomial_tensor_matrix(pts, deg) @ coef.T
    L = np.ascontiguousarray(Ltrue[:, :7])
    D = 1.0 / Ltrue[:, 7]
    for basis in ("legendre", "monomial"):
        c = O.fit_surrogate(level, L, D, deg, s, basis=basis)
        Lw, Dinv = O.eval_surrogate(level, c, deg, basis=basis)
        np.testing.assert_allclose(Lw, L, atol=1e-9 * np.abs(L).max())
        np.testing.assert_allclose(Dinv, 1.0 / D, atol=1e-9 * np.abs(1 / D).max())


def test_degree_zero_fit_is_sample_mean():
    t, P = _jittered(5, *W.KAPPA_SIN)
    L, U, D = P.ilu0()
    c = O.fit_surrogate(5, L, D, 0, 2)
    for slot in range(7):
        idx = O.sample_set(5, slot, 2)
        assert c[slot, 0] == pytest.approx(L[idx, slot].mean(), rel=1e-12)
    assert c[7, 0] == pytest.approx((1.0 / D[O.sample_set(5, 7, 2)]).mean(), rel=1e-12)


def test_fit_is_basis_independent_and_error_falls_with_degree():
    t, P = _jittered(6, *W.KAPPA_SIN)
    L, U, D = P.ilu0()
    errs = []
    for deg in (0, 1, 2, 3):
        cl = O.fit_surrogate(6, L, D, deg, 4, basis="legendre")
        cm = O.fit_surrogate(6, L, D, deg, 4, basis="monomial")
        Ll, Dl = O.eval_surrogate(6, cl, deg, basis="legendre")
        Lm, Dm = O.eval_surrogate(6, cm, deg, basis="monomial")
        np.testing.assert_allclose(Ll, Lm, atol=1e-9)
        np.testing.assert_allclose(Dl, Dm, rtol=1e-9)
        rel, mx = O.surrogate_error(6, L, D, Ll, Dl)
        errs.append(rel.mean())
    # higher degree, smaller overall error (Sec. 4.2, discrete L2 error study)
    assert errs[-1] < errs[0]


def test_surrogate_error_counts_only_interior_neighbours():
    # a known perturbation on the points whose neighbour p + d is interior gives
    # the closed-form error; perturbing the other points changes nothing
    t, P = _jittered(4, *W.KAPPA_SIN)
    L, U, D = P.ilu0()
    inner = P.col[:, :7] >= 0
    eps = 1e-3
    Lw = L + eps * inner + 7.0 * ~inner
    Dinv = 1.0 / D * (1 + eps)
    rel, mx = O.surrogate_error(4, L, D, Lw, Dinv)
    for d in range(7):
        m = inner[:, d]
        assert rel[d] == pytest.approx(eps * np.sqrt(m.sum()) / np.linalg.norm(L[m, d]), rel=1e-12)
        assert mx[d] == pytest.approx(eps, rel=1e-9)
    assert rel[7] == pytest.approx(eps, rel=1e-12)


# ---------------------------------------------------------- boundary variant V1


@pytest.mark.parametrize("level", [2, 3, 4, 5, 6])
def test_boundary_points_closed_form(level):
    # a stencil neighbour leaves the interior exactly when one of the four
    # barycentric lattice coordinates (x, y, z, n-x-y-z) is 1, so the boundary
    # points number C(n-1,3) - C(n-5,3): O(h^-2), four faces of ~n^2/2 points
    t = W.make_tet(3, level, *W.KAPPA_SIN, jitter=0.15)
    P = O.Problem.from_tet(t)
    n = 1 << level
    pts = O.interior_points(level)
    bary = np.column_stack([pts, n - pts.sum(axis=1)])
    m = P.boundary_points()
    assert np.array_equal(m, bary.min(axis=1) == 1)
    assert m.sum() == comb(n - 1, 3) - (comb(n - 5, 3) if n >= 5 else 0)


def test_v1_with_exact_interior_is_the_ilu_smoother():
    # V1 takes the exact factors at the boundary points: with the exact factors
    # everywhere else and arbitrary values at the boundary points as the
    # surrogate, its sweeps are the ILU(0) smoother of the matrix form, while
    # the same weights without the replacement (V2) are far off.  Leaving any
    # boundary weight (L or 1/D) unreplaced fails the first check.
    t, P = _jittered(5, *W.KAPPA_EXP)
    L, U, D = P.ilu0()
    m = P.boundary_points()
    rng = np.random.default_rng(5)
    Lg = L.copy()
    Lg[m] = rng.uniform(-0.5, 0.0, (m.sum(), 7))
    Dg = 1.0 / D
    Dg[m] = rng.uniform(0.5, 2.0, m.sum()) * Dg[m]
    Lw1, Dinv1 = P.v1_weights(Lg, Dg, L, D)
    b = t.rhs()
    x, r = P.smooth(L, D, b, nsweeps=3)
    x1, r1 = P.smooth_stencil(Lw1, Dinv1, b, nsweeps=3)
    np.testing.assert_allclose(x1, x, rtol=0, atol=1e-13 * np.abs(x).max())
    x2, _ = P.smooth_stencil(Lg, Dg, b, nsweeps=3)
    assert np.abs(x2 - x).max() > 1e-2 * np.abs(x).max()


# ---------------------------------------------------------------- contraction


def _dense_lower(P, L):
    Lm, _ = _factor_matrices(P, L, np.ones(P.N))
    return Lm.toarray()


def test_contraction_factor_is_spectral_radius_of_ilu_smoother():
    # power iteration on I - C^{-1} A with C = L D L^T from ILU(0) converges to
    # its spectral radius, computed here by a dense eigen-solver
    t, P = _jittered(3, *W.KAPPA_SIN, seed=7)
    L, U, D = P.ilu0()
    Lm = _dense_lower(P, L)
    C = Lm @ np.diag(D) @ Lm.T
    E = np.eye(P.N) - np.linalg.solve(C, P.csr().toarray())
    radius = np.abs(np.linalg.eigvals(E)).max()
    zero = np.zeros(P.N)
    x0 = W.SplitMix64(11).uniform_array(P.N, -1.0, 1.0)
    rho, rho_res = O.contraction_factor(P, lambda y: P.smooth_stencil(L, 1.0 / D, zero, y, 1)[0], x0, 100)
    assert rho == pytest.approx(radius, rel=1e-10)
    assert 0.9 * radius < rho_res <= radius * (1 + 1e-9)
    assert 0.0 < radius < 0.2


def test_contraction_factor_of_damped_jacobi_and_exact_solve():
    t, P = _jittered(3, *W.KAPPA_SIN, seed=7)
    A = P.csr().toarray()
    zero = np.zeros(P.N)
    x0 = W.SplitMix64(11).uniform_array(P.N, -1.0, 1.0)
    # L = 0: the sweep is a Jacobi step; halve it for a unique dominant eigenvalue
    dinv = 1.0 / P.A[:, 7]
    jac = lambda y: y + 0.5 * (P.smooth_stencil(np.zeros((P.N, 7)), dinv, zero, y, 1)[0] - y)
    radius = np.abs(np.linalg.eigvals(np.eye(P.N) - 0.5 * dinv[:, None] * A)).max()
    rho, _ = O.contraction_factor(P, jac, x0, 200)
    assert rho == pytest.approx(radius, rel=1e-8)
    # an exact solve removes the error in one step
    rho, _ = O.contraction_factor(P, lambda y: y - np.linalg.solve(A, A @ y), x0, 1)
    assert rho < 1e-13


# ---------------------------------------------------------- PCG and the SGS comparator


def test_sgs_factors_define_symmetric_gauss_seidel():
    # L D L^T built from the stencil factors equals (D_A + L_A) D_A^-1 (D_A + L_A)^T
    # built from the assembled matrix (Sec. 2.1)
    t, P = _jittered(4, *W.KAPPA_EXP)
    L, D = P.sgs_factors()
    Lm, Dm = _factor_matrices(P, L, D)
    C = (Lm @ Dm @ Lm.T).toarray()
    A = P.csr().toarray()
    DL = np.tril(A)
    C2 = DL @ np.diag(1.0 / np.diag(A)) @ DL.T
    np.testing.assert_allclose(C, C2, rtol=0, atol=1e-13 * np.abs(A).max())


@pytest.mark.parametrize("which", ["ilu", "sgs", "ilu_f32"])
def test_pcg_matches_scipy_cg(which):
    # same preconditioner handed to scipy's CG: equal iteration counts and iterates
    import scipy.sparse.linalg as sla
    t, P = _jittered(4, *W.KAPPA_SIN, seed=7)
    if which == "sgs":
        L, D = P.sgs_factors()
    else:
        L, U, D = P.ilu0()
    M = P.precond(L, 1.0 / D, f32=which == "ilu_f32")
    b = t.rhs()
    x, k, hist, ok = O.pcg(P, M, b, maxit=300, rel_tol=1e-10)
    assert ok and hist[-1] <= 1e-10 * np.linalg.norm(b) < hist[-2]
    count = [0]

    def cb(_):
        count[0] += 1
    A = P.csr()
    xs, info = sla.cg(A, b, rtol=1e-10, atol=0.0, maxiter=300, M=sla.LinearOperator(A.shape, matvec=M), callback=cb)
    assert info == 0 and count[0] == k
    np.testing.assert_allclose(x, xs, rtol=0, atol=1e-12 * np.abs(x).max())


def test_pcg_special_cases():
    t, P = _jittered(3, *W.KAPPA_SIN, seed=7)
    A = P.csr().toarray()
    b = t.rhs()
    # the exact inverse as preconditioner: one iteration
    x, k, _, ok = O.pcg(P, lambda r: np.linalg.solve(A, r), b, maxit=5, rel_tol=1e-12)
    assert ok and k == 1
    np.testing.assert_allclose(A @ x, b, atol=1e-12)
    # plain CG on N unknowns terminates after at most N steps (exact arithmetic; a
    # few more with rounding)
    x, k, _, ok = O.pcg(P, lambda r: r.copy(), b, maxit=10 * P.N, rel_tol=1e-10)
    assert ok and k <= P.N + 3
    # b = 0 from x = 0: nothing to do
    x, k, _, ok = O.pcg(P, lambda r: r.copy(), np.zeros(P.N), maxit=5, rel_tol=1e-10)
    assert ok and k == 0 and not x.any()


def test_ilu_preconditioner_beats_sgs_and_plain_cg():
    # the ordering reported with the CG experiment of Sec. 4.2: the ILU
    # preconditioner needs fewer CG iterations than symmetric Gauss-Seidel
    t, P = _jittered(5, *W.KAPPA_SIN, seed=7)
    b = t.rhs()
    L, U, D = P.ilu0()
    Ls, Ds = P.sgs_factors()
    k_ilu = O.pcg(P, P.precond(L, 1.0 / D), b, maxit=500, rel_tol=1e-8)[1]
    k_sgs = O.pcg(P, P.precond(Ls, 1.0 / Ds), b, maxit=500, rel_tol=1e-8)[1]
    k_cg = O.pcg(P, lambda r: r.copy(), b, maxit=500, rel_tol=1e-8)[1]
    assert k_ilu < k_sgs < k_cg


# ------------------------------------------------------------------ LFA (Sec. 3)


def _stencil_product(L, D):
    """Offsets and values of L D L^T for constant stencils (L_c = 1)."""
    low = [tuple(O.DIRS[d]) for d in range(7)] + [(0, 0, 0)]
    val = list(L) + [1.0]
    out = {}
    for a, la in zip(low, val):
        for b, lb in zip(low, val):
            off = tuple(np.subtract(a, b))
            out[off] = out.get(off, 0.0) + la * D * lb
    return out


def test_asymptotic_stencil_reproduces_A_on_the_pattern():
    # the fixed point of the stencil equations: (L D L^T)_d = A_d on the 15
    # pattern offsets, plus exactly 12 fill-in offsets (Sec. 3)
    t = W.make_tet(21, 4, W.COEFF_CONST, (1.0,), jitter=0.15)
    A = O.constant_stencil(t.verts)
    L, D = O.asymptotic_stencil(A)
    prod = _stencil_product(L, D)
    for d in range(15):
        assert prod.pop(tuple(O.DIRS[d])) == pytest.approx(A[d], abs=1e-12 * np.abs(A).max())
    assert len([v for v in prod.values() if abs(v) > 1e-14]) == 12
    # so the LFA error symbol D |L|^2 - A is the symbol of the fill-in alone
    th = np.random.default_rng(3).uniform(-np.pi, np.pi, (50, 3))
    Ls = 1 + sum(L[d] * np.exp(1j * th @ O.DIRS[d]) for d in range(7))
    As = sum(A[d] * np.exp(1j * th @ O.DIRS[d]) for d in range(15))
    fill = sum(v * np.exp(1j * th @ np.array(off)) for off, v in prod.items())
    np.testing.assert_allclose(D * np.abs(Ls) ** 2 - As, fill, atol=1e-12 * np.abs(A).max())


def test_smoothing_factor_is_invariant_under_similarity():
    # mu depends on the shape and vertex order only: translation, uniform
    # scaling and rotation leave it unchanged
    v = np.array(W.make_tet(22, 4, W.COEFF_CONST, (1.0,), jitter=0.15).verts)
    mu, best = O.lfa_orientation(v)
    c, s = np.cos(0.7), np.sin(0.7)
    R = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]]) @ np.array([[1, 0, 0], [0, c, s], [0, -s, c]])
    mu2, best2 = O.lfa_orientation(3.5 * v @ R.T + np.array([1.0, -2.0, 0.5]))
    np.testing.assert_allclose(mu2, mu, rtol=1e-9)
    assert best2 == best and 0.0 < mu[best] < 1.0
    # a finer frequency grid moves the sampled supremum only a little
    th = O.lfa_frequencies(48)
    A = O.constant_stencil(O.permute_vertices(v, O.permutations()[best]))
    L, D = O.asymptotic_stencil(A)
    assert abs(O.smoothing_factor(A, L, D, th) - mu[best]) < 0.05


def test_lfa_orientation_matches_printed_choices():
    # Cap and Spade (Table SM1): among the permutations the paper lists, the
    # smallest smoothing factor is at the one its heuristic selected (bold).
    # Spindle: the LFA prefers (1 4 2 3), which the paper's multigrid rates
    # also favour (0.35 vs 0.39 for its bold (1 3 2 4)); recorded, not asserted.
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "orientation_shapes.json")))
    perms = ["".join(map(str, p)) for p in O.permutations()]
    for name in ("Cap", "Spade"):
        sh = g["shapes"][name]
        mu, best = O.lfa_orientation(sh["vertices"])
        listed = {p: mu[perms.index(p)] for p in sh["rho_ilu"]}
        assert min(listed, key=listed.get) == sh["bold"], (name, listed)
        # and the best listed permutation also has the best printed rate
        assert min(sh["rho_ilu"], key=sh["rho_ilu"].get) == sh["bold"]
    sh = g["shapes"]["Spindle"]
    mu, best = O.lfa_orientation(sh["vertices"])
    listed = {p: mu[perms.index(p)] for p in sh["rho_ilu"]}
    assert min(listed, key=listed.get) == min(sh["rho_ilu"], key=sh["rho_ilu"].get) == "1423"


def test_z_only_surrogate_on_a_flat_tetrahedron():
    # distorted tetrahedron of height 0.1 with a unit coefficient (Sec. 4.2):
    # the factors vary mainly along z, so dg_x = dg_y = 0 with a high dg_z
    # comes close to the exact ILU's contraction, while a low dg_z does not
    wl = W.workload("flat_L8_const")
    t = wl.tets[0]
    t5 = W.Tet(t.verts, 5, t.coeff_kind, t.coeff_params, t.rhs_state)
    P = O.Problem.from_tet(t5)
    L, U, D = P.ilu0()
    z = np.zeros(P.N)
    x0 = W.SplitMix64(1).uniform_array(P.N, -1.0, 1.0)
    rho_exact = O.contraction_factor(P, lambda y: P.smooth_stencil(L, 1.0 / D, z, y, 1)[0], x0, 20)[0]
    rho = {}
    for deg in ((0, 0, 6), (0, 0, 3)):
        c = O.fit_surrogate(5, L, D, deg, O.effective_stride(5, deg, 4))
        Lw, Dinv = O.eval_surrogate(5, c, deg)
        rho[deg] = O.contraction_factor(P, lambda y: P.smooth_stencil(Lw, Dinv, z, y, 1)[0], x0, 20)[0]
    assert rho[(0, 0, 6)] < 1.25 * rho_exact < rho[(0, 0, 3)]


# --------------------------------------------------------- surrogate operator


@pytest.mark.parametrize("coeff,deg", [((W.COEFF_CONST, (1.0,)), 0), ((W.COEFF_POLY, (1.0, 10.0, 2.0, 0.0)), 2)])
def test_operator_surrogate_is_exact_for_polynomial_stencils(coeff, deg):
    # kappa = 1 (constant stencil) and kappa = 1 + 10 (x^2 + y^2 + z^2) (the
    # paper's kappa_2) on an affine tetrahedron give stencil entries that are
    # polynomials of degree deg in the lattice point, so the fit reproduces A
    # on the pattern and smoothing with the surrogate operator equals smoothing
    # with A
    t = W.make_tet(23, 5, coeff[0], coeff[1], jitter=0.15)
    P = O.Problem.from_tet(t)
    s = O.effective_stride(5, deg, 4)
    c = O.fit_operator_surrogate(5, P.A, deg, s)
    At = O.eval_operator_surrogate(5, c, deg)
    m = P.col >= 0
    assert np.abs(At[m] - P.A[m]).max() <= 1e-9 * np.abs(P.A).max()
    L, U, D = P.ilu0()
    b = t.rhs()
    x1, _ = P.smooth_stencil(L, 1.0 / D, b, nsweeps=3)
    x2, _ = P.smooth_stencil(L, 1.0 / D, b, nsweeps=3, A=At)
    np.testing.assert_allclose(x2, x1, rtol=0, atol=1e-8 * np.abs(x1).max())


def test_operator_surrogate_is_symmetric_and_close():
    # variable coefficient: the surrogate is symmetric by construction
    # (upper weights are the lower polynomials at p - d), its full rows sum to
    # zero like A's (the centre is minus the neighbour weights), and it is
    # within the fit error of A
    t = W.make_tet(24, 5, *W.KAPPA_EXP, jitter=0.15)
    P = O.Problem.from_tet(t)
    c = O.fit_operator_surrogate(5, P.A, 3, O.effective_stride(5, 3, 4))
    At = O.eval_operator_surrogate(5, c, 3)
    m = P.col >= 0
    for s in range(7):
        j = P.col[:, 8 + s]
        ok = j >= 0
        np.testing.assert_allclose(At[ok, 8 + s], At[j[ok], s], rtol=0, atol=1e-12 * np.abs(P.A).max())
    np.testing.assert_allclose(At.sum(axis=1), 0.0, atol=1e-12 * np.abs(P.A).max())
    # the discrete L2 error of the fitted entries falls with the degree
    errs = []
    for deg in (1, 4):
        c = O.fit_operator_surrogate(5, P.A, deg, O.effective_stride(5, deg, 4))
        At = O.eval_operator_surrogate(5, c, deg)
        errs.append(np.linalg.norm(At[m] - P.A[m]) / np.linalg.norm(P.A[m]))
    assert 1e-8 < errs[1] < errs[0]


def test_operator_surrogate_keeps_the_smoother_contracting():
    # with the centre from the row sums, the surrogate operator at a
    # sufficient degree leaves the smoother's contraction that of A
    t = W.make_tet(5, 6, *W.KAPPA_EXP, jitter=0.15)
    P = O.Problem.from_tet(t)
    L, U, D = P.ilu0()
    deg = 6
    s = O.effective_stride(6, deg, 4)
    Lw, Dinv = O.eval_surrogate(6, O.fit_surrogate(6, L, D, deg, s), deg)
    At = O.eval_operator_surrogate(6, O.fit_operator_surrogate(6, P.A, deg, s), deg)
    z = np.zeros(P.N)
    x0 = W.SplitMix64(1).uniform_array(P.N, -1.0, 1.0)
    rho_a = O.contraction_factor(P, lambda y: P.smooth_stencil(Lw, Dinv, z, y, 1)[0], x0, 40)[0]
    rho_s = O.contraction_factor(P, lambda y: P.smooth_stencil(Lw, Dinv, z, y, 1, A=At)[0], x0, 40)[0]
    assert rho_s == pytest.approx(rho_a, rel=1e-3) and rho_s < 1.0
