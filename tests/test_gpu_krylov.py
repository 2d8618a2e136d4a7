"""GPU parity of the pieces around the smoother, through the C-ABI: the
symmetric Gauss-Seidel comparator, preconditioned CG (ILU as preconditioner,
Sec. 4.2) and the contraction factor, each against the CPU oracle.

Tolerances: FP64 variants take the same decisions as the oracle, so CG runs
the same number of iterations and the iterates differ by rounding amplified
over the iterations (1e-9 relative); the FP32 preconditioner perturbs each
application by a few FP32 ulps, so its iteration count may differ by one."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    return _t


@pytest.fixture(scope="module")
def pkg():
    import paper_2210_15280_amd as P
    P.lib()
    return P


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _dev(torch, a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _setup(pkg, P, t, variant, level, deg=3, **kw):
    """Smoother on the GPU and the matching oracle weights (surrogates: the
    oracle's coefficients are injected, so both sides use the same C)."""
    if variant in ("stored", "sgs"):
        L, D = P.sgs_factors() if variant == "sgs" else P.ilu0()[::2]
        sm = pkg.Smoother([t], pkg.STORED_SGS if variant == "sgs" else pkg.STORED_F64, **kw)
        return sm, L, 1.0 / D, False
    L, U, D = P.ilu0()
    s = O.effective_stride(level, deg, 4)
    c = O.fit_surrogate(level, L, D, deg, s)
    Lw, Dinv = O.eval_surrogate(level, c, deg)
    f32 = variant == "surr_f32"
    sm = pkg.Smoother([t], pkg.SURR_F32 if f32 else pkg.SURR_F64, degree=deg, stride=4, **kw)
    sm.set_surrogate(0, c)
    return sm, Lw, Dinv, f32


@pytest.mark.parametrize("level", [4, 6])
def test_sgs_factor_and_sweep_parity(torch, pkg, level):
    t = W.make_tet(3, level, *W.KAPPA_EXP, jitter=0.15)
    P = O.Problem.from_tet(t)
    L, D = P.sgs_factors()
    sm = pkg.Smoother([t], pkg.STORED_SGS, tile=(8, 8))
    Lg, Dg = sm.factors(0)
    assert _rel(Lg.cpu().numpy(), L) < 1e-13
    assert _rel(Dg.cpu().numpy(), D) < 1e-13
    b = t.rhs()
    x = torch.zeros(P.N, dtype=torch.float64, device="cuda")
    sm.smooth(x, _dev(torch, b), 5)
    want, _ = P.smooth_stencil(L, 1.0 / D, b, nsweeps=5)
    assert _rel(x.cpu().numpy(), want) < 1e-12


@pytest.mark.parametrize("variant", ["stored", "sgs", "surr_f64", "surr_f32"])
@pytest.mark.parametrize("level,tile", [(5, (8, 8)), (6, (16, 16))])
def test_pcg_parity(torch, pkg, variant, level, tile):
    t = W.make_tet(11, level, *W.KAPPA_SIN, jitter=0.15)
    P = O.Problem.from_tet(t)
    sm, Lw, Dinv, f32 = _setup(pkg, P, t, variant, level, tile=tile)
    b = t.rhs()
    want, k_or, hist, ok_or = O.pcg(P, P.precond(Lw, Dinv, f32), b, maxit=400, rel_tol=1e-9)
    assert ok_or
    x = torch.zeros(P.N, dtype=torch.float64, device="cuda")
    k, res, ok = sm.pcg(x, _dev(torch, b), 400, rel_tol=1e-9)
    assert ok
    xg = x.cpu().numpy()
    true_res = np.linalg.norm(b - P.apply(xg))
    assert res == pytest.approx(true_res, rel=1e-6, abs=1e-14)
    if f32:
        # both iterates meet the tolerance; they differ by at most cond(A) times it
        assert abs(k - k_or) <= 1
        assert true_res <= 1.05e-9 * np.linalg.norm(b)
        assert _rel(xg, want) < 1e-5
    else:
        assert k == k_or
        assert _rel(xg, want) < 1e-9


def test_pcg_graph_replay_equals_eager(torch, pkg):
    t = W.make_tet(12, 5, *W.KAPPA_EXP, jitter=0.15)
    b = _dev(torch, t.rhs())
    out = []
    for graph in (True, False):
        sm = pkg.Smoother([t], pkg.SURR_F32, degree=3, stride=4, tile=(8, 8))
        sm.set_graph(graph)
        x = torch.zeros_like(b)
        k, res, ok = sm.pcg(x, b, 300, rel_tol=1e-10)
        assert ok
        # a second call on the same handle (graph already captured) from a new start
        x2 = torch.ones_like(b)
        k2, res2, ok2 = sm.pcg(x2, b, 300, rel_tol=1e-10)
        assert ok2
        out.append((k, x.cpu().numpy(), k2, x2.cpu().numpy()))
    assert out[0][0] == out[1][0] and out[0][2] == out[1][2]
    assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[0][3], out[1][3])


def test_pcg_edge_cases(torch, pkg):
    t = W.make_tet(13, 4, *W.KAPPA_SIN, jitter=0.15)
    P = O.Problem.from_tet(t)
    L, U, D = P.ilu0()
    sm = pkg.Smoother([t], pkg.STORED_F64, tile=(8, 8))
    # b = 0 from x = 0: converged before the first iteration, x untouched
    x = torch.zeros(P.N, dtype=torch.float64, device="cuda")
    k, res, ok = sm.pcg(x, torch.zeros_like(x), 50, rel_tol=1e-10)
    assert ok and k == 0 and res == 0.0 and not x.any()
    # an iteration cap below the need: not converged, and the iterate is the
    # oracle's after exactly that many iterations
    b = t.rhs()
    want, k_or, _, ok_or = O.pcg(P, P.precond(L, 1.0 / D), b, maxit=3, rel_tol=1e-14)
    assert not ok_or and k_or == 3
    k, res, ok = sm.pcg(x, _dev(torch, b), 3, rel_tol=1e-14)
    assert not ok and k == 3
    assert _rel(x.cpu().numpy(), want) < 1e-11
    # absolute tolerance (the criterion of the CG experiment): ||r|| <= 1e-3
    x.zero_()
    want, k_or, hist, _ = O.pcg(P, P.precond(L, 1.0 / D), b, maxit=100, abs_tol=1e-3)
    k, res, ok = sm.pcg(x, _dev(torch, b), 100, abs_tol=1e-3)
    assert ok and k == k_or and hist[-1] <= 1e-3


class _Batch:
    """Block-diagonal operator of several oracle problems (test helper)."""

    def __init__(self, probs):
        self.probs = probs
        self.cuts = np.cumsum([0] + [p.N for p in probs])

    def apply(self, x):
        return np.concatenate([p.apply(x[a:b]) for p, a, b in zip(self.probs, self.cuts[:-1], self.cuts[1:])])

    def precond(self, parts):
        return lambda r: np.concatenate([m(r[a:b]) for m, a, b in zip(parts, self.cuts[:-1], self.cuts[1:])])


def test_pcg_batch_is_one_block_diagonal_system(torch, pkg):
    tets = W.batch_tets(21, 5, (3, 4, 5))
    probs = [O.Problem.from_tet(t) for t in tets]
    B = _Batch(probs)
    precs = []
    for P in probs:
        L, U, D = P.ilu0()
        precs.append(P.precond(L, 1.0 / D))
    b = np.concatenate([t.rhs() for t in tets])
    want, k_or, _, ok_or = O.pcg(B, B.precond(precs), b, maxit=300, rel_tol=1e-10)
    assert ok_or
    sm = pkg.Smoother(tets, pkg.STORED_F64, tile=(8, 8))
    x = torch.zeros(len(b), dtype=torch.float64, device="cuda")
    k, res, ok = sm.pcg(x, _dev(torch, b), 300, rel_tol=1e-10)
    assert ok and k == k_or
    assert _rel(x.cpu().numpy(), want) < 1e-9


@pytest.mark.parametrize("variant", ["stored", "sgs", "surr_f64", "surr_f32"])
def test_contraction_factor_parity(torch, pkg, variant):
    level = 5
    t = W.make_tet(14, level, *W.KAPPA_SIN, jitter=0.15)
    P = O.Problem.from_tet(t)
    sm, Lw, Dinv, f32 = _setup(pkg, P, t, variant, level, tile=(8, 8))
    x0 = W.SplitMix64(99).uniform_array(P.N, -1.0, 1.0)
    zero = np.zeros(P.N)
    if f32:
        L32, D32 = Lw.astype(np.float32), Dinv.astype(np.float32)
        step = lambda y: P.smooth_stencil_f32(L32, D32, zero, y, 1)[0]  # noqa: E731
    else:
        step = lambda y: P.smooth_stencil(Lw, Dinv, zero, y, 1)[0]  # noqa: E731
    rho_or, rr_or = O.contraction_factor(P, step, x0, 20)
    x = _dev(torch, x0)
    rho, rr = sm.contraction(x, 20)
    tol = 1e-5 if f32 else 1e-10
    assert rho == pytest.approx(rho_or, rel=tol)
    assert rr == pytest.approx(rr_or, rel=tol)
    assert abs(np.linalg.norm(x.cpu().numpy()) - 1.0) < 1e-12
    assert 0.0 < rho < 1.0


@pytest.mark.parametrize("variant", ["surr_f64", "surr_f32"])
def test_surrogate_error_parity(torch, pkg, variant):
    # per-direction surrogate error (relative discrete L2 and max-abs against
    # the exact ILU, over the points whose neighbour is interior) from the GPU's
    # exact factors and surrogate weights vs the oracle's.  The oracle's
    # coefficients are injected (the fit itself is compared in the sweep parity
    # tests), so the FP64 weights agree to rounding and the FP32 ones to FP32
    # resolution, far below the errors measured (1e-4 and above).
    level, deg = 6, 3
    t = W.make_tet(15, level, *W.KAPPA_EXP, jitter=0.15)
    P = O.Problem.from_tet(t)
    L, U, D = P.ilu0()
    c = O.fit_surrogate(level, L, D, deg, O.effective_stride(level, deg, 4))
    rel_or, mx_or = O.surrogate_error(level, L, D, *O.eval_surrogate(level, c, deg))
    assert rel_or.min() > 1e-4
    st = pkg.Smoother([t], pkg.STORED_F64, tile=(8, 8))
    su = pkg.Smoother([t], pkg.SURR_F32 if variant == "surr_f32" else pkg.SURR_F64, degree=deg, stride=4,
                      tile=(8, 8))
    su.set_surrogate(0, c)
    Lg, Dg = (a.cpu().numpy() for a in st.factors(0))
    Ls, Ds = (a.cpu().numpy() for a in su.surrogate_values(0))
    rel, mx = O.surrogate_error(level, Lg, Dg, Ls, Ds)
    tol = 1e-3 if variant == "surr_f32" else 1e-8
    np.testing.assert_allclose(rel, rel_or, rtol=tol)
    np.testing.assert_allclose(mx, mx_or, rtol=10 * tol)
