"""GPU parity of the surrogate operator (ILU_A_SURROGATE; Sec. 4.2
approximates A by surrogate polynomials too), through the C-ABI.

With the oracle's coefficients injected, both sides evaluate the same
polynomials: FP64 tables agree to rounding (1e-12 on A x, 1e-11 after
smoothing), FP32 tables to FP32 resolution of the weights (1e-6 on A x)."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from parity_util import f64_sweep_parity

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


def _case(level=6, deg=3, coeff=W.KAPPA_EXP, seed=25):
    t = W.make_tet(seed, level, *coeff, jitter=0.15)
    P = O.Problem.from_tet(t)
    L, U, D = P.ilu0()
    s = O.effective_stride(level, deg, 4)
    c = O.fit_surrogate(level, L, D, deg, s)
    ca = O.fit_operator_surrogate(level, P.A, deg, s)
    return t, P, c, ca


@pytest.mark.parametrize("variant", ["surr_f64", "surr_f32"])
def test_operator_fit_and_apply_parity(torch, pkg, variant):
    level, deg = 6, 3
    t, P, c, ca = _case(level, deg)
    v = pkg.SURR_F32 if variant == "surr_f32" else pkg.SURR_F64
    sm = pkg.Smoother([t], v, degree=deg, stride=4, tile=(8, 8), a_mode=pkg.A_SURROGATE)
    # the GPU fit evaluates like the oracle's (TSQR vs pivoted QR: 1e-7)
    got = O.eval_operator_surrogate(level, sm.surrogate_a(0), deg)
    want = O.eval_operator_surrogate(level, ca, deg)
    m = P.col >= 0
    assert _rel(got[m], want[m]) < 1e-7
    # y = A~ x with the oracle's coefficients
    sm.set_surrogate_a(0, ca)
    x = np.random.default_rng(5).uniform(-1, 1, P.N)
    y = sm.apply(torch.tensor(x, device="cuda")).cpu().numpy()
    assert _rel(y, P.apply(x, A=want)) < (1e-6 if variant == "surr_f32" else 1e-12)


@pytest.mark.parametrize("variant", ["surr_f64", "surr_f32"])
def test_operator_surrogate_smoothing_parity(torch, pkg, variant):
    level, deg = 6, 3
    t, P, c, ca = _case(level, deg)
    f32 = variant == "surr_f32"
    sm = pkg.Smoother([t], pkg.SURR_F32 if f32 else pkg.SURR_F64, degree=deg, stride=4, tile=(16, 16),
                      a_mode=pkg.A_SURROGATE)
    sm.set_surrogate(0, c)
    sm.set_surrogate_a(0, ca)
    Lw, Dinv = O.eval_surrogate(level, c, deg)
    At = O.eval_operator_surrogate(level, ca, deg)
    b = t.rhs()
    x = torch.zeros(P.N, dtype=torch.float64, device="cuda")
    sm.smooth(x, torch.tensor(b, device="cuda"), 6)
    if f32:
        want, _ = P.smooth_stencil_f32(Lw.astype(np.float32), Dinv.astype(np.float32), b, nsweeps=6, A=At)
        assert _rel(x.cpu().numpy(), want) < 2e-5
    else:
        wg = tuple(a.cpu().numpy() for a in sm.surrogate_values(0))
        f64_sweep_parity(P, x.cpu().numpy(), wg, (Lw, Dinv), b, 6, A=At)


def test_operator_surrogate_exact_for_polynomial_coefficient(torch, pkg):
    # kappa_2 = 1 + 10 (x^2 + y^2 + z^2): stencil entries are degree-2
    # polynomials of the lattice point, so the degree-2 surrogate operator is A
    t = W.make_tet(26, 6, W.COEFF_POLY, (1.0, 10.0, 2.0, 0.0), jitter=0.15)
    exact = pkg.Smoother([t], pkg.SURR_F64, degree=2, stride=4, tile=(8, 8))
    sur = pkg.Smoother([t], pkg.SURR_F64, degree=2, stride=4, tile=(8, 8), a_mode=pkg.A_SURROGATE)
    x = torch.tensor(np.random.default_rng(6).uniform(-1, 1, exact.n_total), device="cuda")
    assert _rel(sur.apply(x).cpu().numpy(), exact.apply(x).cpu().numpy()) < 1e-9


def test_operator_surrogate_refinement_and_graph_rebuild(torch, pkg):
    # refinement converges for the surrogate operator; replacing the
    # coefficients after a graph replay rebuilds the tables and the graph
    level, deg = 5, 3
    t, P, c, ca = _case(level, deg, coeff=W.KAPPA_SIN, seed=27)
    b = torch.tensor(t.rhs(), device="cuda")
    # FP64 tables: the oracle's A~ from the same coefficients is the operator the
    # GPU refined against (FP32 tables would differ from it by FP32 rounding)
    sm = pkg.Smoother([t], pkg.SURR_F64, degree=deg, stride=4, tile=(8, 8), a_mode=pkg.A_SURROGATE)
    x = torch.zeros_like(b)
    rel, ok = sm.smooth(x, b, 600, rel_tol=1e-10)
    assert ok and rel <= 1e-10
    At = O.eval_operator_surrogate(level, sm.surrogate_a(0), deg)
    xs = x.cpu().numpy()
    assert np.linalg.norm(t.rhs() - P.apply(xs, A=At)) <= 1.01e-10 * np.linalg.norm(t.rhs())
    sm = pkg.Smoother([t], pkg.SURR_F32, degree=deg, stride=4, tile=(8, 8), a_mode=pkg.A_SURROGATE)
    x.zero_()
    sm.smooth(x, b, 3)                      # captures and replays the sweep graph
    sm.set_surrogate(0, c)
    sm.set_surrogate_a(0, ca)
    x.zero_()
    sm.smooth(x, b, 3)
    fresh = pkg.Smoother([t], pkg.SURR_F32, degree=deg, stride=4, tile=(8, 8), a_mode=pkg.A_SURROGATE)
    fresh.set_surrogate(0, c)
    fresh.set_surrogate_a(0, ca)
    x2 = torch.zeros_like(b)
    fresh.smooth(x2, b, 3)
    assert np.array_equal(x.cpu().numpy(), x2.cpu().numpy())
