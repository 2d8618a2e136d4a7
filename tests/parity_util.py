"""Comparison helpers shared by the GPU parity tests (test infrastructure)."""
import numpy as np


def rel(a, b):
    """Largest difference relative to the largest entry of b."""
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def colrel(a, b):
    """Largest difference per column relative to that column's largest entry
    (the weights of different stencil directions differ by orders of
    magnitude), maximised over the columns."""
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return max(np.abs(a[:, k] - b[:, k]).max() / max(np.abs(b[:, k]).max(), 1e-300) for k in range(a.shape[1]))


def f64_sweep_parity(P, xg, weights_gpu, weights_oracle, b, nsweeps, x0=None, A=None):
    """FP64 surrogate sweeps against the oracle's Alg. 2, two ways:
    * with the weights the kernels use on both sides, only the order of the
      sums differs: 1e-12, the stored-factor bar;
    * with the oracle's own evaluation of the same polynomials, the iterates
      may differ by no more than the weights do (per direction).
    Returns (difference with the kernel's weights, with the oracle's, weight
    difference)."""
    Lg, Dg = weights_gpu
    Lw, Dinv = weights_oracle
    own, _ = P.smooth_stencil(Lg, Dg, b, x0=x0, nsweeps=nsweeps, A=A)
    want, _ = P.smooth_stencil(Lw, Dinv, b, x0=x0, nsweeps=nsweeps, A=A)
    e_own, e_or = rel(xg, own), rel(xg, want)
    ew = colrel(np.column_stack([Lg, Dg]), np.column_stack([Lw, Dinv]))
    assert e_own < 1e-12, e_own
    assert e_or <= max(1e-12, ew), (e_or, ew)
    return e_own, e_or, ew
