"""GPU parity at the surrogate degrees the workloads use, and of the persistent
sweep when its workgroups take several blocks each.

* Degree 4 (the level-7 and level-8 workloads and the batch: five Horner
  coefficients per row and direction) on the level-7 workload itself, and
  degree 6 (the level-9 workload: seven coefficients) on a level-7 lattice of
  the level-9 workload's geometry and coefficient.
* The least-squares fit (Sec. 4.1) at these degrees is ill-conditioned: the
  shifted Legendre tensor basis, orthogonal on the cube, is nearly dependent
  on the simplex (condition 2e8 at degree 4, 1e13 at degree 6 on level 7).
  So the coefficients, and the surrogate values away from the samples, are
  fixed only to that conditioning: backward-stable FP64 solvers (pivoted QR,
  plain QR, SVD, TSQR) disagree by up to 1e-2 of the values at degree 6.
  What is unique is the minimal residual on each sample set and the fitted
  values on the samples; the GPU fit must reach both, and its other values
  must lie within the first-order perturbation bound of least squares.
* The fitted coefficients are large and cancel (up to 1e7 at degree 6 for
  weights of size 1e-2 .. 1), so evaluating the polynomial in FP64 in any
  order carries a rounding error of a few units of 2^-53 times
  S(p) = sum_k |c_k Phi_k(p)|, up to 1e10 times the value.  The tables are
  checked against that a priori bound: the handle's own coefficients,
  evaluated by the oracle, against the values the sweeps use.
* The sweeps are pinned with the weights they use on both sides (FP64:
  1e-12, the stored-factor bar), and with the oracle's own evaluation of the
  same coefficients the iterates may differ by no more than the weights do.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

LEVEL = 7
TILES = [(8, 8), (16, 16), (16, 32)]
# FP32 unit roundoff
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    return _t


@pytest.fixture(scope="module")
def pkg():
    import paper_2210_15280_amd as P
    P.lib()
    return P


def _tet(deg):
    if deg == 4:
        return W.workload("jit_L7_sin").tets[0]
    return W.make_tet(5, LEVEL, *W.KAPPA_EXP, jitter=0.15)  # level-9 workload's geometry and coefficient


_CACHE = {}


def _case(deg):
    """Oracle side of one degree: problem, exact factors, fit and its values."""
    if deg not in _CACHE:
        t = _tet(deg)
        P = O.Problem.from_tet(t)
        L, U, D = P.ilu0()
        s = O.effective_stride(LEVEL, deg, 4)
        c = O.fit_surrogate(LEVEL, L, D, deg, s)
        Lw, Dinv = O.eval_surrogate(LEVEL, c, deg)
        _CACHE[deg] = dict(t=t, P=P, L=L, D=D, s=s, c=c, Lw=Lw, Dinv=Dinv)
    return _CACHE[deg]


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _colrel(a, b):
    # worst relative difference per direction (columns scaled separately:
    # the weights of different directions differ by orders of magnitude)
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    return max(np.abs(a[:, k] - b[:, k]).max() / max(np.abs(b[:, k]).max(), 1e-300) for k in range(a.shape[1]))


def _note(msg):
    print("[parity] " + msg, flush=True)


# a priori rounding bound of evaluating sum_k c_k Phi_k(p) in FP64 in any
# order: (number of terms + recurrence and collapse depth) units of 2^-53
# times sum_k |c_k Phi_k(p)|; 512 units covers 343 terms plus the Legendre
# recurrences (3 x 6), the GPU's collapse over (y, z) (49 terms), the
# conversion to the row coordinate (7) and Horner (7)
GAMMA64 = 512 * 2.0 ** -53


def _eval_bound(level, coeffs, deg):
    """S(p) = sum_k |c_k Phi_k(p)| per point and direction, (N, 8)."""
    pts = O.interior_points(level).astype(np.float64) / (1 << level)
    return np.abs(O.legendre_tensor_matrix(pts, deg)) @ np.abs(np.asarray(coeffs)).T


@pytest.mark.parametrize("deg", [4, 6])
def test_fit_reaches_the_least_squares_minimum(torch, pkg, deg):
    # the GPU TSQR fit on S_d against the oracle's pivoted QR:
    # * equal residual norms: the minimum is unique where the solution is not;
    # * equal fitted values on the sample points (the projection of the
    #   samples onto the polynomial space is unique): since r_o is orthogonal
    #   to the space, ||V (c_g - c_o)||^2 = ||r_g||^2 - ||r_o||^2, so the
    #   residual bound gives ||V dc|| <= sqrt(2e-6) ||r_o||, plus rounding;
    # * values away from the samples within the first-order perturbation bound
    #   of least squares, 10 cond(V) 2^-53 of the values (cond(V) of each
    #   direction's sample matrix; 1e13 at degree 6 on level 7, where FP64
    #   solvers differ by up to 1e-2 there)
    k = _case(deg)
    sm = pkg.Smoother([k["t"]], pkg.SURR_F64, degree=deg, stride=4, tile=(16, 16))
    assert sm.sample_stride(0) == k["s"]
    cg = sm.surrogate(0)
    pts = O.interior_points(LEVEL).astype(np.float64) / (1 << LEVEL)
    Vall = O.legendre_tensor_matrix(pts, deg)
    worst, worst_s, worst_v, cmax = 0.0, 0.0, 0.0, 0.0
    for row, slot in enumerate(list(range(O.NLOW)) + [O.CENTRE]):
        idx = O.sample_set(LEVEL, slot, k["s"])
        V = Vall[idx]
        y = k["L"][idx, slot] if slot < O.NLOW else 1.0 / k["D"][idx]
        ro = np.linalg.norm(V @ k["c"][row] - y)
        rg = np.linalg.norm(V @ cg[row] - y)
        worst = max(worst, abs(rg - ro) / ro)
        assert abs(rg - ro) <= 1e-6 * ro, (O.DIR_NAMES[slot], rg, ro)
        ds = np.linalg.norm(V @ (cg[row] - k["c"][row]))
        worst_s = max(worst_s, ds / ro)
        assert ds <= np.sqrt(2e-6) * ro + 1e-12 * np.linalg.norm(y), O.DIR_NAMES[slot]
        cond = np.linalg.cond(V)
        cmax = max(cmax, cond)
        vg, vo = Vall @ cg[row], Vall @ k["c"][row]
        dv = np.abs(vg - vo).max() / np.abs(vo).max()
        worst_v = max(worst_v, dv)
        assert dv <= 10 * cond * 2.0 ** -53, (O.DIR_NAMES[slot], dv, cond)
    _note("deg %d fit: residual norms agree to %.1e, sample values to %.1e of ||r||, values to %.1e "
          "(largest cond %.1e)" % (deg, worst, worst_s, worst_v, cmax))


@pytest.mark.parametrize("variant", ["SURR_F64", "SURR_F32"])
@pytest.mark.parametrize("deg", [4, 6])
def test_tables_evaluate_the_fitted_polynomials(torch, pkg, deg, variant):
    # the per-row Horner tables give the values of the handle's own fitted
    # polynomials at every point (collapse over (y, z), conversion to the row
    # coordinate, Horner), within the FP64 evaluation bound GAMMA64 S(p); for
    # FP32 plus the FP32 Horner error, a few units of 2^-24 of the direction's
    # size
    k = _case(deg)
    v = getattr(pkg, variant)
    sm = pkg.Smoother([k["t"]], v, degree=deg, stride=4, tile=(16, 16))
    cg = sm.surrogate(0)
    Lo, Do = O.eval_surrogate(LEVEL, cg, deg)
    Lg, Dg = (a.cpu().numpy() for a in sm.surrogate_values(0))
    got = np.column_stack([Lg, Dg])
    ref = np.column_stack([Lo, Do])
    bound = GAMMA64 * _eval_bound(LEVEL, cg, deg)
    if v == pkg.SURR_F32:
        # plus the FP32 Horner of the row polynomial (coefficients rounded to
        # FP32, dg_x steps): a few units of 2^-24 of the direction's size
        bound = bound + 4 * (deg + 2) * U32 * np.abs(ref).max(axis=0)
    ratio = (np.abs(got - ref) / bound).max()
    _note("deg %d %s tables: %.1e of max per direction, %.2f of the rounding bound"
          % (deg, variant, _colrel(got, ref), ratio))
    assert ratio <= 1.0


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("deg", [4, 6])
def test_f64_sweeps_with_oracle_coefficients(torch, pkg, deg, tile):
    # Alg. 2 (V2) in FP64 with the oracle's coefficients injected:
    # * with the weights the kernels evaluate on both sides, 6 sweeps agree to
    #   1e-12 (only the order of the sums differs);
    # * the weights agree with the oracle's evaluation within the rounding
    #   bound of the evaluation, and the iterates with the oracle's weights
    #   differ by no more than the weights do
    k = _case(deg)
    sm = pkg.Smoother([k["t"]], pkg.SURR_F64, degree=deg, stride=4, tile=tile)
    sm.set_surrogate(0, k["c"])
    Lg, Dg = (a.cpu().numpy() for a in sm.surrogate_values(0))
    got = np.column_stack([Lg, Dg])
    ref = np.column_stack([k["Lw"], k["Dinv"]])
    assert (np.abs(got - ref) <= GAMMA64 * _eval_bound(LEVEL, k["c"], deg)).all()
    ew = _colrel(got, ref)
    b = k["t"].rhs()
    x = torch.zeros(k["P"].N, dtype=torch.float64, device="cuda")
    sm.smooth(x, torch.tensor(b, device="cuda"), 6)
    xg = x.cpu().numpy()
    own, _ = k["P"].smooth_stencil(Lg, Dg, b, nsweeps=6)
    want, _ = k["P"].smooth_stencil(k["Lw"], k["Dinv"], b, nsweeps=6)
    e_own, e_or = _rel(xg, own), _rel(xg, want)
    _note("deg %d tile %s FP64 sweeps: x vs oracle with the kernel's weights %.1e; weights vs oracle's %.1e, x %.1e"
          % (deg, tile, e_own, ew, e_or))
    assert e_own <= 1e-12
    assert e_or <= max(1e-12, ew)


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("deg", [4, 6])
def test_f32_sweeps(torch, pkg, deg, tile):
    # FP32 weights and substitutions, FP64 residual and update:
    # * one sweep from x = 0 leaves x = (double) w with w in FP32, so every
    #   entry is an FP32 number (an FP64 substitution fails this);
    # * with the kernel's own FP32 weights on both sides, 8 sweeps match the
    #   oracle's FP32 emulation to a few FP32 roundings of the corrections
    #   (the seven products are summed in another order on the GPU);
    # * the weights match the oracle's FP64 values to the FP32 evaluation error.
    k = _case(deg)
    sm = pkg.Smoother([k["t"]], pkg.SURR_F32, degree=deg, stride=4, tile=tile)
    sm.set_surrogate(0, k["c"])
    Lg, Dg = (a.cpu().numpy() for a in sm.surrogate_values(0))
    ew = max(_colrel(Lg, k["Lw"]), _rel(Dg, k["Dinv"]))
    assert ew <= 256 * U32
    L32, D32 = Lg.astype(np.float32), Dg.astype(np.float32)
    assert np.array_equal(L32.astype(np.float64), Lg) and np.array_equal(D32.astype(np.float64), Dg)
    b = k["t"].rhs()
    bd = torch.tensor(b, device="cuda")
    x = torch.zeros(k["P"].N, dtype=torch.float64, device="cuda")
    sm.smooth(x, bd, 1)
    x1 = x.cpu().numpy()
    assert np.array_equal(x1.astype(np.float32).astype(np.float64), x1)
    want1, _ = k["P"].smooth_stencil_f32(L32, D32, b, nsweeps=1)
    e1 = _rel(x1, want1)
    sm.smooth(x, bd, 7)
    want, _ = k["P"].smooth_stencil_f32(L32, D32, b, nsweeps=8)
    e8 = _rel(x.cpu().numpy(), want)
    w64, _ = k["P"].smooth_stencil(Lg, Dg, b, nsweeps=8)
    gap = _rel(want, w64)
    _note("deg %d tile %s FP32: weights %.1e, x after 1 sweep %.1e, after 8 %.1e (FP32 vs FP64 oracle %.1e)"
          % (deg, tile, ew, e1, e8, gap))
    assert e1 <= 16 * U32
    assert e8 <= 64 * U32


# ------------------------------------------------ several blocks per workgroup

def _nblocks(level, bv, bw):
    # blocks of the (v, w) row triangle v in [2, n-2], w in [1, v-1] holding a row
    n = 1 << level
    nbv = max(1, (n - 3 + bv - 1) // bv)
    nbw = max(1, (n - 3 + bw - 1) // bw)
    return sum(1 for kv in range(nbv) for kw in range(nbw) if 1 + bw * kw <= min(n - 2, 1 + bv * (kv + 1)) - 1)


@pytest.mark.parametrize("grid", [1, 3])
@pytest.mark.parametrize("tile", [(8, 8), (16, 16)])
def test_capped_grid_stored_parity(torch, pkg, grid, tile):
    # with the persistent grid capped, every workgroup takes many blocks in turn
    # (LDS grid cleared, halo roles and ticket taken again per block): the
    # stored-factor sweeps still match the oracle to 1e-12 and the uncapped
    # run bit for bit
    level = 6
    t = W.make_tet(21, level, *W.KAPPA_SIN, jitter=0.15)
    P = O.Problem.from_tet(t)
    L, U, D = P.ilu0()
    b = t.rhs()
    bd = torch.tensor(b, device="cuda")
    sm = pkg.Smoother([t], pkg.STORED_F64, tile=tile)
    x_free = torch.zeros_like(bd)
    sm.smooth(x_free, bd, 5)
    assert sm.set_flow_grid(grid) == grid < _nblocks(level, *tile)
    x = torch.zeros_like(bd)
    sm.smooth(x, bd, 5)
    want, _ = P.smooth(L, D, b, nsweeps=5)
    assert _rel(x.cpu().numpy(), want) < 1e-12
    assert torch.equal(x, x_free)
    assert sm.set_flow_grid(0) > grid


@pytest.mark.parametrize("variant", ["SURR_F32", "SURR_F64"])
@pytest.mark.parametrize("boundary", ["BOUNDARY_V2", "BOUNDARY_V1"])
def test_capped_grid_surrogate_parity(torch, pkg, variant, boundary):
    # the surrogate sweeps (both boundary variants) on a grid of 2 workgroups,
    # with the oracle's coefficients injected: bitwise equal to the uncapped
    # grid, and against the oracle's Alg. 2 with the weights the kernels use
    # (checked against the oracle's own to the evaluation's rounding at
    # degree 4: 1e-9 FP64, 1e-5 FP32): FP64 to 1e-12, FP32 to a few FP32
    # roundings of the corrections
    level, deg = 6, 4
    t = W.make_tet(22, level, *W.KAPPA_EXP, jitter=0.15)
    P = O.Problem.from_tet(t)
    L, U, D = P.ilu0()
    s = O.effective_stride(level, deg, 4)
    c = O.fit_surrogate(level, L, D, deg, s)
    Lw, Dinv = O.eval_surrogate(level, c, deg)
    v = getattr(pkg, variant)
    bnd = getattr(pkg, boundary)
    sm = pkg.Smoother([t], v, degree=deg, stride=4, tile=(8, 8), boundary=bnd)
    sm.set_surrogate(0, c)
    b = t.rhs()
    bd = torch.tensor(b, device="cuda")
    x_free = torch.zeros_like(bd)
    sm.smooth(x_free, bd, 5)
    assert sm.set_flow_grid(2) == 2
    x = torch.zeros_like(bd)
    sm.smooth(x, bd, 5)
    assert torch.equal(x, x_free)
    # the weights the kernels use (V1: the exact factors at the boundary
    # points) against the oracle's, then the sweeps with those weights
    Lg, Dg = (a.cpu().numpy() for a in sm.surrogate_values(0))
    if bnd == pkg.BOUNDARY_V1:
        Lw, Dinv = P.v1_weights(Lw, Dinv, L, D)
    tol_w = 1e-9 if v == pkg.SURR_F64 else 1e-5
    assert _colrel(np.column_stack([Lg, Dg]), np.column_stack([Lw, Dinv])) < tol_w
    if v == pkg.SURR_F64:
        want, _ = P.smooth_stencil(Lg, Dg, b, nsweeps=5)
        assert _rel(x.cpu().numpy(), want) < 1e-12
    else:
        want, _ = P.smooth_stencil_f32(Lg.astype(np.float32), Dg.astype(np.float32), b, nsweeps=5)
        assert _rel(x.cpu().numpy(), want) < 64 * U32


def test_batch_with_second_tickets(torch, pkg):
    # 64 level-6 tetrahedra on 8x8 blocks: more blocks than resident
    # workgroups, so the default grid takes second tickets; stored FP64
    # tetrahedron by tetrahedron against the oracle (1e-12), FP32 surrogate
    # against the oracle's FP32 emulation with the kernel's weights
    tets = W.batch_tets(31, 64, (6,))
    bd = torch.tensor(np.concatenate([t.rhs() for t in tets]), device="cuda")
    st = pkg.Smoother(tets, pkg.STORED_F64, tile=(8, 8))
    grid = st.set_flow_grid(0)
    assert grid < 64 * _nblocks(6, 8, 8)
    x = torch.zeros_like(bd)
    st.smooth(x, bd, 3)
    xs = x.cpu().numpy()
    sm = pkg.Smoother(tets, pkg.SURR_F32, degree=4, stride=4, tile=(8, 8))
    assert sm.set_flow_grid(0) < 64 * _nblocks(6, 8, 8)
    x.zero_()
    sm.smooth(x, bd, 3)
    x32 = x.cpu().numpy()
    worst64 = worst32 = 0.0
    for i, t in enumerate(tets):
        o, n = st.offsets[i], st.counts[i]
        P = O.Problem.from_tet(t)
        L, U, D = P.ilu0()
        want, _ = P.smooth(L, D, t.rhs(), nsweeps=3)
        worst64 = max(worst64, _rel(xs[o:o + n], want))
        Lg, Dg = (a.cpu().numpy() for a in sm.surrogate_values(i))
        want32, _ = P.smooth_stencil_f32(Lg.astype(np.float32), Dg.astype(np.float32), t.rhs(), nsweeps=3)
        worst32 = max(worst32, _rel(x32[o:o + n], want32))
    _note("batch of 64 (grid %d): stored %.1e, FP32 %.1e" % (grid, worst64, worst32))
    assert worst64 < 1e-12
    assert worst32 < 64 * U32
