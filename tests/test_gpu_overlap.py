"""The residual overlapped with, or fused into, the forward substitution
(ilu_set_overlap): every mode gives bitwise the same iterates as the default
(residual kernel, then the forward substitution), eagerly and from the
captured graph, for every kernel variant, block shape and a batch, and with
the refinement loop; where the overlap is not available it is off and cannot
be switched on.  The default mode is checked against the oracle by the sweep
parity tests (and here once more for the stored factors)."""
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


def _run(torch, sm, b, nsweeps, mode, graph):
    sm.set_overlap(mode)
    sm.set_graph(graph)
    x = torch.zeros_like(b)
    sm.smooth(x, b, nsweeps)
    return x.cpu().numpy()


@pytest.mark.parametrize("variant", [0, 1, 2])
@pytest.mark.parametrize("tile", [(8, 8), (16, 16), (16, 32)])
def test_modes_agree_bitwise(torch, pkg, variant, tile):
    t = W.make_tet(51, 6, *W.KAPPA_SIN, jitter=0.15)
    kw = {} if variant == 0 else dict(degree=3, stride=4)
    sm = pkg.Smoother([t], variant, tile=tile, **kw)
    assert sm.overlap() == pkg.OVERLAP_OFF
    b = torch.tensor(t.rhs(), device="cuda")
    ref = _run(torch, sm, b, 5, pkg.OVERLAP_OFF, False)
    for mode in (pkg.OVERLAP_ON, pkg.OVERLAP_FUSED):
        for graph in (False, True):
            assert np.array_equal(_run(torch, sm, b, 5, mode, graph), ref), (mode, graph)
    # against the oracle once, with the default mode (FP64 stored factors)
    if variant == 0:
        P = O.Problem.from_tet(t)
        L, U, D = P.ilu0()
        want, _ = P.smooth(L, D, t.rhs(), nsweeps=5)
        assert np.abs(ref - want).max() <= 1e-12 * np.abs(want).max()


def test_graph_replays_with_overlap_match_eager(torch, pkg):
    # several replays in a row, with eager work between them
    t = W.make_tet(52, 7, *W.KAPPA_EXP, jitter=0.15)
    sm = pkg.Smoother([t], pkg.SURR_F32, degree=4, stride=4, tile=(16, 16))
    b = torch.tensor(t.rhs(), device="cuda")
    sm.set_overlap(pkg.OVERLAP_ON)
    sm.set_graph(True)
    xg = torch.zeros_like(b)
    for _ in range(3):
        sm.smooth(xg, b, 4)
        torch.cuda.synchronize()
        _ = (xg * 2.0).sum().item()
    sm.set_overlap(pkg.OVERLAP_OFF)
    sm.set_graph(False)
    xe = torch.zeros_like(b)
    sm.smooth(xe, b, 12)
    assert torch.equal(xg, xe)


def test_refinement_with_overlap(torch, pkg):
    # rel_tol > 0: the overlapped residual kernel also reduces the norm
    t = W.make_tet(53, 5, *W.KAPPA_SIN, jitter=0.15)
    sm = pkg.Smoother([t], pkg.SURR_F32, degree=3, stride=4, tile=(8, 8))
    b = torch.tensor(t.rhs(), device="cuda")
    out = []
    for mode in (pkg.OVERLAP_OFF, pkg.OVERLAP_ON, pkg.OVERLAP_FUSED):
        sm.set_overlap(mode)
        x = torch.zeros_like(b)
        rel, ok = sm.smooth(x, b, 3000, rel_tol=1e-10, want_relres=True)
        assert ok and rel <= 1e-10
        out.append((sm.last_sweeps, x.cpu().numpy()))
    assert out[0][0] == out[1][0] == out[2][0]
    assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[0][1], out[2][1])


@pytest.mark.parametrize("tile", [(8, 8), (16, 16)])
def test_batch_modes_agree(torch, pkg, tile):
    # both block shapes of the LDS-staged residual: its tagged form walks the
    # absolute bands of every tetrahedron of the batch
    tets = W.batch_tets(54, 12, (4, 5, 6))
    sm = pkg.Smoother(tets, pkg.SURR_F32, degree=2, stride=4, tile=tile)
    b = torch.tensor(np.concatenate([t.rhs() for t in tets]), device="cuda")
    ref = _run(torch, sm, b, 4, pkg.OVERLAP_OFF, False)
    assert np.array_equal(_run(torch, sm, b, 4, pkg.OVERLAP_ON, True), ref)
    assert np.array_equal(_run(torch, sm, b, 4, pkg.OVERLAP_FUSED, False), ref)


def test_overlap_availability(pkg):
    import paper_2210_15280_amd._lib as L
    t = W.make_tet(55, 4, *W.KAPPA_SIN, jitter=0.15)
    cases = [pkg.Smoother([t], pkg.STORED_F64, schedule=pkg.SCHED_PLANE),
             pkg.Smoother([t], pkg.SURR_F64, degree=2, stride=4, tile=(8, 8), boundary=pkg.BOUNDARY_V1),
             pkg.Smoother([t], pkg.SURR_F32, degree=2, stride=4, tile=(8, 8), a_mode=pkg.A_SURROGATE)]
    for sm in cases:
        assert sm.overlap() == pkg.OVERLAP_OFF
        for mode in (pkg.OVERLAP_ON, pkg.OVERLAP_FUSED):
            with pytest.raises(L.ILUError):
                sm.set_overlap(mode)
        sm.set_overlap(pkg.OVERLAP_OFF)
    sm = pkg.Smoother([t], pkg.STORED_F64, tile=(8, 8))
    with pytest.raises(L.ILUError):
        sm.set_overlap(3)


@pytest.mark.parametrize("grid", [1, 3, 0])
@pytest.mark.parametrize("variant", [0, 2])
def test_overlap_on_capped_grids(torch, pkg, variant, grid):
    # the overlapped residual beside a forward sweep on a capped grid (the
    # combination the autotuner picks for large tetrahedra): the sweep waits
    # for the residual's band marks, and the iterates equal the sequential
    # ones bit for bit, eagerly and from the graph, on a batch
    tets = W.batch_tets(53, 4, (5, 6))
    kw = {} if variant == 0 else dict(degree=3, stride=4)
    sm = pkg.Smoother(tets, variant, tile=(8, 8), **kw)
    b = torch.tensor(np.concatenate([t.rhs() for t in tets]), device="cuda")
    ref = _run(torch, sm, b, 4, pkg.OVERLAP_OFF, False)
    assert sm.set_flow_grid(grid) >= 1
    for graph in (False, True):
        assert np.array_equal(_run(torch, sm, b, 4, pkg.OVERLAP_ON, graph), ref), graph
    rel, ok = sm.smooth(torch.zeros_like(b), b, 16, rel_tol=1e-3)
    sm.set_overlap(pkg.OVERLAP_OFF)
    rel0, ok0 = sm.smooth(torch.zeros_like(b), b, 16, rel_tol=1e-3)
    assert rel == rel0 and ok == ok0


def test_full_size_level9_modes_agree_bitwise(torch, pkg):
    # the benchmark's headline variant and workload at full size (level 9,
    # 22,108,415 points, FP32 surrogate dg 6, 16x16 blocks, the full
    # persistent grid): from a random start (so that the residual beside the
    # forward sweep is not just b), three sweeps give bitwise the same iterate
    # with the residual before, beside and inside the forward substitution,
    # eagerly and as one captured graph
    wl = W.workload("jit_L9_exp")
    t = wl.tets[0]
    sm = pkg.Smoother([t], pkg.SURR_F32, tile=(16, 16), degree=wl.degree, stride=wl.stride)
    b = torch.tensor(t.rhs(), device="cuda")
    x0 = torch.rand(b.shape, dtype=torch.float64, generator=torch.Generator().manual_seed(10)).to("cuda") - 0.5

    def run(mode, graph):
        sm.set_overlap(mode)
        sm.set_graph(graph)
        x = x0.clone()
        sm.smooth(x, b, 3)
        return x

    ref = run(pkg.OVERLAP_OFF, False)
    assert not torch.equal(ref, x0)
    for mode, graph in ((pkg.OVERLAP_ON, False), (pkg.OVERLAP_ON, True), (pkg.OVERLAP_FUSED, False)):
        assert torch.equal(run(mode, graph), ref), (mode, graph)
