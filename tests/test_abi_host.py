"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every symbol include/ilu.h declares, and rejects bad arguments before any
device work (geometry, level, degree, rank of the sampled problems)."""
import ctypes
import os

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    import paper_2210_15280_amd as pkg
    if not os.path.exists(pkg.library_path()):
        from paper_2210_15280_amd import build
        build.build()
    pkg.lib()
    return pkg


def test_header_symbols_exported(P):
    names = P.header_symbols()
    for must in ("ilu_setup_surrogate", "ilu_smooth", "stencil_apply", "ilu_layout", "ilu_destroy",
                 "ilu_strerror", "ilu_get_stencil", "ilu_get_factors", "ilu_get_surrogate",
                 "ilu_set_surrogate", "ilu_get_surrogate_values", "ilu_sample_stride", "ilu_last_timing"):
        assert must in names
    assert P.exported_symbols() == names


def test_strerror(P):
    L = P.lib()
    assert L.ilu_strerror(0) == b"success"
    assert b"breakdown" in L.ilu_strerror(-4)
    assert L.ilu_strerror(-99) == b"unknown error"


def _setup(P, tets, variant=0, degree=(4, 4, 4), stride=4, boundary=0, tile=(0, 0)):
    from paper_2210_15280_amd._lib import ilu_opts, ilu_tet_desc
    arr = (ilu_tet_desc * len(tets))()
    for i, t in enumerate(tets):
        arr[i].vertex[:] = [c for row in t.verts for c in row]
        arr[i].level = t.level
        arr[i].coeff_kind = t.coeff_kind
        arr[i].coeff_param[:] = list(t.coeff_params)
    o = ilu_opts()
    o.variant = variant
    o.degree[:] = list(degree)
    o.sample_stride = stride
    o.boundary = boundary
    o.tile[:] = list(tile)
    h = ctypes.c_void_p()
    return P.lib().ilu_setup_surrogate(arr, len(tets), ctypes.byref(o), None, ctypes.byref(h))


def test_degenerate_tet_is_rejected_and_either_orientation_accepted(P):
    from paper_2210_15280_amd._lib import _tet_array, ilu_opts
    flat = W.Tet(((0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0)), 4, 0, (1.0, 0, 0, 0), 0)
    assert _setup(P, [flat]) == -6
    # swapping two vertices flips det J: accepted (the layout replay runs on the host)
    t = W.make_tet(1, 4, W.COEFF_CONST, (1.0,))
    v = list(t.verts)
    v[1], v[2] = v[2], v[1]
    inv = W.Tet(tuple(v), 4, 0, (1.0, 0, 0, 0), t.rhs_state)
    o = ilu_opts()
    o.variant, o.tile[:] = 0, [8, 8]
    bad = ctypes.c_int64(-1)
    assert P.lib().ilu_check_layout(_tet_array([inv]), 1, ctypes.byref(o), ctypes.byref(bad)) == 0
    assert bad.value == 0


def test_lfa_orientation_argument_checks(P):
    from paper_2210_15280_amd._lib import _tet_array
    t = W.make_tet(1, 4, W.COEFF_CONST, (1.0,))
    mu = (ctypes.c_double * 24)()
    best = (ctypes.c_int32 * 1)()
    L = P.lib()
    for samples in (0, 2, 6, 18, 260):
        assert L.ilu_lfa_orientation(_tet_array([t]), 1, samples, mu, best, None) == -1
    assert L.ilu_lfa_orientation(_tet_array([t]), 1, 16, None, None, None) == -1
    assert L.ilu_lfa_orientation(_tet_array([t]), 0, 16, mu, best, None) == -1
    flat = W.Tet(((0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0)), 4, 0, (1.0, 0, 0, 0), 0)
    assert L.ilu_lfa_orientation(_tet_array([flat]), 1, 16, mu, best, None) == -6


def test_invalid_arguments(P):
    t = W.make_tet(1, 4, W.COEFF_CONST, (1.0,))
    assert _setup(P, []) == -1                                               # no tetrahedron
    assert _setup(P, [W.Tet(t.verts, 1, 0, (1.0, 0, 0, 0), 0)]) == -1      # level < 2
    assert _setup(P, [W.Tet(t.verts, 11, 0, (1.0, 0, 0, 0), 0)]) == -1     # level > 10
    assert _setup(P, [W.Tet(t.verts, 4, 9, (1.0, 0, 0, 0), 0)]) == -1      # coefficient kind
    assert _setup(P, [t], variant=1, degree=(7, 7, 7)) == -1                 # degree
    assert _setup(P, [t], variant=1, stride=3) == -1                         # stride not a power of two
    assert _setup(P, [t], variant=1, boundary=2) == -1                       # boundary variant
    assert _setup(P, [t], variant=0, boundary=1) == -1                       # V1 needs a surrogate
    assert _setup(P, [t], tile=(8, 16)) == -1                                # unsupported block shape
    assert _setup(P, [t], variant=5) == -1
    L = P.lib()
    assert L.ilu_smooth(None, None, None, 1, 0.0, None, None) == -1
    assert L.stencil_apply(None, None, None, None) == -1
    assert L.ilu_destroy(None) == 0


def test_rank_deficient_sampling_is_rejected(P):
    # level 3 has 7 intervals per edge: no stride leaves a sample simplex of side
    # >= 12 for degree 4, so every LSQ problem is rank deficient
    t = W.make_tet(1, 3, W.COEFF_CONST, (1.0,))
    assert _setup(P, [t], variant=1, degree=(4, 4, 4)) == -5


def _check_layout(P, tets, variant=0, degree=2, stride=4, tile=(0, 0)):
    from paper_2210_15280_amd._lib import ilu_opts, ilu_tet_desc
    arr = (ilu_tet_desc * len(tets))()
    for i, t in enumerate(tets):
        arr[i].vertex[:] = [c for row in t.verts for c in row]
        arr[i].level = t.level
        arr[i].coeff_kind = t.coeff_kind
        arr[i].coeff_param[:] = list(t.coeff_params)
    o = ilu_opts()
    o.variant = variant
    o.degree[:] = [degree] * 3
    o.sample_stride = stride
    o.tile[:] = list(tile)
    bad = ctypes.c_int64(-1)
    rc = P.lib().ilu_check_layout(arr, len(tets), ctypes.byref(o), ctypes.byref(bad))
    return rc, bad.value


@pytest.mark.parametrize("tile", [(8, 8), (16, 16), (16, 32)])
@pytest.mark.parametrize("level", [2, 3, 4, 5, 6, 7])
def test_layout_replay_has_no_violations(P, level, tile):
    # every index the residual, hyperplane and dataflow kernels form stays in its
    # stream and addresses the intended point (or a never-written zero slot);
    # every interior point is covered exactly once; orders are topological
    t = W.make_tet(5, level, *W.KAPPA_SIN, jitter=0.15)
    assert _check_layout(P, [t], tile=tile) == (0, 0)
    if level >= 5:
        assert _check_layout(P, [t], variant=2, degree=2, tile=tile) == (0, 0)


@pytest.mark.parametrize("tile", [(8, 8), (16, 16)])
def test_layout_replay_batch(P, tile):
    tets = W.batch_tets(11, 24, (4, 5, 6))
    assert _check_layout(P, tets, variant=2, degree=1, stride=2, tile=tile) == (0, 0)
