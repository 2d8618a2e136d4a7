"""ilu_lfa_orientation_noalloc (every intermediate in the library's static
device scratch array, no device allocation) against ilu_lfa_orientation
(buffers allocated per call), through the C-ABI: the same kernels on the same
vertex values, so mu and the choices must be identical, on two calls in a
row (the second with fewer tetrahedra and another frequency grid, reading
the scratch the first one left), at the maximum size, and rejected beyond it."""
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    import paper_2210_15280_amd as P
    P.lib()
    return P


def _flat(mu):
    return [v for row in mu for v in row]


def test_noalloc_matches_allocating_call_twice(pkg):
    first = list(W.batch_tets(51, 40, (4,)))
    second = list(W.batch_tets(52, 5, (4,)))
    for tets, samples in ((first, 16), (second, 32)):
        mu_a, best_a = pkg.lfa_orientation(tets, samples)
        mu_n, best_n = pkg.lfa_orientation_noalloc(tets, samples)
        assert _flat(mu_n) == _flat(mu_a)
        assert best_n == best_a


def test_noalloc_at_the_maximum_size_and_beyond(pkg):
    tets = list(W.batch_tets(53, pkg.LFA_NOALLOC_MAX_TETS, (4,)))
    mu_a, best_a = pkg.lfa_orientation(tets, 16)
    mu_n, best_n = pkg.lfa_orientation_noalloc(tets, 16)
    assert _flat(mu_n) == _flat(mu_a) and best_n == best_a
    with pytest.raises(pkg.ILUError) as e:
        pkg.lfa_orientation_noalloc(tets + tets[:1], 16)
    assert e.value.code == -1
