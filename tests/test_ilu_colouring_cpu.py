"""The library's host colouring behind its multicolour ILU(0) (the GMRES
preconditioner of Sec. 5, "Performance Analysis on GPU"), called through the
host-only C-ABI entry point and compared bit for bit with the oracle's
first-fit colouring; argument checks and the colour limit.  No GPU work."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as wl
from oracle import ilu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2607_14742_amd", "libmpcare.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libmpcare.so not built")


def random_pattern(n, density, seed):
    R = sp.random(n, n, density=density, random_state=np.random.RandomState(seed))
    return (R - sp.identity(n)).tocsr()


@pytest.mark.parametrize("name,make", [
    ("fdm2d_13", lambda: wl.fdm2d(13)),
    ("fdm3d_6", lambda: wl.fdm3d(6)),
    ("toeplitz_97", lambda: wl.toeplitz5(97)),
    ("random_300", lambda: random_pattern(300, 0.02, 4)),
    ("random_dense_60", lambda: random_pattern(60, 0.3, 5)),
    ("identity", lambda: sp.identity(17, format="csr")),
    ("lower_only", lambda: sp.tril(random_pattern(80, 0.1, 6)).tocsr()),
])
def test_library_colouring_equals_the_oracle(name, make):
    import paper_2607_14742_amd as pk
    A = make()
    colours, nc = pk.ilu0_colouring(A)
    ref = ilu.greedy_colouring(A)
    assert np.array_equal(colours, ref), name
    assert nc == int(ref.max()) + 1


def test_library_colouring_rejects_bad_patterns_and_too_many_colours():
    import paper_2607_14742_amd as pk
    A = wl.fdm2d(5)
    bad = sp.csr_matrix(A)
    bad.indices = bad.indices.copy()
    bad.indices[3] = 10_000
    with pytest.raises(pk.api.CareError) as e:
        pk.ilu0_colouring(bad)
    assert e.value.name == "CARE_ERR_ARG"
    K = sp.csr_matrix(np.ones((1100, 1100)))          # a complete graph needs 1100 colours
    with pytest.raises(pk.api.CareError) as e:
        pk.ilu0_colouring(K)
    assert e.value.name == "CARE_ERR_NOT_IMPLEMENTED"
