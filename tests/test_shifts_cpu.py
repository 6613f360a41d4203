"""Shift heuristic (Ritz values + greedy min-max, one reading of the
Krylov-subspace shifts of Sec. 5): the oracle pinned to closed forms, and
the library's host steps (Hessenberg eigenvalues, greedy choice) checked
against the oracle and LAPACK.  No GPU work."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as wl
from oracle import adi
from oracle import shifts as osh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2607_14742_amd", "libmpcare.so")
needs_lib = pytest.mark.skipif(not os.path.exists(LIB), reason="libmpcare.so not built")


# ---------------------------------------------------------------- oracle pins
def test_arnoldi_stops_on_invariant_subspace_with_exact_ritz_values():
    # diag with three distinct eigenvalues: the Krylov space of ones has
    # dimension 3, so Arnoldi stops after 3 steps and the Ritz values are them
    a = np.repeat([-1.0, -7.0, -30.0], [5, 9, 4])
    H = osh.arnoldi(lambda v: a * v, np.ones(a.size), 10)
    assert H.shape == (3, 3)
    assert np.allclose(np.sort(np.linalg.eigvals(H).real), [-30.0, -7.0, -1.0], rtol=1e-12)


def test_ritz_values_of_symmetric_operator_lie_in_the_closed_form_spectrum():
    N = 20
    A = wl.fdm2d(N, 0.0)                     # no convection: symmetric
    lam = np.sort(wl.fdm2d_eigenvalues(N, 0.0).real)
    R = osh.ritz_candidates(A, kp=20, km=10)
    assert np.all(np.abs(R.imag) < 1e-8 * np.abs(R.real))
    assert R.real.min() >= lam[0] * (1 + 1e-10) and R.real.max() <= lam[-1] * (1 - 1e-10)
    # the inverse steps converge to the eigenvalue nearest zero (its mode,
    # sin(pi x) sin(pi y), dominates the start vector of ones); the forward
    # steps approach the far end of the spectrum (the top mode itself is odd
    # about the centre and absent from ones, hence the loose bound)
    assert abs(R.real.max() - lam[-1]) < 1e-8 * abs(lam[-1])
    assert abs(R.real.min() - lam[0]) < 3e-2 * abs(lam[0])


def test_greedy_choice_by_hand():
    # first: minimise max |(t-p)/(t+p)|: p=-2 gives max(1/3, 98/102) = 0.961 < 99/101;
    # then t=-100 (0.961 > 1/3), then t=-1
    assert np.allclose(osh.penzl_select([-1.0, -2.0, -100.0], 3), [-2.0, -100.0, -1.0])
    assert np.allclose(osh.penzl_select([-1.0, -2.0, -100.0], 1), [-2.0])
    # a complex first choice scores 2 (|(-4j)/(-2)|) against its own conjugate, so -5 comes first;
    # the pair then joins whole, Im > 0 first, even past l0
    P = osh.penzl_select([-1 + 2j, -1 - 2j, -5.0], 2)
    assert np.allclose(P, [-5.0, -1 + 2j, -1 - 2j])
    # unstable candidates never take part
    assert np.allclose(osh.penzl_select([0.5, -3.0, 2.0 + 1j], 4), [-3.0])


def test_greedy_choice_is_scale_invariant():
    rng = np.random.default_rng(3)
    R = -np.exp(rng.uniform(0, 6, 25)) + 1j * np.where(rng.random(25) < 0.3, rng.uniform(1, 30, 25), 0)
    R = np.concatenate([R, np.conj(R[R.imag != 0])])
    P1 = osh.penzl_select(R, 10)
    P2 = osh.penzl_select(37.5 * R, 10)
    assert np.allclose(37.5 * P1, P2, rtol=1e-12)


def test_penzl_shifts_annihilate_a_diagonal_lyapunov_equation():
    # the Ritz values of a diagonal matrix with 4 distinct eigenvalues are
    # exact, the heuristic returns exactly those 4, and 4 ADI steps with them
    # leave a zero residual (each factor (a - p)/(a + p) vanishes on one)
    a = np.repeat([-2.0, -11.0, -60.0, -400.0], [6, 5, 7, 4])
    A = sp.diags(a).tocsr()
    P = osh.penzl_shifts(A, l0=4, kp=8, km=0)
    assert np.allclose(np.sort(P.real), [-400.0, -60.0, -11.0, -2.0], rtol=1e-10)
    W0 = np.random.default_rng(5).standard_normal((a.size, 2))
    _, W, info = adi.lradi(A, None, None, W0, P, tol=0.0, jmax=4)
    assert np.linalg.norm(W.T @ W) <= 1e-18 * np.linalg.norm(W0.T @ W0)


# ------------------------------------------------------- library host logic
@needs_lib
def test_library_hessenberg_eigenvalues_match_lapack():
    import paper_2607_14742_amd as pk
    rng = np.random.default_rng(11)
    for k in list(range(1, 33)) + [50, 80]:
        for kind in range(3):
            H = np.triu(rng.standard_normal((k, k)), -1)
            if kind == 1 and k > 3:
                H[k // 2, k // 2 - 1] = 0.0          # split into two blocks
            if kind == 2:
                H = np.triu(H)                        # already triangular
            got = np.sort_complex(pk.ritz_values(H))
            ref = np.sort_complex(np.linalg.eigvals(H))
            assert np.max(np.abs(got - ref)) <= 1e-11 * max(1.0, np.max(np.abs(ref))), (k, kind)


@needs_lib
def test_library_hessenberg_eigenvalues_of_arnoldi_matrices():
    import paper_2607_14742_amd as pk
    A = wl.fdm3d(6, 100.0, "rotating")
    H = osh.arnoldi(lambda v: A.T @ v, np.ones(A.shape[0]), 20)
    got = np.sort_complex(pk.ritz_values(H))
    ref = np.sort_complex(np.linalg.eigvals(H))
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))
    assert np.any(np.abs(ref.imag) > 1e-6 * np.abs(ref))   # the rotating field gives complex pairs


@needs_lib
def test_library_greedy_choice_matches_oracle():
    import paper_2607_14742_amd as pk
    rng = np.random.default_rng(7)
    for trial in range(150):
        nr = int(rng.integers(1, 30))
        R = -np.exp(rng.uniform(0, 8, nr)) + 1j * np.where(rng.random(nr) < 0.3, rng.uniform(-50, 50, nr), 0.0)
        R = np.concatenate([R, np.conj(R[R.imag != 0]), [0.3, 1.0 + 2j]])   # plus unstable values
        l0 = int(rng.integers(1, 20))
        got, ref = pk.penzl_select(R, l0), osh.penzl_select(R, l0)
        assert got.shape == ref.shape and np.allclose(got, ref, rtol=1e-13), trial
        # pairs adjacent, Im > 0 first
        i = 0
        while i < got.size:
            if got[i].imag != 0:
                assert got[i].imag > 0 and got[i + 1] == np.conj(got[i])
                i += 2
            else:
                i += 1


@needs_lib
def test_library_rejects_all_unstable_candidates():
    import paper_2607_14742_amd as pk
    with pytest.raises(pk.CareError):
        pk.penzl_select([0.1, 2.0 + 1j, 2.0 - 1j], 4)


# ------------------------------------------------- Wachspress real shift sets
@pytest.mark.parametrize("lo,hi,J", [(69.74, 2.008e6, 12), (1.0, 1e3, 5), (3.0, 40.0, 3)])
def test_wachspress_shifts_equioscillate(lo, hi, J):
    # the minimax rational function prod (l - p)/(l + p) over [lo, hi] has
    # |r| equal at its J + 1 extremal points: both ends and one point
    # between each pair of neighbouring shifts (Chebyshev alternation)
    p = -wl.wachspress_real_shifts(lo, hi, J).real
    assert p.size == J and np.all(np.diff(p) < 0) and lo <= p.min() and p.max() <= hi
    lam = np.geomspace(lo, hi, 400001)
    r = np.ones_like(lam)
    for pj in p:
        r *= (lam - pj) / (lam + pj)
    a = np.abs(r)
    inner = np.nonzero((a[1:-1] > a[:-2]) & (a[1:-1] >= a[2:]))[0] + 1
    ext = np.concatenate([[a[0]], a[inner], [a[-1]]])
    assert ext.size == J + 1
    assert ext.max() / ext.min() - 1 < 1e-4
    # and a log-spaced set of the same size does worse
    q = np.geomspace(lo, hi, J)
    rq = np.ones_like(lam)
    for qj in q:
        rq *= (lam - qj) / (lam + qj)
    assert np.abs(rq).max() > ext.max()


# ---------------------------------------------------------------------------
# projection shifts (oracle): pinned to hand-computed Ritz values
# ---------------------------------------------------------------------------
def _as_set(z):
    return sorted(np.round(np.asarray(z), 12), key=lambda t: (t.real, t.imag))


def test_projection_shifts_on_an_invariant_subspace_are_its_eigenvalues():
    # span(V) = span(e2, e5, e7) is invariant under a diagonal A: the Ritz
    # values are A's eigenvalues there, whatever basis V holds
    A = sp.diags(-np.arange(1.0, 11.0)).tocsr()
    V = np.zeros((10, 3))
    V[2, 0], V[5, 1], V[2, 1], V[7, 2] = 3.0, 1.0, 1.0, 0.5
    got = osh.projection_shifts(A, V, l0=5)
    assert _as_set(got) == _as_set([-3.0, -6.0, -8.0])


def test_projection_shifts_of_a_rotation_block_are_a_conjugate_pair():
    a, b = -2.0, 3.0
    A = np.diag([-5.0, 0.0, 0.0, -7.0])
    A[1:3, 1:3] = [[a, b], [-b, a]]
    V = np.zeros((4, 2))
    V[1, 0] = V[2, 1] = 1.0
    got = osh.projection_shifts(A, V, l0=4)
    assert len(got) == 2
    assert np.allclose(got, [complex(a, b), complex(a, -b)], atol=1e-12)   # Im > 0 first


def test_projection_shifts_mirror_unstable_ritz_values():
    A = sp.diags([2.0, -3.0, -4.0]).tocsr()
    V = np.eye(3)[:, :2]
    assert _as_set(osh.projection_shifts(A, V, l0=4)) == _as_set([-2.0, -3.0])


def test_projection_shifts_use_the_closed_loop_operator():
    # F = A^T - K B^T with B = e1, K = c e1: F = diag(-1 - c, -2, -3)
    c = 4.0
    A = sp.diags([-1.0, -2.0, -3.0]).tocsr()
    B = np.array([[1.0], [0.0], [0.0]])
    K = c * B
    V = np.eye(3)[:, :2]
    assert _as_set(osh.projection_shifts(A, V, l0=4, B=B, K=K)) == _as_set([-1.0 - c, -2.0])


def test_projection_shifts_depend_on_the_subspace_only():
    A = wl.fdm2d(9)
    rng = np.random.default_rng(5)
    V = rng.standard_normal((81, 5))
    R = rng.standard_normal((5, 5)) + 5.0 * np.eye(5)
    s1 = osh.projection_shifts(A, V, l0=8)
    s2 = osh.projection_shifts(A, np.hstack([V @ R, V[:, :2]]), l0=8)   # another basis, with repeated columns
    assert np.allclose(_as_set(s1), _as_set(s2), rtol=1e-9, atol=0)
