"""Pins of the CPU oracle against facts fixed by the paper and by mathematics
(closed forms, identities, library routines, brute force on tiny inputs).
None of these compares the oracle with itself."""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import workloads as wl
from oracle import adi, care, lowrank, riccati

RNG = np.random.default_rng(7)


def scalar_care(a, b2, c2):
    """Stabilizing root of 2 a x - b2 x^2 + c2 = 0 (n = 1), cancellation free."""
    if b2 == 0:
        return -c2 / (2 * a)
    d = math.sqrt(a * a + b2 * c2)
    return (a + d) / b2 if a >= 0 else c2 / (d - a)


def random_stable_sparse(n, density, rng, margin=1.0):
    """Nonsymmetric sparse matrix shifted to be stable (Gershgorin)."""
    R = sp.random(n, n, density=density, random_state=np.random.RandomState(rng.integers(1 << 30)))
    R = R - R.T * 0.3
    d = np.asarray(abs(R).sum(axis=1)).ravel() + margin
    return (R - sp.diags(d)).tocsr()


# --------------------------------------------------------------------------
# scalar and decoupled closed forms
# --------------------------------------------------------------------------
@pytest.mark.parametrize("a,m,p", [(-2.0, 1, 1), (-0.3, 3, 2), (1.5, 2, 4), (-40.0, 4, 1)])
def test_scalar_closed_form_dense(a, m, p):
    B = RNG.standard_normal((1, m))
    C = RNG.standard_normal((p, 1))
    x = scalar_care(a, float((B @ B.T)[0, 0]), float((C.T @ C)[0, 0]))
    assert abs(riccati.care_schur(np.array([[a]]), B, C)[0, 0] - x) <= 1e-12 * x
    if a < 0:
        X, _ = riccati.newton_kleinman_dense(np.array([[a]]), B, C)
        assert abs(X[0, 0] - x) <= 1e-12 * x


def test_scalar_closed_form_framework():
    """n = 1: one ADI step with shift p = a solves the Lyapunov equation
    exactly; the whole Framework 1 must reproduce the scalar root."""
    a = -3.0
    A = sp.csr_matrix(np.array([[a]]))
    B = np.array([[0.7, -1.1]])
    C = np.array([[2.0], [0.5]])
    x = scalar_care(a, float((B @ B.T)[0, 0]), float((C.T @ C)[0, 0]))
    Z, info = care.framework1(A, B, C, np.array([a + 0j]), tol=1e-14)
    assert abs((Z @ Z.T)[0, 0] - x) <= 1e-13 * x


def test_decoupled_diagonal_care():
    n = 6
    a = -RNG.uniform(0.5, 5.0, n)
    b = RNG.uniform(0.2, 2.0, n)
    c = RNG.uniform(0.2, 2.0, n)
    A, B, C = np.diag(a), np.diag(b), np.diag(c)
    Xcf = np.diag([scalar_care(a[i], b[i] ** 2, c[i] ** 2) for i in range(n)])
    assert np.allclose(riccati.care_schur(A, B, C), Xcf, rtol=0, atol=1e-12 * Xcf.max())
    X, _ = riccati.newton_kleinman_dense(A, B, C)
    assert np.allclose(X, Xcf, rtol=0, atol=1e-12 * Xcf.max())
    Z, _ = care.framework1(sp.csr_matrix(A), B, C, wl.logspaced_real_shifts(0.5, 5.0, 6), tol=1e-13)
    assert np.allclose(Z @ Z.T, Xcf, rtol=0, atol=1e-11 * Xcf.max())


# --------------------------------------------------------------------------
# Lyapunov / ADI closed forms
# --------------------------------------------------------------------------
def test_cauchy_lyapunov_closed_form():
    """Diagonal A: X_ij = -(W W^T)_ij / (a_i + a_j) solves A^T X + X A + W W^T = 0."""
    n, w = 30, 3
    a = -np.geomspace(1.0, 100.0, n)
    W = RNG.standard_normal((n, w))
    Xcf = -(W @ W.T) / (a[:, None] + a[None, :])
    Z, Wj, info = adi.lradi(sp.diags(a).tocsr(), None, None, W, wl.logspaced_real_shifts(1.0, 100.0, 8),
                            tol=1e-15, jmax=200)
    assert np.linalg.norm(Z @ Z.T - Xcf) <= 1e-13 * np.linalg.norm(Xcf)
    X_bs = riccati.lyap_bartels_stewart(np.diag(a), -(W @ W.T))
    assert np.linalg.norm(X_bs - Xcf) <= 1e-13 * np.linalg.norm(Xcf)


@pytest.mark.parametrize("shifts", [
    [-1.0, -7.0, -30.0],
    [-2.0 + 3.0j, -2.0 - 3.0j, -15.0],
    [-5.0, -1.0 + 0.5j, -1.0 - 0.5j, -40.0 + 60.0j, -40.0 - 60.0j],
])
def test_adi_diagonal_product_formula(shifts):
    """Diagonal A: after the steps, W(i,:) = prod_j (a_i - p_j)/(a_i + p_j) W0(i,:),
    a conjugate pair contributing |(a - p)/(a + p)|^2."""
    n, w = 25, 2
    a = -np.geomspace(0.5, 80.0, n)
    W0 = RNG.standard_normal((n, w))
    s = np.asarray(shifts, dtype=np.complex128)
    Z, Wj, info = adi.lradi(sp.diags(a).tocsr(), None, None, W0, s, tol=0.0, jmax=len(s))
    assert info["steps"] == len(s)
    fac = np.ones(n)
    for p in s:
        fac = fac * ((a - p) / (a + p))
    assert np.allclose(fac.imag, 0, atol=1e-13)
    assert np.allclose(Wj, fac.real[:, None] * W0, rtol=1e-12, atol=1e-14)
    # residual identity F Z Z^T + Z Z^T F^T + W0 W0^T = W W^T
    X = Z @ Z.T
    R = a[:, None] * X + X * a[None, :] + W0 @ W0.T
    assert np.linalg.norm(R - Wj @ Wj.T) <= 1e-12 * np.linalg.norm(W0 @ W0.T)


def test_adi_shift_annihilates_row():
    a = -np.array([1.0, 3.0, 9.0, 27.0])
    W0 = np.ones((4, 1))
    _, Wj, _ = adi.lradi(sp.diags(a).tocsr(), None, None, W0, np.array([-9.0 + 0j]), tol=0, jmax=1)
    assert abs(Wj[2, 0]) < 1e-15 and abs(Wj[0, 0]) > 0.1


def test_complex_pair_equals_two_complex_steps():
    """The real double step for (p, conj p) gives the same Z Z^T and W as two
    plain complex ADI steps V_j = (F + p_j I)^{-1} W_{j-1} on a nonsymmetric A."""
    n, w = 40, 2
    A = random_stable_sparse(n, 0.15, RNG).toarray()
    W0 = RNG.standard_normal((n, w))
    p = -3.0 + 5.0j
    Z, Wr, _ = adi.lradi(sp.csr_matrix(A), None, None, W0, np.array([p, np.conj(p)]), tol=0, jmax=2)
    W = W0.astype(np.complex128)
    Zc = []
    for pj in (p, np.conj(p)):
        V = np.linalg.solve(A.T + pj * np.eye(n), W)
        W = W - 2 * pj.real * V
        Zc.append(math.sqrt(-2 * pj.real) * V)
    Zc = np.hstack(Zc)
    Xc = Zc @ Zc.conj().T
    assert np.abs(Xc.imag).max() <= 1e-12 * np.abs(Xc).max()
    assert np.linalg.norm(Z @ Z.T - Xc.real) <= 1e-12 * np.linalg.norm(Xc)
    assert np.allclose(Wr, W.real, atol=1e-12 * np.abs(W0).max()) and np.abs(W.imag).max() < 1e-12


def test_adi_order_independence():
    """The ADI factors commute: the same shift set in another order gives the
    same Z Z^T after the same number of steps."""
    A = wl.fdm2d(9, 10.0)
    W0 = RNG.standard_normal((81, 2))
    s = np.array([-50.0, -300.0 + 200.0j, -300.0 - 200.0j, -900.0, -2500.0])
    s2 = np.array([-900.0, -2500.0, -300.0 + 200.0j, -300.0 - 200.0j, -50.0])
    Z1, W1, _ = adi.lradi(A, None, None, W0, s, tol=0, jmax=5)
    Z2, W2, _ = adi.lradi(A, None, None, W0, s2, tol=0, jmax=5)
    assert lowrank.factored_diff_norm(Z1, Z2) <= 1e-12 * lowrank.factored_norm(Z1)
    assert np.allclose(W1, W2, atol=1e-11 * np.abs(W0).max())


@pytest.mark.parametrize("p", [-4.0, -2.0 + 7.0j])
def test_smw_shifted_solve(p):
    """SMW solve of (A_k^T + p I) V = W with A_k = A - B K^T against a dense solve."""
    n, m, w = 60, 3, 4
    A = random_stable_sparse(n, 0.1, RNG)
    B = RNG.standard_normal((n, m))
    K = 0.3 * RNG.standard_normal((n, m))
    W = RNG.standard_normal((n, w))
    V = adi.ShiftedSolver(A, B, K).solve(p, W)
    Ak = A.toarray() - B @ K.T
    Vd = np.linalg.solve(Ak.T + p * np.eye(n), W)
    assert np.linalg.norm(V - Vd) <= 1e-12 * np.linalg.norm(Vd)


def test_lradi_closed_loop_vs_bartels_stewart():
    n, m = 49, 2
    A = wl.fdm2d(7, 10.0)
    B = RNG.standard_normal((n, m))
    K = 0.5 * RNG.standard_normal((n, m))
    W0 = RNG.standard_normal((n, 3))
    lo, hi = wl.fdm2d_spectral_bounds(7, 10.0)
    Z, _, info = adi.lradi(A, B, K, W0, wl.logspaced_real_shifts(lo, hi, 10), tol=1e-14, jmax=300)
    Ak = A.toarray() - B @ K.T
    X = riccati.lyap_bartels_stewart(Ak.T, -(W0 @ W0.T))
    assert np.linalg.norm(Z @ Z.T - X) <= 1e-11 * np.linalg.norm(X)


# --------------------------------------------------------------------------
# Algorithm 1 and Algorithm 2 identities
# --------------------------------------------------------------------------
def _small_problem(n=50, m=2, p=3, r=6):
    A = random_stable_sparse(n, 0.12, RNG)
    B = RNG.standard_normal((n, m))
    C = RNG.standard_normal((p, n))
    Z = RNG.standard_normal((n, r)) * 0.2
    return A, B, C, Z


def test_alg1_exact_without_truncation():
    A, B, C, Z = _small_problem()
    Cp, Cm, res = lowrank.residual_factor(A, B, C, Z, eta_r_rel=0.0)
    R = riccati.riccati_residual(A, B, C, Z @ Z.T)
    assert np.linalg.norm(Cp @ Cp.T - Cm @ Cm.T - R) <= 1e-12 * np.linalg.norm(R)
    assert abs(res - np.linalg.norm(R, "fro")) <= 1e-12 * res
    # brute force: the nonzero spectrum of R is the spectrum of H
    ev = np.linalg.eigvalsh(R)
    big = ev[np.abs(ev) > 1e-10 * np.abs(ev).max()]
    full = lowrank.residual_factor(A, B, C, Z, 0.0, full=True)
    lam = full["lam"][np.abs(full["lam"]) > 1e-10 * np.abs(full["lam"]).max()]
    assert np.allclose(np.sort(big), np.sort(lam), rtol=1e-9)


def test_alg1_truncation_thresholds():
    A, B, C, Z = _small_problem()
    eta_rel = 1e-2
    full = lowrank.residual_factor(A, B, C, Z, eta_rel, full=True)
    lam, eta = full["lam"], full["eta"]
    assert full["Cp"].shape[1] == np.sum(lam >= eta) and full["Cm"].shape[1] == np.sum(lam <= -eta)
    R = riccati.riccati_residual(A, B, C, Z @ Z.T)
    err = np.linalg.norm(full["Cp"] @ full["Cp"].T - full["Cm"] @ full["Cm"].T - R)
    dropped = lam[np.abs(lam) < eta]
    assert abs(err - np.sqrt(np.sum(dropped ** 2))) <= 1e-10 * np.linalg.norm(R)


def test_alg1_signs_and_blocks():
    """Each block of M matters: Z with B = 0 and C = 0 leaves A^T X + X A,
    whose trace is 2 tr(A^T Z Z^T) (sign/transposition check)."""
    A, B, C, Z = _small_problem()
    Cp, Cm, res = lowrank.residual_factor(A, B * 0, C * 0, Z, 0.0)
    tr = np.trace(Cp @ Cp.T) - np.trace(Cm @ Cm.T)
    assert abs(tr - 2 * np.trace(A.T @ Z @ Z.T)) <= 1e-11 * abs(tr)
    # only the -X B B^T X term: A = 0, C = 0 -> R = -(Z Z^T B)(Z Z^T B)^T is NSD
    Cp, Cm, res = lowrank.residual_factor(A * 0, B, C * 0, Z, 0.0)
    K = Z @ (Z.T @ B)
    assert np.linalg.norm(Cm @ Cm.T - K @ K.T) <= 1e-12 * np.linalg.norm(K @ K.T)
    assert Cp.shape[1] == 0 or np.linalg.norm(Cp) <= 1e-7 * np.linalg.norm(Cm)


def test_alg2_exact_psd_update():
    n = 70
    Z = RNG.standard_normal((n, 5))
    Zp = 0.1 * RNG.standard_normal((n, 4))
    Zm = 0.5 * Z[:, :2] @ np.array([[0.6, 0.0], [0.8, 0.0]])   # X - Zm Zm^T stays PSD
    Znew = lowrank.solution_factor(Z, Zp, Zm, eta_s_rel=0.0)
    Xt = Z @ Z.T + Zp @ Zp.T - Zm @ Zm.T
    assert np.linalg.norm(Znew @ Znew.T - Xt) <= 1e-12 * np.linalg.norm(Xt)
    assert Znew.shape[1] <= 9


def test_alg2_drops_negative_part():
    n = 40
    Z = RNG.standard_normal((n, 3))
    Zm = RNG.standard_normal((n, 2))            # makes G N G^T indefinite
    full = lowrank.solution_factor(Z, np.zeros((n, 0)), Zm, 0.0, full=True)
    Xt = Z @ Z.T - Zm @ Zm.T
    ev, Q = np.linalg.eigh(Xt)
    Xpos = (Q[:, ev > 0] * ev[ev > 0]) @ Q[:, ev > 0].T
    assert np.linalg.norm(full["Z"] @ full["Z"].T - Xpos) <= 1e-11 * np.linalg.norm(Xpos)
    assert full["eta_n"] > 0.01


def test_factored_diff_norm_brute_force():
    Z = RNG.standard_normal((30, 4))
    Y = Z + 1e-9 * RNG.standard_normal((30, 4))
    d = lowrank.factored_diff_norm(Z, Y)
    assert abs(d - np.linalg.norm(Z @ Z.T - Y @ Y.T)) <= 1e-6 * d


# --------------------------------------------------------------------------
# whole-solver pins
# --------------------------------------------------------------------------
def test_newton_kleinman_matches_schur():
    n, m, p = 30, 2, 3
    A = random_stable_sparse(n, 0.2, RNG).toarray()
    B = RNG.standard_normal((n, m))
    C = RNG.standard_normal((p, n))
    Xs = riccati.care_schur(A, B, C)
    Xn, hist = riccati.newton_kleinman_dense(A, B, C)
    assert np.linalg.norm(Xn - Xs) <= 1e-11 * np.linalg.norm(Xs)
    assert hist[-1] < 1e-12


def _check_solution_properties(A, B, C, Z, Xref, xtol):
    X = Z @ Z.T
    assert np.linalg.norm(X - Xref) <= xtol * np.linalg.norm(Xref)
    assert np.linalg.eigvalsh(Xref).min() >= -1e-12 * np.abs(Xref).max()
    Acl = A.toarray() - B @ (B.T @ X)
    assert np.linalg.eigvals(Acl).real.max() < 0


def test_framework1_config1_vs_schur():
    P = wl.config1()
    Z, info = care.framework1(P.A, P.B, P.C, P.shifts, tol=1e-13)
    Xs = riccati.care_schur(P.A, P.B, P.C)
    _check_solution_properties(P.A, P.B, P.C, Z, Xs, 1e-11)
    assert info["hist"][-1] <= 1e-13


def test_framework1_refines_perturbed_start():
    """Starting Framework 1 from a deliberately poor Z_1 (a truncated solution)
    the refinement loop (Alg. 1 -> LR-ADI -> Alg. 2) must converge to Schur."""
    P = wl.fdm2d_problem(12, 2, 2)
    Xs = riccati.care_schur(P.A, P.B, P.C)
    ev, Q = np.linalg.eigh(Xs)
    keep = ev > 1e-4 * ev.max()
    Z1 = Q[:, keep] * np.sqrt(ev[keep]) * 0.97
    Z, info = care.framework1(P.A, P.B, P.C, P.shifts, tol=1e-12, Z1=Z1, tau_L=1e-13, jmax=200)
    assert info["iter"][0] >= 3 and info["iter"][1] > 0
    _check_solution_properties(P.A, P.B, P.C, Z, Xs, 1e-10)


def test_framework1_nonsymmetric_complex_shifts():
    """A 3D rotating-field FDM matrix (complex spectrum) with complex shift pairs."""
    A = wl.fdm3d(5, nu=100.0)
    n = A.shape[0]
    B, C = wl.gaussian_factors(n, 2, 3, seed=5)
    ev = np.linalg.eigvals(A.toarray())
    assert np.abs(ev.imag).max() > 1.0
    s = np.array([-40.0 + 25.0j, -40.0 - 25.0j, -150.0, -500.0 + 100.0j, -500.0 - 100.0j, -1500.0])
    Z, info = care.framework1(A, B, C, s, tol=1e-13)
    Xs = riccati.care_schur(A, B, C)
    _check_solution_properties(A, B, C, Z, Xs, 1e-10)


# --------------------------------------------------------------------------
# generator pins (closed forms of the synthetic workloads)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("N", [6, 13, 20])
def test_fdm2d_closed_form_spectrum(N):
    A = wl.fdm2d(N, 10.0)
    assert A.nnz == 5 * N * N - 4 * N
    ev = np.sort(np.linalg.eigvals(A.toarray()).real)
    cf = np.sort(wl.fdm2d_eigenvalues(N, 10.0))
    assert np.abs(ev - cf).max() <= 1e-11 * np.abs(cf).max()
    lo, hi = wl.fdm2d_spectral_bounds(N, 10.0)
    assert np.isclose(-cf.max(), lo) and np.isclose(-cf.min(), hi)


def test_fdm_sizes_match_configs():
    assert wl.config1().A.nnz == 1920
    N = 500
    assert 5 * N * N - 4 * N == 1_248_000
    assert wl.fdm3d(64).nnz == 1_810_432
    Ns, ms, ps = wl.fdm_batch_sizes()
    assert Ns[0] == 100 and Ns[-1] == 632 and sum(N * N for N in Ns) == 3_484_121


def test_fdm3d_constant_field_is_kronecker_sum():
    N, nu = 4, 10.0
    A = wl.fdm3d(N, nu=nu, field_kind="constant").toarray()
    lo, d, up = wl.fdm1d_coeffs(N, nu)
    T = np.diag(np.full(N, d)) + np.diag(np.full(N - 1, lo), -1) + np.diag(np.full(N - 1, up), 1)
    I = np.eye(N)
    K = np.kron(np.kron(I, I), T) + np.kron(np.kron(I, T), I) + np.kron(np.kron(T, I), I)
    assert np.allclose(A, K)


def test_ex1_gallery_orthog():
    V = wl.gallery_orthog(64)
    assert np.allclose(V, V.T) and np.allclose(V @ V, np.eye(64), atol=1e-13)
    A, B, C = wl.ex1(64, 3, 2, q=3.0)
    s = np.linalg.svd(A, compute_uv=False)
    assert np.isclose(s.max() / s.min(), 1e3)


def test_toeplitz5_definition_and_dissipativity():
    # the Toeplitz example (Sec. 5.2): sub-diagonal 1, diagonal -2.8, the
    # first three super-diagonals -1, every other entry 0
    n = 9
    A = wl.toeplitz5(n).toarray()
    for i in range(n):
        for j in range(n):
            want = {-1: 1.0, 0: -2.8, 1: -1.0, 2: -1.0, 3: -1.0}.get(j - i, 0.0)
            assert A[i, j] == want, (i, j)
    # The symmetric part is the Hermitian Toeplitz section of the symbol
    # s(t) = -2.8 - cos 2t - cos 3t, so its eigenvalues lie below max s
    # (Grenander-Szego).  That maximum is negative, so A is dissipative and
    # hence stable, with the field of values left of it.
    t = np.linspace(0.0, np.pi, 100001)
    smax = (-2.8 - np.cos(2 * t) - np.cos(3 * t)).max()
    assert smax < -1.0
    A = wl.toeplitz5(300).toarray()
    lam_s = np.linalg.eigvalsh((A + A.T) / 2)
    assert lam_s.max() <= smax + 1e-12 and lam_s.max() >= smax - 1e-2
    assert np.linalg.eigvals(A).real.max() <= smax + 1e-12
    P = wl.toeplitz_problem(300)
    assert P.B.shape == (300, 10) and P.C.shape == (5, 300)
    assert np.isclose(np.linalg.norm(P.B), 1.0)


# --------------------------------------------------------------------------
# the paper's reported residual "Res" (Sec. 5) on a hand-worked example
# --------------------------------------------------------------------------
def hand_worked_res_example():
    """A = diag(-1, -2), Z = [sqrt 2; 0], B = [1; 1], C = [3, 0].
    By hand: X = Z Z^T = 2 e1 e1^T; A^T X + X A = -4 e1 e1^T;
    X B B^T X = (X B)(X B)^T = 4 e1 e1^T; C^T C = 9 e1 e1^T; so
    R(X) = e1 e1^T and ||R||_F = 1.  Norms: ||A||_F = sqrt 5,
    ||Z^T Z||_F = 2, ||B^T B||_F = 2, ||C C^T||_F = 9.  The denominator of
    Res is 2 sqrt5 2 + 2 2^2 + 9 = 17 + 4 sqrt 5."""
    A = sp.csr_matrix(np.diag([-1.0, -2.0]))
    Z = np.array([[math.sqrt(2.0)], [0.0]])
    B = np.array([[1.0], [1.0]])
    C = np.array([[3.0, 0.0]])
    return A, B, C, Z, 1.0 / (17.0 + 4.0 * math.sqrt(5.0))


def test_paper_res_hand_worked_example():
    A, B, C, Z, expected = hand_worked_res_example()
    R = riccati.riccati_residual(A, B, C, Z @ Z.T)
    assert np.allclose(R, np.array([[1.0, 0.0], [0.0, 0.0]]), atol=1e-14, rtol=0)
    res = np.linalg.norm(R, "fro")
    # (Z holds sqrt 2 rounded, so ||R||_F carries a few ulps)
    assert abs(riccati.paper_res(A, B, C, Z, res) - expected) <= 1e-13 * expected
    # a dense A gives the same value
    assert abs(riccati.paper_res(A.toarray(), B, C, Z, res) - expected) <= 1e-13 * expected


def test_paper_res_scaling_law():
    """Scaling C by t and Z by sqrt(t) scales the denominator's first and last
    terms by t and the middle one by t^2; with B -> B / sqrt(t) every term
    scales by t, and R(Z) scales by t (R is homogeneous of degree one in
    (Z Z^T, C^T C) once B B^T is scaled by 1/t), so Res is unchanged."""
    n, m, p, r = 12, 2, 3, 4
    rng = np.random.default_rng(5)
    A = random_stable_sparse(n, 0.3, rng)
    B = rng.standard_normal((n, m))
    C = rng.standard_normal((p, n))
    Z = 0.2 * rng.standard_normal((n, r))
    t = 7.0

    def res(A, B, C, Z):
        R = riccati.riccati_residual(A, B, C, Z @ Z.T)
        return riccati.paper_res(A, B, C, Z, np.linalg.norm(R, "fro"))
    r0 = res(A, B, C, Z)
    r1 = res(A, B / math.sqrt(t), math.sqrt(t) * C, math.sqrt(t) * Z)
    assert abs(r1 - r0) <= 1e-13 * r0


# --------------------------------------------------------------------------
# shift-set validation (Sec. 4: Re p < 0, conjugate pairs adjacent)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shifts", [
    [-1.0, -2.0],
    [-1.0 + 2.0j, -1.0 - 2.0j],
    [-3.0, -1.0 + 2.0j, -1.0 - 2.0j, -0.5],
])
def test_check_shifts_accepts_valid_sets(shifts):
    s = adi.check_shifts(np.array(shifts))
    assert s.dtype == np.complex128 and s.size == len(shifts)


@pytest.mark.parametrize("shifts", [
    [],                                    # empty set
    [-1.0, 0.0],                           # Re p = 0 (the ADI factor (a - p)/(a + p) is not contractive)
    [-1.0, 0.5],                           # Re p > 0
    [0.5 + 1.0j, 0.5 - 1.0j],              # pair in the right half-plane
    [-1.0 + 2.0j],                         # complex shift without its conjugate
    [-1.0 + 2.0j, -2.0],                   # conjugate not adjacent
    [-1.0 - 2.0j, -1.0 + 2.0j],            # Im < 0 first
    [-1.0 + 2.0j, -1.0 - 3.0j],            # second entry is not the conjugate
])
def test_check_shifts_rejects_invalid_sets(shifts):
    with pytest.raises(ValueError):
        adi.check_shifts(np.array(shifts, dtype=np.complex128))


# --------------------------------------------------------------------------
# Hamiltonian-Schur CARE solver and the Kronecker plane-wise shifted solver
# --------------------------------------------------------------------------
@pytest.mark.parametrize("a,m,p", [(-2.0, 1, 1), (1.5, 2, 4)])
def test_hamiltonian_scalar_closed_form(a, m, p):
    B = RNG.standard_normal((1, m))
    C = RNG.standard_normal((p, 1))
    x = scalar_care(a, float((B @ B.T)[0, 0]), float((C.T @ C)[0, 0]))
    assert abs(riccati.care_hamiltonian(np.array([[a]]), B, C)[0, 0] - x) <= 1e-12 * x


def test_hamiltonian_decoupled_and_vs_library():
    n = 6
    a = -RNG.uniform(0.5, 5.0, n)
    b = RNG.uniform(0.2, 2.0, n)
    c = RNG.uniform(0.2, 2.0, n)
    Xcf = np.diag([scalar_care(a[i], b[i] ** 2, c[i] ** 2) for i in range(n)])
    X = riccati.care_hamiltonian(np.diag(a), np.diag(b), np.diag(c))
    assert np.allclose(X, Xcf, rtol=0, atol=1e-12 * Xcf.max())
    # a nonsymmetric 40 x 40 problem against the library's QZ-based routine
    A = random_stable_sparse(40, 0.2, RNG).toarray()
    B = RNG.standard_normal((40, 3))
    C = RNG.standard_normal((2, 40))
    Xh = riccati.care_hamiltonian(A, B, C)
    Xs = riccati.care_schur(A, B, C)
    assert np.linalg.norm(Xh - Xs) <= 1e-11 * np.linalg.norm(Xs)
    assert np.all(np.linalg.eigvals(A - B @ (B.T @ Xh)).real < 0)


@pytest.mark.parametrize("p", [-300.0, -150.0 + 400.0j])
def test_kron_z_solver_matches_sparse_lu(p):
    """The plane-wise solve of A^T + p I for the rotating-field 3D matrix
    (no z-convection) against a sparse LU of the whole matrix, with and
    without the SMW feedback term."""
    A = wl.fdm3d(6, 100.0, "rotating")
    n = A.shape[0]
    Ap, T = adi.kron_z_split(A)
    assert Ap.shape == (36, 36) and T.shape == (6, 6)
    B = RNG.standard_normal((n, 2))
    K = 0.01 * RNG.standard_normal((n, 2))
    W = RNG.standard_normal((n, 3))
    for b, k in ((None, None), (B, K)):
        ref = adi.ShiftedSolver(A, b, k).solve(p, W)
        got = adi.KronZShiftedSolver(A, b, k).solve(p, W)
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_kron_z_split_rejects_z_convection():
    # a constant field has z-convection: the plane coupling is not symmetric
    with pytest.raises(ValueError):
        adi.kron_z_split(wl.fdm3d(5, 10.0, "constant"))
