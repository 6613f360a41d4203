"""Plant plausible mistakes in the oracle (on the CPU, via monkeypatching)
and check that the pins catch them: a dropped sign in the residual core
matrix, a wrong ADI coefficient, a transposed operand in the shifted solve,
a wrong complex-pair weight."""
import math

import numpy as np
import scipy.sparse as sp

import workloads as wl
from oracle import adi, lowrank, riccati

RNG = np.random.default_rng(11)


def _alg1_pin_error():
    n, m, p, r = 40, 2, 3, 5
    A = (sp.random(n, n, density=0.15, random_state=np.random.RandomState(3)) - 4 * sp.identity(n)).tocsr()
    B = RNG.standard_normal((n, m))
    C = RNG.standard_normal((p, n))
    Z = 0.3 * RNG.standard_normal((n, r))
    Cp, Cm, _ = lowrank.residual_factor(A, B, C, Z, 0.0)
    R = riccati.riccati_residual(A, B, C, Z @ Z.T)
    return np.linalg.norm(Cp @ Cp.T - Cm @ Cm.T - R) / np.linalg.norm(R)


def test_alg1_pin_catches_wrong_sign(monkeypatch):
    assert _alg1_pin_error() < 1e-12
    orig = lowrank.residual_core_matrix

    def wrong(r, m, p):
        M = orig(r, m, p)
        M[2 * r:2 * r + m, 2 * r:2 * r + m] *= -1.0     # + X B B^T X instead of -
        return M
    monkeypatch.setattr(lowrank, "residual_core_matrix", wrong)
    assert _alg1_pin_error() > 1e-3


def _adi_product_error():
    a = -np.geomspace(0.5, 80.0, 20)
    W0 = RNG.standard_normal((20, 2))
    s = np.array([-3.0, -1.0 + 2.0j, -1.0 - 2.0j])
    _, Wj, _ = adi.lradi(sp.diags(a).tocsr(), None, None, W0, s, tol=0, jmax=3)
    fac = np.prod([(a - p) / (a + p) for p in s], axis=0).real
    return np.abs(Wj - fac[:, None] * W0).max()


def test_adi_pin_catches_wrong_update(monkeypatch):
    assert _adi_product_error() < 1e-12

    class WrongSolver(adi.ShiftedSolver):
        def solve(self, p, W):                  # (F - p I)^{-1} instead of (F + p I)^{-1}
            return super().solve(-np.conj(p), W) * -1.0
    monkeypatch.setattr(adi, "ShiftedSolver", WrongSolver)
    assert _adi_product_error() > 1e-3


def test_smw_pin_catches_transpose(monkeypatch):
    n, m = 30, 2
    A = (sp.random(n, n, density=0.2, random_state=np.random.RandomState(5)) - 5 * sp.identity(n)).tocsr()
    B = RNG.standard_normal((n, m))
    K = 0.4 * RNG.standard_normal((n, m))
    W = RNG.standard_normal((n, 3))
    Vd = np.linalg.solve((A.toarray() - B @ K.T).T - 2.0 * np.eye(n), W)
    good = adi.ShiftedSolver(A, B, K).solve(-2.0, W)
    assert np.linalg.norm(good - Vd) < 1e-12 * np.linalg.norm(Vd)
    bad = adi.ShiftedSolver(A.T.tocsr(), B, K).solve(-2.0, W)     # A instead of A^T
    assert np.linalg.norm(bad - Vd) > 1e-3 * np.linalg.norm(Vd)


def test_complex_pair_pin_catches_missing_weight(monkeypatch):
    n = 30
    A = (sp.random(n, n, density=0.2, random_state=np.random.RandomState(9)) - 6 * sp.identity(n)).toarray()
    W0 = RNG.standard_normal((n, 2))
    p = -2.0 + 4.0j

    def two_complex_steps():
        W = W0.astype(np.complex128)
        Zc = []
        for pj in (p, np.conj(p)):
            V = np.linalg.solve(A.T + pj * np.eye(n), W)
            W = W - 2 * pj.real * V
            Zc.append(math.sqrt(-2 * pj.real) * V)
        Zc = np.hstack(Zc)
        return (Zc @ Zc.conj().T).real

    Xc = two_complex_steps()
    Z, _, _ = adi.lradi(sp.csr_matrix(A), None, None, W0, np.array([p, np.conj(p)]), tol=0, jmax=2)
    assert np.linalg.norm(Z @ Z.T - Xc) < 1e-12 * np.linalg.norm(Xc)
    # drop the sqrt(delta^2 + 1) weight of the second block
    delta = p.real / p.imag
    Zbad = Z.copy()
    Zbad[:, 2:] /= math.sqrt(delta * delta + 1.0)
    assert np.linalg.norm(Zbad @ Zbad.T - Xc) > 1e-3 * np.linalg.norm(Xc)


def test_paper_res_pin_catches_dropped_term(monkeypatch):
    """Drop the ||B^T B||_F ||Z^T Z||_F^2 term of the paper's Res denominator
    (or square the wrong factor): the hand-worked example must fail."""
    from tests.test_oracle_pins import hand_worked_res_example
    A, B, C, Z, expected = hand_worked_res_example()

    def dropped(A, B, C, Z, res_fro):
        nA = sp.linalg.norm(A, "fro")
        ZtZ = np.linalg.norm(Z.T @ Z, "fro")
        return res_fro / (2 * nA * ZtZ + np.linalg.norm(C @ C.T, "fro"))

    def unsquared(A, B, C, Z, res_fro):
        nA = sp.linalg.norm(A, "fro")
        ZtZ = np.linalg.norm(Z.T @ Z, "fro")
        return res_fro / (2 * nA * ZtZ + np.linalg.norm(B.T @ B, "fro") * ZtZ + np.linalg.norm(C @ C.T, "fro"))
    for bad in (dropped, unsquared):
        monkeypatch.setattr(riccati, "paper_res", bad)
        assert abs(riccati.paper_res(A, B, C, Z, 1.0) - expected) > 1e-3 * expected


def test_check_shifts_pin_catches_lenient_sign(monkeypatch):
    """A checker that lets Re p = 0 through (or skips the pairing rule) must
    fail the rejection pins."""
    import pytest as _pt

    def lenient(shifts):
        s = np.asarray(shifts, dtype=np.complex128)
        if s.size == 0 or np.any(s.real > 0):
            raise ValueError("bad")
        return s
    monkeypatch.setattr(adi, "check_shifts", lenient)
    for bad in ([-1.0, 0.0], [-1.0 + 2.0j], [-1.0 - 2.0j, -1.0 + 2.0j]):
        try:
            adi.check_shifts(np.array(bad, dtype=np.complex128))
            caught = False
        except ValueError:
            caught = True
        assert not caught       # the lenient checker accepts what the pins reject
    _pt.raises(ValueError, adi.check_shifts, np.array([1.0]))
