"""Dense Riccati references (FP64).

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def _dense(A):
    return A.toarray() if sp.issparse(A) else np.asarray(A, dtype=np.float64)


def riccati_residual(A, B, C, X):
    """Riccati operator R(X) = A^T X + X A - X B B^T X + C^T C  (Sec. 2, the
    operator whose Frechet derivative gives the Newton correction)."""
    A = _dense(A)
    XB = X @ B
    return A.T @ X + X @ A - XB @ XB.T + C.T @ C


def care_schur(A, B, C):
    """Stabilizing solution by the Hamiltonian Schur method (Laub, cited in
    Sec. 1) - SciPy's library routine with R = I_m, Q = C^T C."""
    A = _dense(A)
    m = B.shape[1]
    return sla.solve_continuous_are(A, B, C.T @ C, np.eye(m))


def lyap_bartels_stewart(F, Q):
    """Solve F X + X F^T = Q (Bartels-Stewart, SciPy library routine)."""
    return sla.solve_continuous_lyapunov(F, Q)


def newton_kleinman_dense(A, B, C, X0=None, tol=1e-14, kmax=60, stagnation=0.999):
    """Dense Newton iteration for the CARE (Sec. 2): X_{k+1} = X_k + Y_k with
    (A - B B^T X_k)^T Y_k + Y_k (A - B B^T X_k) = -R(X_k)  (eq. (2.1)).

    Written in the equivalent Kleinman form
        A_k^T X_{k+1} + X_{k+1} A_k = -(C^T C + X_k B B^T X_k),  A_k = A - B B^T X_k,
    each step solved by Bartels-Stewart.  X_0 = 0 needs A stable.
    Returns (X, history of ||R||_F / ||C^T C||_F)."""
    A = _dense(A)
    n = A.shape[0]
    X = np.zeros((n, n)) if X0 is None else np.array(X0, dtype=np.float64)
    CtC = C.T @ C
    nrm = np.linalg.norm(CtC, "fro")
    hist = []
    prev = None
    for _ in range(kmax):
        K = X @ B
        Ak = A - B @ K.T
        Xn = lyap_bartels_stewart(Ak.T, -(CtC + K @ K.T))
        X = 0.5 * (Xn + Xn.T)
        res = np.linalg.norm(riccati_residual(A, B, C, X), "fro") / nrm
        hist.append(res)
        if res <= tol:
            break
        if prev is not None and res / prev > stagnation:
            break
        prev = res
    return X, hist


def paper_res(A, B, C, Z, res_fro):
    """The paper's reported relative residual "Res" (Sec. 5):
    ||R||_F / (2 ||A||_F ||Z^T Z||_F + ||B^T B||_F ||Z^T Z||_F^2 + ||C C^T||_F)."""
    if sp.issparse(A):
        nA = sp.linalg.norm(A, "fro")
    else:
        nA = np.linalg.norm(A, "fro")
    ZtZ = np.linalg.norm(Z.T @ Z, "fro")
    den = 2 * nA * ZtZ + np.linalg.norm(B.T @ B, "fro") * ZtZ ** 2 + np.linalg.norm(C @ C.T, "fro")
    return res_fro / den


def care_hamiltonian(A, B, C):
    """Stabilizing solution from the stable invariant subspace of the
    Hamiltonian matrix (Laub's Schur method, the family cited in Sec. 1):

        H = [[A, -B B^T], [-C^T C, -A^T]],   H [I; X] = [I; X] (A - B B^T X),

    so an ordered real Schur form H U = U T with the n eigenvalues of negative
    real part first gives span [U11; U21] = span [I; X] and X = U21 U11^{-1}.
    A library Schur decomposition of the 2n x 2n matrix (no generalized QZ):
    much faster than ``care_schur`` at n in the thousands."""
    A = _dense(A)
    n = A.shape[0]
    H = np.block([[A, -B @ B.T], [-C.T @ C, -A.T]])
    _, U, sdim = sla.schur(H, output="real", sort="lhp")
    if sdim != n:
        raise ValueError(f"Hamiltonian has {sdim} stable eigenvalues, expected {n}")
    U11, U21 = U[:n, :n], U[n:, :n]
    X = np.linalg.solve(U11.T, U21.T).T
    return 0.5 * (X + X.T)
