"""Low-rank factor decompositions (FP64, Householder QR).

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def residual_core_matrix(r, m, p):
    """Signature matrix M of the factored residual R(Z) = F M F^T with
    F = [Z, A^T Z, Z Z^T B, C^T]  (Sec. 2, factored form of eq. (2.2)):
    M = [[0, I_r, 0, 0], [I_r, 0, 0, 0], [0, 0, -I_m, 0], [0, 0, 0, I_p]]."""
    q = 2 * r + m + p
    M = np.zeros((q, q))
    M[:r, r:2 * r] = np.eye(r)
    M[r:2 * r, :r] = np.eye(r)
    M[2 * r:2 * r + m, 2 * r:2 * r + m] = -np.eye(m)
    M[2 * r + m:, 2 * r + m:] = np.eye(p)
    return M


def residual_factor(A, B, C, Z, eta_r_rel=1e-4, full=False):
    """Algorithm 1 (Residual Factor Decomposition).

    1. F = [Z, A^T Z, Z Z^T B, C^T], thin QR F = U T (Householder).
    2. H = T M T^T, spectral decomposition H = Q Lambda Q^T.
    3./4. J+ = {lambda >= eta_r}, J- = {lambda <= -eta_r} with
       eta_r = eta_r_rel * max|lambda(H)| (the relative threshold of Sec. 5).
    5. C+ = U Q(:,J+) Lambda+^(1/2),  C- = U Q(:,J-) (-Lambda-)^(1/2).
    ||R(Z)||_F = ||H||_F from the eigenvalues before truncation (Sec. 2).

    With eta_r_rel = 0 the split follows the untruncated sets of Sec. 2
    (lambda > 0 and lambda < 0; exact zeros contribute nothing).
    Returns (C+, C-, ||R||_F) or, with full=True, a dict of intermediates."""
    Z = np.asarray(Z, dtype=np.float64)
    r = Z.shape[1]
    m = B.shape[1]
    p = C.shape[0]
    AtZ = A.T @ Z
    if sp.issparse(AtZ):
        AtZ = AtZ.toarray()
    F = np.hstack([Z, AtZ, Z @ (Z.T @ B), C.T])
    U, T = np.linalg.qr(F, mode="reduced")
    M = residual_core_matrix(r, m, p)
    H = T @ M @ T.T
    H = 0.5 * (H + H.T)
    lam, Q = np.linalg.eigh(H)
    res_fro = float(np.sqrt(np.sum(lam ** 2)))
    eta = eta_r_rel * (np.max(np.abs(lam)) if lam.size else 0.0)
    if eta > 0:
        Jp, Jm = lam >= eta, lam <= -eta
    else:
        Jp, Jm = lam > 0, lam < 0
    Cp = (U @ Q[:, Jp]) * np.sqrt(lam[Jp])
    Cm = (U @ Q[:, Jm]) * np.sqrt(-lam[Jm])
    if full:
        return dict(Cp=Cp, Cm=Cm, res_fro=res_fro, lam=lam, eta=eta, F=F, U=U, T=T, H=H)
    return Cp, Cm, res_fro


def solution_factor(Z, Zp, Zm, eta_s_rel=10 * np.finfo(np.float64).eps / 2, full=False):
    """Algorithm 2 (Solution Factor Decomposition).

    1. G = [Z, Z+, Z-], thin QR G = V Gamma (Householder).
    2. P = Gamma N Gamma^T with N = diag(I, I, -I); P = Theta Sigma Theta^T.
    3. J+ = {sigma >= eta_s}, eta_s = eta_s_rel * max|sigma(P)|  (Sec. 5 uses
       eta_s = 10 u max|lambda(P)| with u the FP64 unit roundoff).
    4. Z_new = V Theta(:,J+) Sigma+^(1/2).
    Also reports eta_n = ||P-||_F / ||P||_F (Lemma 1).
    Returns Z_new or, with full=True, a dict."""
    blocks = [np.asarray(b, dtype=np.float64) for b in (Z, Zp, Zm)]
    sign = np.concatenate([np.ones(blocks[0].shape[1]), np.ones(blocks[1].shape[1]),
                           -np.ones(blocks[2].shape[1])])
    G = np.hstack(blocks)
    return signed_truncate(G, sign, eta_s_rel, full=full)


def signed_truncate(G, sign, eta_s_rel, full=False):
    """Steps 1-4 of Algorithm 2 for a general signature N = diag(sign)."""
    V, Gam = np.linalg.qr(G, mode="reduced")
    P = (Gam * sign) @ Gam.T
    P = 0.5 * (P + P.T)
    sig, Th = np.linalg.eigh(P)
    eta = eta_s_rel * (np.max(np.abs(sig)) if sig.size else 0.0)
    J = sig >= eta if eta > 0 else sig > 0
    Znew = (V @ Th[:, J]) * np.sqrt(sig[J])
    nP = np.sqrt(np.sum(sig ** 2))
    eta_n = float(np.sqrt(np.sum(sig[sig < 0] ** 2)) / nP) if nP > 0 else 0.0
    if full:
        return dict(Z=Znew, sig=sig, eta=eta, eta_n=eta_n, V=V, Gam=Gam, P=P)
    return Znew


def factored_diff_norm(Z, Y):
    """||Z Z^T - Y Y^T||_F without forming n x n matrices and without the
    cancellation of the trace expansion: [Z, Y] = U [T1, T2] (Householder),
    then ||Z Z^T - Y Y^T||_F = ||T1 T1^T - T2 T2^T||_F."""
    Z = np.asarray(Z, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    if Z.shape[1] + Y.shape[1] == 0:
        return 0.0
    _, T = np.linalg.qr(np.hstack([Z, Y]), mode="reduced")
    T1, T2 = T[:, :Z.shape[1]], T[:, Z.shape[1]:]
    return float(np.linalg.norm(T1 @ T1.T - T2 @ T2.T, "fro"))


def factored_norm(Z):
    """||Z Z^T||_F = ||Z^T Z||_F."""
    Z = np.asarray(Z, dtype=np.float64)
    return float(np.linalg.norm(Z.T @ Z, "fro"))


def residual_norm(A, B, C, Z):
    """||R(Z Z^T)||_F via Algorithm 1's core matrix (no truncation)."""
    return residual_factor(A, B, C, Z, eta_r_rel=0.0)[2]
