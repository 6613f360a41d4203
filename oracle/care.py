"""NLR-ADI initial solve and Framework 1 (FP64 everywhere).

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

import numpy as np

from . import adi, lowrank

U64 = np.finfo(np.float64).eps / 2      # FP64 unit roundoff (Table 1)


def nlradi(A, B, C, shifts, tol=1e-13, kmax=20, adi_tol=1e-13, jmax=100, stagnation=0.999,
           compress_rel=10 * U64, solver_factory=None):
    """Initial CARE approximation by Newton-Kleinman with LR-ADI inner solves
    (NLR-ADI, Sec. 4):  with K_0 = 0 (A stable), step i solves
        A_i^T X_{i+1} + X_{i+1} A_i = -[C^T, K_i] [C^T, K_i]^T,  A_i = A - B K_i^T,
    by LR-ADI, then K_{i+1} = Z_{i+1} (Z_{i+1}^T B).  The loop stops when
    ||R(Z)||_F <= tol ||C^T C||_F, when the residual ratio exceeds
    `stagnation`, or after kmax steps.  The final factor is compressed with
    Algorithm 2 (signature +I) at the relative threshold compress_rel.
    solver_factory(A, B, K), if given, builds the shifted solver of each
    Lyapunov equation (default: adi.ShiftedSolver).  Returns (Z, info)."""
    n = A.shape[0]
    m = B.shape[1]
    nrm = np.linalg.norm(C @ C.T, "fro")
    K = np.zeros((n, m))
    hist, inner = [], 0
    Z = None
    prev = None
    for i in range(kmax):
        W0 = C.T if i == 0 else np.hstack([C.T, K])
        Ki = K if i else None
        solver = solver_factory(A, B, Ki) if solver_factory else None
        Z, _, info = adi.lradi(A, B, Ki, W0, shifts, adi_tol, jmax, solver=solver)
        inner += info["steps"]
        K = Z @ (Z.T @ B)
        res = lowrank.residual_norm(A, B, C, Z) / nrm
        hist.append(res)
        if res <= tol:
            break
        if prev is not None and res / prev > stagnation:
            break
        prev = res
    Zc = lowrank.signed_truncate(Z, np.ones(Z.shape[1]), compress_rel)
    return Zc, dict(outer=len(hist), inner=inner, hist=hist)


def framework1(A, B, C, shifts, tol=1e-10, kmax=20, eta_r_rel=1e-4, eta_s_rel=10 * U64,
               tau_L=1e-12, jmax=50, stagnation=0.999, Z1=None, stage0=None, solver_factory=None):
    """Framework 1 (Factorization-based Mixed Precision Newton Iterative
    Refinement), all precisions FP64 here:

      Z_1 from NLR-ADI (or given);  for k = 1..kmax:
        (C+, C-, ||R||_F) = Algorithm 1 (Z_k);
        stop if ||R||_F <= tol ||C^T C||_F  (or stagnation, Sec. 5);
        solve A_k^T X^+- + X^+- A_k + C+- C+-^T = 0 by one LR-ADI run on the
        combined right-hand side [C+, C-] (Sec. 4), A_k = A - B (Z_k Z_k^T B)^T;
        Z_{k+1} = Algorithm 2 (Z_k, Z+, Z-).
    solver_factory as in nlradi.  Returns (Z, info) with the paper's
    outer(inner) counts."""
    nrm = np.linalg.norm(C @ C.T, "fro")      # = ||C^T C||_F
    if Z1 is None:
        Z, info0 = nlradi(A, B, C, shifts, solver_factory=solver_factory, **(stage0 or {}))
    else:
        Z, info0 = np.asarray(Z1, dtype=np.float64), dict(outer=0, inner=0, hist=[])
    hist, inner, outer = [], 0, 0
    prev = None
    stagnated = False
    for k in range(kmax):
        Cp, Cm, res = lowrank.residual_factor(A, B, C, Z, eta_r_rel)
        outer += 1
        hist.append(res / nrm)
        if res <= tol * nrm:
            break
        if prev is not None and res / prev > stagnation:
            stagnated = True
            break
        prev = res
        K = Z @ (Z.T @ B)
        W0 = np.hstack([Cp, Cm])
        solver = solver_factory(A, B, K) if solver_factory else None
        Zpm, _, info = adi.lradi(A, B, K, W0, shifts, tau_L, jmax, solver=solver)
        inner += info["steps"]
        Zp, Zm = adi.split_columns(Zpm, W0.shape[1], Cp.shape[1])
        Z = lowrank.solution_factor(Z, Zp, Zm, eta_s_rel)
    return Z, dict(iter0=(info0["outer"], info0["inner"]), iter=(outer, inner), hist=hist,
                   hist0=info0["hist"], rank=Z.shape[1], stagnated=stagnated)
