"""Shifted solves and residual-based low-rank ADI (FP64, sparse direct).

Test infrastructure only (see the package docstring).

The paper uses LR-ADI as its inner Lyapunov solver without printing it
(Sec. 4 and Sec. 5 cite the NLR-ADI/LR-ADI family).  The recurrence below is
the residual-based LR-ADI of that family, written from its mathematics:

  for  F X + X F^T + W0 W0^T = 0,  F = A_k^T,  A_k = A - B K^T:
  real shift p:     V = (F + p I)^{-1} W,  W <- W - 2 p V,  Z <- [Z, sqrt(-2p) V]
  complex pair (p, conj p), delta = Re p / Im p:
                    V = (F + p I)^{-1} W  (complex),  Vh = Re V + delta Im V,
                    W <- W - 4 Re(p) Vh,
                    Z <- [Z, sqrt(2) g Vh, sqrt(2) g sqrt(delta^2 + 1) Im V],  g = sqrt(-2 Re p)
  Lyapunov residual after each step: F Z Z^T + Z Z^T F^T + W0 W0^T = W W^T,
  so ||residual||_F = ||W^T W||_F.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl


class ShiftedSolver:
    """Applies (A_k^T + p I)^{-1} with A_k = A - B K^T through the
    Sherman-Morrison-Woodbury formula of Sec. 4:

      (A_k + p I)^{-T} = M^{-1} + M^{-1} K (I_m - B^T M^{-1} K)^{-1} B^T M^{-1},
      M = (A + p I)^T,

    i.e. solve M [Vh, S] = [W, K], T = I_m - B^T S, V = Vh + S T^{-1} (B^T Vh).
    M^{-1} is a sparse LU (SuperLU) cached per distinct shift; M^{-1} K and
    T are cached per shift too (K is fixed for one Lyapunov equation)."""

    def __init__(self, A, B=None, K=None):
        self.At = sp.csc_matrix(A.T) if sp.issparse(A) else np.asarray(A, dtype=np.float64).T.copy()
        self.sparse = sp.issparse(A)
        self.n = self.At.shape[0]
        self.B = None if B is None else np.asarray(B, dtype=np.float64)
        self.K = None if K is None else np.asarray(K, dtype=np.float64)
        if self.K is not None and not np.any(self.K):
            self.K = None
        self._lu = {}
        self._smw = {}

    def _factor(self, p):
        key = complex(p)
        if key not in self._lu:
            if self.sparse:
                dt = np.complex128 if key.imag != 0 else np.float64
                pv = key if key.imag != 0 else key.real
                M = (self.At.astype(dt) + pv * sp.identity(self.n, dtype=dt, format="csc")).tocsc()
                lu = spl.splu(M)
                self._lu[key] = lu.solve
            else:
                import scipy.linalg as sla
                pv = key if key.imag != 0 else key.real
                M = self.At + pv * np.eye(self.n)
                f = sla.lu_factor(M)
                self._lu[key] = lambda rhs, f=f: sla.lu_solve(f, rhs)
        return self._lu[key]

    def solve_base(self, p, W):
        """M^{-1} W with M = A^T + p I (no feedback term)."""
        solve = self._factor(p)
        Wd = np.asarray(W, dtype=np.complex128 if complex(p).imag != 0 else np.float64)
        if Wd.ndim == 1:
            return solve(Wd)
        return np.column_stack([solve(Wd[:, j]) for j in range(Wd.shape[1])]) if Wd.shape[1] else \
            np.zeros((self.n, 0), dtype=Wd.dtype)

    def solve(self, p, W):
        """(A_k^T + p I)^{-1} W via SMW."""
        Vh = self.solve_base(p, W)
        if self.K is None:
            return Vh
        key = complex(p)
        if key not in self._smw:
            S = self.solve_base(p, self.K)
            T = np.eye(self.K.shape[1]) - self.B.T @ S
            self._smw[key] = (S, T)
        S, T = self._smw[key]
        return Vh + S @ np.linalg.solve(T, self.B.T @ Vh)


def check_shifts(shifts):
    """Shifts must have negative real part; complex ones come as adjacent
    conjugate pairs with positive imaginary part first."""
    s = np.asarray(shifts, dtype=np.complex128)
    if s.size == 0 or np.any(s.real >= 0):
        raise ValueError("shifts must be non-empty with Re(p) < 0")
    i = 0
    while i < s.size:
        if s[i].imag != 0:
            if s[i].imag < 0 or i + 1 >= s.size or s[i + 1] != np.conj(s[i]):
                raise ValueError("complex shifts must come as (p, conj(p)) with Im(p) > 0 first")
            i += 2
        else:
            i += 1
    return s


def lradi(A, B, K, W0, shifts, tol=1e-12, jmax=50, solver=None):
    """Residual-based LR-ADI for  A_k^T X + X A_k + W0 W0^T = 0,  A_k = A - B K^T
    (the inner Lyapunov solver of Sec. 4; recurrence in the module docstring).

    Shifts are cycled when more steps than shifts are needed; a complex pair
    counts as two steps.  Stops when ||W^T W||_F <= tol ||W0^T W0||_F or after
    jmax steps.  Returns (Z, W, info) where column block j of Z has the same
    column order as W0 (so columns coming from distinct W0 columns can be
    separated, Sec. 4's combined right-hand side)."""
    s = check_shifts(shifts)
    W = np.array(W0, dtype=np.float64, copy=True)
    w = W.shape[1]
    solver = solver or ShiftedSolver(A, B, K)
    nrm0 = np.linalg.norm(W.T @ W, "fro")
    blocks = []
    hist = []
    j = 0
    i = 0
    if nrm0 == 0 or w == 0:
        return np.zeros((W.shape[0], 0)), W, dict(steps=0, hist=hist, res0=nrm0)
    while j < jmax:
        p = s[i % s.size]
        if p.imag == 0:
            pr = p.real
            V = solver.solve(pr, W).real
            W = W - 2.0 * pr * V
            blocks.append(math.sqrt(-2.0 * pr) * V)
            j += 1
            i += 1
        else:
            V = solver.solve(p, W)
            delta = p.real / p.imag
            Vh = V.real + delta * V.imag
            W = W - 4.0 * p.real * Vh
            g = math.sqrt(-2.0 * p.real)
            blocks.append(math.sqrt(2.0) * g * Vh)
            blocks.append(math.sqrt(2.0) * g * math.sqrt(delta * delta + 1.0) * V.imag)
            j += 2
            i += 2
        res = np.linalg.norm(W.T @ W, "fro")
        hist.append(res / nrm0)
        if res <= tol * nrm0:
            break
    Z = np.hstack(blocks)
    return Z, W, dict(steps=j, hist=hist, res0=nrm0, w=w)


def split_columns(Z, w, first):
    """Split an LR-ADI factor computed for W0 = [W1, W2] (W1 with `first`
    columns, w columns in total) into the factors belonging to W1 and W2:
    ADI acts column-wise on W0, so every block of w columns keeps that order."""
    nb = Z.shape[1] // w if w else 0
    idx1 = np.concatenate([np.arange(b * w, b * w + first) for b in range(nb)]) if nb else np.zeros(0, int)
    idx2 = np.concatenate([np.arange(b * w + first, (b + 1) * w) for b in range(nb)]) if nb else np.zeros(0, int)
    return Z[:, idx1], Z[:, idx2]
