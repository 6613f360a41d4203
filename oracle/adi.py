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
import time

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
        # work counters (no effect on the arithmetic): factorizations done and
        # columns solved, with the seconds spent in each
        self.counts = dict(factorizations=0, factor_s=0.0, columns=0, solve_s=0.0)

    def _factor(self, p):
        key = complex(p)
        if key not in self._lu:
            t0 = time.perf_counter()
            self.counts["factorizations"] += 1
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
            self.counts["factor_s"] += time.perf_counter() - t0
        return self._lu[key]

    def solve_base(self, p, W):
        """M^{-1} W with M = A^T + p I (no feedback term)."""
        solve = self._factor(p)
        Wd = np.asarray(W, dtype=np.complex128 if complex(p).imag != 0 else np.float64)
        t0 = time.perf_counter()
        if Wd.ndim == 1:
            out = solve(Wd)
        elif Wd.shape[1]:
            out = np.column_stack([solve(Wd[:, j]) for j in range(Wd.shape[1])])
        else:
            out = np.zeros((self.n, 0), dtype=Wd.dtype)
        self.counts["columns"] += 1 if Wd.ndim == 1 else Wd.shape[1]
        self.counts["solve_s"] += time.perf_counter() - t0
        return out

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


class KronZShiftedSolver(ShiftedSolver):
    """The shifted solves of ShiftedSolver for an operator with the Kronecker
    structure  A = I_Nz (x) A_p + T (x) I_Np  (plane operator A_p of order Np,
    symmetric Nz x Nz coupling T between planes; planes are the slowest index):
    the 3D convection-diffusion matrix with a field that has no z-component.

    With T = S diag(mu) S^T (library eigh, S orthogonal),
      (A^T + p I) = (S (x) I) (I (x) A_p^T + diag(mu) (x) I + p I) (S^T (x) I),
    so one shifted solve is a transform along z, Nz independent sparse LU
    solves of order Np with the shifts mu_k + p, and the inverse transform: an
    exact direct solve (up to rounding) at a fraction of the fill of a 3D LU.
    The per-plane factorizations are cached per shift in `cache` (a dict that
    several solvers of one problem may share; they do not depend on K)."""

    def __init__(self, A, B=None, K=None, planes=None, cache=None):
        super().__init__(A, B, K)
        self.Ap, self.T = kron_z_split(A, planes)
        self.nz = self.T.shape[0]
        self.npl = self.Ap.shape[0]
        self.mu, self.S = np.linalg.eigh(self.T)
        self.ApT = sp.csc_matrix(self.Ap.T)
        self._plane_lu = {} if cache is None else cache

    def _plane_factors(self, p):
        key = complex(p)
        if key not in self._plane_lu:
            cplx = key.imag != 0
            dt = np.complex128 if cplx else np.float64
            pv = key if cplx else key.real
            I = sp.identity(self.npl, dtype=dt, format="csc")
            self._plane_lu[key] = [spl.splu((self.ApT.astype(dt) + (self.mu[k] + pv) * I).tocsc())
                                   for k in range(self.nz)]
        return self._plane_lu[key]

    def solve_base(self, p, W):
        lus = self._plane_factors(p)
        cplx = complex(p).imag != 0
        Wd = np.asarray(W, dtype=np.complex128 if cplx else np.float64)
        one = Wd.ndim == 1
        Wd = Wd.reshape(self.n, -1)
        w = Wd.shape[1]
        Y = np.einsum("zk,zpw->kpw", self.S, Wd.reshape(self.nz, self.npl, w))   # S^T along z
        for k in range(self.nz):
            Y[k] = lus[k].solve(np.ascontiguousarray(Y[k]))
        V = np.einsum("zk,kpw->zpw", self.S, Y).reshape(self.n, w)              # S along z
        return V[:, 0] if one else V


def kron_z_split(A, planes=None):
    """Split A = I_Nz (x) A_p + T (x) I_Np exactly (A sparse, planes = Np;
    default: the plane size of a cubic grid, n^(2/3)).  A_p is the diagonal
    block of the first plane minus T's diagonal; T holds the couplings
    between planes, which must be multiples of the identity (checked: the
    reassembled matrix must equal A entry for entry, else ValueError)."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    if planes is None:
        N = int(round(n ** (1.0 / 3.0)))
        planes = N * N
    if n % planes:
        raise ValueError("plane size does not divide n")
    nz = n // planes
    T = np.zeros((nz, nz))
    for a in range(nz):
        for b in range(max(0, a - 1), min(nz, a + 2)):
            if a != b:
                blk = A[a * planes:(a + 1) * planes, b * planes:(b + 1) * planes]
                T[a, b] = blk[0, 0]
    # the diagonal of T (the share of A's diagonal that belongs to the
    # coupling between planes): the second difference along z has rows that
    # sum to zero in the interior, T[a, a] = -(T[a, a-1] + T[a, a+1]), and the
    # same value on the boundary planes (Dirichlet)
    if nz > 2:
        tdiag = -(T[1, 0] + T[1, 2])
    elif nz == 2:
        tdiag = -2.0 * T[0, 1]
    else:
        tdiag = 0.0
    np.fill_diagonal(T, tdiag)
    Ap = (A[:planes, :planes] - tdiag * sp.identity(planes)).tocsr()
    R = (sp.kron(sp.identity(nz), Ap) + sp.kron(sp.csr_matrix(T), sp.identity(planes)) - A).tocsr()
    R.eliminate_zeros()
    if R.nnz and abs(R).max() > 1e-12 * abs(A).max():
        raise ValueError("A is not of the form I (x) A_p + T (x) I")
    if not np.allclose(T, T.T, rtol=0, atol=0):
        raise ValueError("plane coupling T is not symmetric")
    return Ap, T


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
