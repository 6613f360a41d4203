"""Heuristic ADI shifts from Ritz values (FP64).

Test infrastructure only (see the package docstring).

Sec. 5 says only that the shifts are generated from Krylov subspaces.  The
reading used here is Penzl's heuristic (Penzl, SIAM J. Sci. Comput. 21(4),
2000, Sec. 5), written from its description:

  1. kp Arnoldi steps with F = A^T from b0 = ones / sqrt(n): Ritz values R+,
     the eigenvalues of the kp x kp Hessenberg matrix;
  2. km Arnoldi steps with F^{-1}: Ritz values R-, inverted;
  3. candidates R = R+ and R- that lie in the open left half-plane;
  4. the first shift minimises  max_{t in R} |(t - p) / (t + p)|  over p in R;
     then, while fewer than l0 shifts are chosen, the candidate t where
     s(t, P) = prod_{p in P} |(t - p) / (t + p)|  is largest joins P.
     A complex choice brings its conjugate along (so |P| may reach l0 + 1).

The candidates are taken in lexicographic (Re, Im) order, so that ties (a
Ritz value and its conjugate score alike) resolve the same way everywhere.
A complex pair is stored with Im > 0 first.

The other reading, projection shifts (Benner, Kuerschner and Saak, ETNA 43,
2014), draws each set from a subspace the ADI run itself produces:
projection_shifts below.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl


def arnoldi(apply, b, k):
    """k steps of the Arnoldi process (modified Gram-Schmidt) for the
    operator `apply` from b.  Returns the square Hessenberg matrix H of the
    steps completed (fewer than k if an invariant subspace is met)."""
    n = b.shape[0]
    V = np.zeros((n, k + 1))
    H = np.zeros((k + 1, k))
    V[:, 0] = b / np.linalg.norm(b)
    for j in range(k):
        w = apply(V[:, j])
        for i in range(j + 1):
            H[i, j] = V[:, i] @ w
            w = w - H[i, j] * V[:, i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] <= 1e-12 * np.linalg.norm(H[: j + 2, j]):
            return H[: j + 1, : j + 1]
        V[:, j + 1] = w / H[j + 1, j]
    return H[:k, :k]


def ritz_candidates(A, kp=20, km=10, real_only=False, inv_apply=None):
    """Steps 1-3: stable Ritz values of A^T and inverted Ritz values of A^-T.
    (A and A^T share their spectrum; the ADI operator is A^T.)  inv_apply(v),
    if given, applies A^-T (default: a sparse LU of A^T)."""
    At = sp.csr_matrix(A.T) if sp.issparse(A) else np.asarray(A, dtype=np.float64).T
    n = At.shape[0]
    b0 = np.ones(n) / np.sqrt(n)
    R = list(np.linalg.eigvals(arnoldi(lambda v: At @ v, b0, kp)))
    if km > 0:
        if inv_apply is not None:
            inv = inv_apply
        elif sp.issparse(At):
            lu = spl.splu(sp.csc_matrix(At))
            inv = lu.solve
        else:
            inv = lambda v: np.linalg.solve(At, v)  # noqa: E731
        R += [1.0 / t for t in np.linalg.eigvals(arnoldi(inv, b0, km))]
    R = np.array(R, dtype=np.complex128)
    if real_only:
        R = R.real.astype(np.complex128)
    return R[(R.real < 0) & np.isfinite(R)]


def penzl_select(R, l0):
    """Step 4: greedy min-max choice of l0 shifts among the candidates R."""
    R = np.asarray(R, dtype=np.complex128).ravel()
    R = R[(R.real < 0) & np.isfinite(R)]          # step 3: stable candidates only
    R = R[np.lexsort((R.imag, R.real))]
    if R.size == 0:
        raise ValueError("no stable Ritz values")

    def ratio(t, p):
        return np.abs((t - p) / (t + p))

    first = int(np.argmin([np.max(ratio(R, p)) for p in R]))
    P = []

    def add(p):
        if p.imag != 0.0:
            P.append(complex(p.real, abs(p.imag)))
            P.append(complex(p.real, -abs(p.imag)))
        else:
            P.append(complex(p.real, 0.0))

    add(R[first])
    while len(P) < l0:
        s = np.ones(R.size)
        for p in P:
            s *= ratio(R, p)
        i = int(np.argmax(s))
        if s[i] == 0.0:
            break
        add(R[i])
    return np.array(P, dtype=np.complex128)


def penzl_shifts(A, l0=16, kp=20, km=10, real_only=False, inv_apply=None):
    """Penzl's heuristic shift set for the ADI operator A^T."""
    return penzl_select(ritz_candidates(A, kp, km, real_only, inv_apply), l0)


def projection_shifts(A, V, l0, B=None, K=None, smax=64, rel=1e-10):
    """Projection shifts: the Ritz values of F = A^T - K B^T on span(V).

    1. Q: orthonormal basis of the dominant directions of span(V), the left
       singular vectors of V with sigma^2 > rel * sigma_max^2 (at most smax);
    2. H = Q^T F Q;
    3. its eigenvalues, those in the right half-plane mirrored into the left
       one (t -> -conj(t));
    4. at most l0 of them by the greedy min-max rule (penzl_select).
    B, K: n x m or None."""
    At = A.T
    V = np.asarray(V, dtype=np.float64)
    U, s, _ = np.linalg.svd(V, full_matrices=False)
    keep = s ** 2 > rel * s[0] ** 2
    Q = U[:, keep][:, :smax]
    Y = At @ Q
    if sp.issparse(Y):
        Y = Y.toarray()
    Y = np.asarray(Y)
    if B is not None and K is not None:
        Y = Y - K @ (B.T @ Q)
    H = Q.T @ Y
    theta = np.linalg.eigvals(H).astype(np.complex128)
    theta = np.where(theta.real > 0, -np.conj(theta), theta)
    return penzl_select(theta, l0)
