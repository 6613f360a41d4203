"""ILU(0) of the shifted matrices A^T + p I in a multicolour ordering: the
preconditioner of the restarted-GMRES inner solves in Sec. 5 ("Performance
Analysis on GPU").

Test infrastructure only (see the package docstring).

The paper names the preconditioner (incomplete LU without fill) and not the
ordering of the unknowns.  The ordering here is multicolour:

  colouring   first-fit greedy colouring of the undirected graph whose edges
              are the off-diagonal nonzeros of A (in either direction): the
              vertices are visited in their natural order and each takes the
              smallest colour that no already coloured neighbour holds;
  order       the vertices of colour 0 in increasing index, then those of
              colour 1, and so on.

With P the permutation matrix of that order and Mp = P (A^T + p I) P^T,
ILU(0) is the pair (L, U), L unit lower and U upper triangular, both with
nonzeros only on the pattern S of Mp (the nonzeros of A^T plus the
diagonal), such that (L U)_ij = (Mp)_ij for every (i, j) in S.  It is
computed row by row in the usual IKJ form: for row i and each lower
position k of S in increasing order, the multiplier l_ik = m_ik / u_kk is
formed and m_ij -= l_ik u_kj for every later position j of row i that is
also in row k's pattern; positions outside S (the fill) are never formed.

Parity pins: the defining equations above on random patterns, exact LU when
no fill arises (tridiagonal matrices), the closed form of the red-black
block factorisation of a five-point stencil, the properness and first-fit
property of the colouring and its checkerboard on grids."""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl


def greedy_colouring(A):
    """First-fit colours (int32 array) of the vertices 0..n-1 of the graph of
    the off-diagonal nonzeros of A, visited in natural order."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    P = sp.csr_matrix((np.ones(A.nnz), A.indices, A.indptr), shape=A.shape)
    G = (P + P.T).tocsr()
    colours = np.full(n, -1, dtype=np.int64)
    for i in range(n):
        nbrs = G.indices[G.indptr[i]:G.indptr[i + 1]]
        used = {int(colours[j]) for j in nbrs if j != i and colours[j] >= 0}
        c = 0
        while c in used:
            c += 1
        colours[i] = c
    return colours.astype(np.int32)


def colour_order(colours):
    """Vertices sorted by colour, increasing index within a colour."""
    colours = np.asarray(colours)
    return np.lexsort((np.arange(colours.size), colours))


def ilu0(M):
    """ILU(0) of the sparse matrix M on its own pattern plus the diagonal,
    in M's index order.  Returns (L, U) as CSR matrices (L with its unit
    diagonal stored)."""
    M = sp.csr_matrix(M, dtype=np.float64)
    n = M.shape[0]
    rows = []
    for i in range(n):
        sl = slice(M.indptr[i], M.indptr[i + 1])
        r = {int(j): float(v) for j, v in zip(M.indices[sl], M.data[sl])}
        r.setdefault(i, 0.0)
        rows.append(r)
    for i in range(n):
        r = rows[i]
        for k in sorted(j for j in r if j < i):
            r[k] = r[k] / rows[k][k]
            for j, ukj in rows[k].items():
                if j > k and j in r:
                    r[j] -= r[k] * ukj
    li, lj, lv, ui, uj, uv = [], [], [], [], [], []
    for i, r in enumerate(rows):
        for j, v in r.items():
            if j < i:
                li.append(i), lj.append(j), lv.append(v)
            else:
                ui.append(i), uj.append(j), uv.append(v)
    L = sp.csr_matrix((lv, (li, lj)), shape=(n, n)) + sp.identity(n, format="csr")
    U = sp.csr_matrix((uv, (ui, uj)), shape=(n, n))
    return L.tocsr(), U.tocsr()


class ShiftedIlu0:
    """ILU(0) of A^T + p I in the multicolour order of A (real p)."""

    def __init__(self, A, p):
        A = sp.csr_matrix(A, dtype=np.float64)
        n = A.shape[0]
        self.n = n
        self.colours = greedy_colouring(A)
        self.order = colour_order(self.colours)
        self.inv = np.empty(n, dtype=np.int64)
        self.inv[self.order] = np.arange(n)
        M = (A.T + float(p) * sp.identity(n)).tocsr()
        Mp = M[self.order][:, self.order]
        self.L, self.U = ilu0(Mp)

    def apply(self, B):
        """(P^T L U P)^{-1} B for an n x k block (the preconditioner solve)."""
        B = np.asarray(B, dtype=np.float64)
        vec = B.ndim == 1
        Bp = (B[:, None] if vec else B)[self.order]
        Y = spl.spsolve_triangular(self.L, Bp, lower=True, unit_diagonal=True)
        X = spl.spsolve_triangular(self.U, Y, lower=False)
        out = np.empty_like(X)
        out[self.order] = X
        return out[:, 0] if vec else out

    def entries(self, At):
        """Factor values at the positions of A^T's off-diagonal nonzeros in
        row-major order (l_ij where j precedes i in the colour order, u_ij
        otherwise), and the diagonal u_ii, both in the original indexing."""
        At = sp.csr_matrix(At)
        At.sort_indices()
        L, U = self.L.tolil(), self.U.tolil()
        off = []
        for i in range(self.n):
            for j in At.indices[At.indptr[i]:At.indptr[i + 1]]:
                if j == i:
                    continue
                pi, pj = self.inv[i], self.inv[j]
                off.append(L[pi, pj] if pj < pi else U[pi, pj])
        diag = np.array([U[self.inv[i], self.inv[i]] for i in range(self.n)])
        return np.array(off, dtype=np.float64), diag
