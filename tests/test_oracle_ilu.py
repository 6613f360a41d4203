"""Pins of the oracle's multicolour ILU(0) (the preconditioner of the
restarted-GMRES inner solves, Sec. 5 "Performance Analysis on GPU") against
facts fixed by its definition and by textbook cases:

* the defining equations (L U)_ij = m_ij on the pattern, with L and U on the
  pattern, for random nonsymmetric patterns;
* no fill (tridiagonal): ILU(0) is the exact LU;
* the red-black five-point stencil: the closed form of its block
  factorisation (multipliers a_ik / (d + p), black pivots
  d + p - sum_k a_ik a_ki / (d + p));
* the colouring: proper, first-fit, a checkerboard on grids, i mod 4 on the
  Toeplitz band, n colours on a complete graph;
* the preconditioner solve against the explicitly formed P^T L U P.
A planted mistake (row k of M instead of the factored row k) must fail the
defining-equation pin."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import workloads as wl
from oracle import ilu

RNG = np.random.default_rng(23)


def random_pattern(n, density, seed):
    R = sp.random(n, n, density=density, random_state=np.random.RandomState(seed))
    R = (R - 0.4 * R.T).tocsr()
    d = np.asarray(abs(R).sum(axis=1)).ravel() + 1.0
    return (R - sp.diags(d)).tocsr()


def defining_error(A, p):
    """max over the pattern S of |(L U)_ij - m_ij| / max|m|, plus whether L
    and U stay on S."""
    f = ilu.ShiftedIlu0(A, p)
    n = A.shape[0]
    M = (sp.csr_matrix(A).T + p * sp.identity(n)).tocsr()
    Mp = M[f.order][:, f.order].tocoo()
    S = set(zip(Mp.row.tolist(), Mp.col.tolist())) | {(i, i) for i in range(n)}
    LU = (f.L @ f.U).toarray()
    Md = Mp.toarray()
    err = max(abs(LU[i, j] - Md[i, j]) for (i, j) in S) / abs(Md).max()
    on_pattern = all((i, j) in S for i, j in zip(*f.L.nonzero())) and \
        all((i, j) in S for i, j in zip(*f.U.nonzero()))
    lower = np.all(np.triu(f.L.toarray(), 1) == 0) and np.allclose(np.diag(f.L.toarray()), 1.0)
    upper = np.all(np.tril(f.U.toarray(), -1) == 0)
    return err, on_pattern and lower and upper, f, LU, Md


@pytest.mark.parametrize("n,density,seed", [(12, 0.3, 1), (40, 0.12, 2), (90, 0.05, 3)])
def test_ilu0_satisfies_its_defining_equations(n, density, seed):
    A = random_pattern(n, density, seed)
    err, structure, f, LU, Md = defining_error(A, -0.7)
    assert structure
    assert err <= 1e-13
    # incomplete: some fill position of the exact LU is nonzero (dense enough patterns)
    if n >= 40:
        assert np.abs(LU - Md).max() > 1e-8


def test_ilu0_is_exact_lu_without_fill():
    """A tridiagonal matrix in its natural order has no fill: ILU(0) is the LU
    factorisation, here the one LAPACK's getrf returns (column diagonal
    dominance, so partial pivoting exchanges no rows)."""
    n = 25
    M = sp.diags([RNG.uniform(0.1, 1, n - 1), -RNG.uniform(3, 4, n), RNG.uniform(0.1, 1, n - 1)],
                 [-1, 0, 1], format="csr")
    L, U = ilu.ilu0(M)
    P, Lr, Ur = sla.lu(M.toarray())
    assert np.array_equal(P, np.eye(n))
    assert np.abs(L.toarray() - Lr).max() <= 1e-14
    assert np.abs(U.toarray() - Ur).max() <= 1e-14 * np.abs(Ur).max()
    # in the red-black order of the same matrix the exact LU fills in, ILU(0) does not
    f = ilu.ShiftedIlu0(M.T, 0.0)
    assert list(f.colours) == [i % 2 for i in range(n)]
    Mp = M.toarray()[np.ix_(f.order, f.order)]
    assert np.abs((f.L @ f.U).toarray() - Mp).max() > 1e-3


def test_ilu0_red_black_five_point_closed_form():
    N = 7
    A = wl.fdm2d(N, 10.0)
    n = N * N
    p = -3.0
    At = A.T.tocsr()
    d = A.diagonal()[0]
    assert np.all(A.diagonal() == d)
    f = ilu.ShiftedIlu0(A, p)
    ix, iy = np.arange(n) % N, np.arange(n) // N
    assert np.array_equal(f.colours, (ix + iy) % 2)
    off, diag = f.entries(At)
    # expected, in the same row-major order of A^T's off-diagonal entries
    exp_off, exp_diag = [], np.full(n, d + p)
    for i in range(n):
        for e in range(At.indptr[i], At.indptr[i + 1]):
            k = At.indices[e]
            if k == i:
                continue
            if f.colours[i] == 1:          # black row: multiplier of a red neighbour
                exp_off.append(At.data[e] / (d + p))
                exp_diag[i] -= At.data[e] * At[k, i] / (d + p)
            else:                          # red row: U row = the row of M
                exp_off.append(At.data[e])
    assert np.allclose(off, exp_off, rtol=1e-14, atol=0)
    assert np.allclose(diag, exp_diag, rtol=1e-14, atol=0)


def test_colouring_is_proper_and_first_fit():
    for A in (random_pattern(60, 0.08, 4), wl.fdm3d(4), wl.toeplitz5(30)):
        A = sp.csr_matrix(A)
        c = ilu.greedy_colouring(A)
        G = (abs(A) + abs(A.T)).tocsr()
        for i in range(A.shape[0]):
            nb = [j for j in G.indices[G.indptr[i]:G.indptr[i + 1]] if j != i]
            assert all(c[j] != c[i] for j in nb)                      # proper
            earlier = {c[j] for j in nb if j < i}
            assert c[i] == min(set(range(len(nb) + 2)) - earlier)    # first fit
    assert list(ilu.greedy_colouring(wl.toeplitz5(17))) == [i % 4 for i in range(17)]
    K = sp.csr_matrix(np.ones((6, 6)))
    assert list(ilu.greedy_colouring(K)) == list(range(6))
    assert list(ilu.greedy_colouring(sp.identity(5, format="csr"))) == [0] * 5


def test_preconditioner_solve_inverts_the_factor_product():
    A = random_pattern(50, 0.1, 6)
    f = ilu.ShiftedIlu0(A, -0.9)
    P = np.eye(50)[f.order]
    Mt = P.T @ (f.L @ f.U).toarray() @ P
    B = RNG.standard_normal((50, 4))
    X = f.apply(B)
    assert np.abs(Mt @ X - B).max() <= 1e-12 * np.abs(B).max() * np.linalg.cond(Mt)
    assert np.allclose(f.apply(B[:, 0]), X[:, 0], rtol=1e-15, atol=0)


def test_defining_pin_catches_unfactored_rows(monkeypatch):
    A = random_pattern(40, 0.12, 2)
    assert defining_error(A, -0.7)[0] <= 1e-13

    def wrong(M):
        # plausible mistake: updates use row k of M itself, not the factored row k
        M = sp.csr_matrix(M, dtype=np.float64)
        n = M.shape[0]
        orig = [dict(zip(M.indices[M.indptr[i]:M.indptr[i + 1]].tolist(), M.data[M.indptr[i]:M.indptr[i + 1]]))
                for i in range(n)]
        rows = [dict(r) for r in orig]
        for i in range(n):
            r = rows[i]
            for k in sorted(j for j in r if j < i):
                r[k] = r[k] / rows[k][k]
                for j, mkj in orig[k].items():
                    if j > k and j in r:
                        r[j] -= r[k] * mkj
        L = sp.lil_matrix((n, n))
        U = sp.lil_matrix((n, n))
        for i, r in enumerate(rows):
            for j, v in r.items():
                (L if j < i else U)[i, j] = v
        return (L + sp.identity(n)).tocsr(), U.tocsr()
    monkeypatch.setattr(ilu, "ilu0", wrong)
    assert defining_error(A, -0.7)[0] > 1e-6
