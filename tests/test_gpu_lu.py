"""The batched dense LU of the shifted matrices A^T + p I and its triangular
solves (the direct shifted solves of the dense problems, Sec. 5.1; one
factorisation per shift serves every Newton step under the SMW form of
Sec. 4), called through the C ABI.

Checks: the row order is a permutation; partial pivoting bounds |L| by 1; the
backward error ||P M - L U|| sits at the rounding level of the precision; in
FP64 the pivots and factors agree with LAPACK's getrf (scipy's lu_factor);
solves agree with the oracle's shifted solver (FP64 LU) within the
precision's kappa u bound and leave a residual at its rounding level; a zero
pivot is reported as getrf reports it."""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as wl
from oracle import adi as oadi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

U = {"fp32": 2.0 ** -24, "fp64": 2.0 ** -53}
DT = {"fp32": torch.float32, "fp64": torch.float64}


@pytest.fixture(scope="module")
def pk():
    import paper_2607_14742_amd as pk
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pk.load()
    return pk


@pytest.fixture(scope="module")
def ctx(pk):
    c = pk.Context(0)
    yield c
    c.close()


def factors(F):
    """Unit lower L and upper U of one n x n factor as returned (column-major)."""
    A = F.T.double().cpu().numpy()
    return np.tril(A, -1) + np.eye(A.shape[0]), np.triu(A)


def perm_from_piv(piv):
    perm = np.arange(piv.size)
    for i, p in enumerate(piv):
        perm[[i, p]] = perm[[p, i]]
    return perm


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("n", [1, 5, 16, 17, 100, 257, 1000, 2048])
def test_lu_factor_backward_error_and_pivot_growth(pk, ctx, prec, n):
    print(f"LU factor {prec} n={n}", flush=True)
    rng = np.random.default_rng(100 + n)
    M0 = rng.standard_normal((n, n))
    shifts = [-1.0, -0.25 * n, 3.5]
    M0d = torch.as_tensor(M0, device="cuda")
    F, perm, info = pk.shifted_lu_factor(ctx, M0d, shifts, prec=prec)
    assert info == [0, 0, 0]
    M0r = M0d.to(DT[prec]).double().cpu().numpy()      # the input as the kernel sees it
    for s, p in enumerate(shifts):
        M = M0r + float(np.asarray(p, dtype=np.float32 if prec == "fp32" else np.float64)) * np.eye(n)
        pr = perm[s].cpu().numpy()
        assert sorted(pr.tolist()) == list(range(n))
        L, Uf = factors(F[s])
        assert np.abs(L).max() <= 1.0 + 1e-6
        E = M[pr] - L @ Uf
        bound = 2.0 * n * U[prec] * np.linalg.norm(np.abs(L) @ np.abs(Uf))
        err = np.linalg.norm(E)
        print(f"  shift {p}: ||PM - LU||_F {err:.3e}  bound {bound:.3e}", flush=True)
        assert err <= bound
        if prec == "fp64" and n <= 1000:
            # same pivots as LAPACK getrf (random Gaussian matrices have no ties)
            lu, piv = sla.lu_factor(M)
            assert np.array_equal(pr, perm_from_piv(piv))
            Fh = F[s].T.cpu().numpy()
            assert np.linalg.norm(Fh - lu) <= 1e-12 * n * np.linalg.norm(lu)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("n,q", [(256, 2.0), (300, 2.0), (600, 3.0), (2048, 2.0)])
def test_lu_solve_matches_oracle_shifted_solver(pk, ctx, prec, n, q):
    """(A^T + p I) X = W for the dense test family of Sec. 5.1
    (A = -Q diag(logspace(0, q, n)) Q^T), every shift of a logspaced set,
    k = 1, 4, 5 and 13 right-hand sides (whole and ragged column groups)."""
    print(f"LU solve {prec} n={n} q={q}", flush=True)
    rng = np.random.default_rng(7 + n)
    Q = wl.haar_orthogonal(n, rng)
    A = -(Q * np.logspace(0.0, q, n)) @ Q.T
    shifts = wl.logspaced_real_shifts(1.0, 10.0 ** q, 6).real
    At = torch.as_tensor(A.T.copy(), device="cuda")
    F, perm, info = pk.shifted_lu_factor(ctx, At, shifts, prec=prec)
    assert info == [0] * len(shifts)
    ref = oadi.ShiftedSolver(A)
    for s, p in enumerate(shifts):
        M = A.T + p * np.eye(n)
        kappa = np.linalg.cond(M)
        for k in (1, 4, 5, 13):
            W = rng.standard_normal((n, k))
            X = pk.shifted_lu_solve(ctx, F[s], perm[s], torch.as_tensor(W, device="cuda"), prec=prec)
            Xh = X.double().cpu().numpy()
            Xr = ref.solve_base(p, W)
            fwd = np.linalg.norm(Xh - Xr) / np.linalg.norm(Xr)
            res = np.linalg.norm(M @ Xh - W) / (np.linalg.norm(M, 2) * np.linalg.norm(Xh))
            assert fwd <= 20.0 * n * kappa * U[prec], (p, k, fwd, kappa)
            assert res <= 20.0 * n * U[prec], (p, k, res)
        print(f"  shift {p:.3e}: kappa {kappa:.2e}  last forward error {fwd:.2e}  residual {res:.2e}", flush=True)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_lu_solve_in_place_and_zero_columns(pk, ctx, prec):
    n = 300
    rng = np.random.default_rng(3)
    M0 = torch.as_tensor(rng.standard_normal((n, n)), device="cuda")
    F, perm, _ = pk.shifted_lu_factor(ctx, M0, [-2.0], prec=prec)
    B = torch.as_tensor(rng.standard_normal((n, 6)), device="cuda", dtype=DT[prec])
    B = B.t().contiguous().t()
    X = pk.shifted_lu_solve(ctx, F[0], perm[0], B, prec=prec)
    lib = pk.load()
    code = pk.CARE_FP32 if prec == "fp32" else pk.CARE_FP64
    import ctypes as C
    st = lib.care_shifted_lu_solve(ctx.h, code, n, C.c_void_p(F[0].data_ptr()), C.c_void_p(perm[0].data_ptr()), 6,
                                   C.c_void_p(B.data_ptr()), n, C.c_void_p(B.data_ptr()), n)
    assert st == 0
    torch.cuda.synchronize()
    assert torch.equal(B, X)
    # k = 0 is a no-op
    st = lib.care_shifted_lu_solve(ctx.h, code, n, C.c_void_p(F[0].data_ptr()), C.c_void_p(perm[0].data_ptr()), 0,
                                   C.c_void_p(B.data_ptr()), n, C.c_void_p(B.data_ptr()), n)
    assert st == 0


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_lu_zero_pivot_is_reported_like_getrf(pk, ctx, prec):
    n = 40
    M0 = np.random.default_rng(5).standard_normal((n, n))
    M0[:, 17] = 0.0                      # a zero column: the pivot of column 17 is 0
    F, perm, info = pk.shifted_lu_factor(ctx, torch.as_tensor(M0, device="cuda"), [0.0, -1.0], prec=prec)
    assert info[0] == 18                 # 1-based, as getrf's info
    assert info[1] == 0
    Z = torch.zeros((n, n), device="cuda", dtype=torch.float64)
    _, _, info = pk.shifted_lu_factor(ctx, Z, [0.0], prec=prec)
    assert info == [1]


def test_lu_rejects_bad_arguments(pk, ctx):
    M0 = torch.zeros((2049, 2049), device="cuda")
    with pytest.raises(pk.api.CareError):
        pk.shifted_lu_factor(ctx, M0, [-1.0], prec="fp32")
    with pytest.raises(ValueError):
        pk.shifted_lu_factor(ctx, M0[:4, :4], [-1.0], prec="bf16")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_dense_solve_uses_the_batched_factors(pk, ctx, prec):
    """A dense CARE at n = 256 (Sec. 5.1's family, kappa 1e2) solved through
    care_solve_dense: its shifted solves run on the batched LU, and the result
    still meets the residual gate against the oracle's Schur solution."""
    from oracle import riccati
    A, B, C, q = wl.dense_instance(0, 64)
    n = A.shape[0]
    shifts = wl.logspaced_real_shifts(1.0, 10.0 ** q, 16)
    Z, s, st = pk.care_solve_dense(ctx, torch.as_tensor(A, device="cuda"), torch.as_tensor(B, device="cuda"),
                                   torch.as_tensor(C, device="cuda"), tol=1e-10, shifts=shifts, prec=prec)
    assert st == 0 and s["res_rel"] <= 1e-10
    X = riccati.care_hamiltonian(A, B, C)
    Zh = Z.cpu().numpy()
    err = np.linalg.norm(Zh @ Zh.T - X) / np.linalg.norm(X)
    print(f"dense n={n} {prec}: rank {s['rank']} relres {s['res_rel']:.2e} X error {err:.2e}", flush=True)
    assert err <= 1e-8
