"""GPU parity of the HIP library (through its C ABI) against the CPU FP64
oracle, on seeded synthetic inputs of the paper's workload families."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as wl
from oracle import adi, care as ocare, lowrank, riccati

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


def dev(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().cpu().numpy()


RNG = np.random.default_rng(2024)


def rand_sparse(n, density, seed, shift=2.0):
    R = sp.random(n, n, density=density, random_state=np.random.RandomState(seed), format="csr")
    R = R - 0.4 * R.T
    d = np.asarray(abs(R).sum(axis=1)).ravel() + shift
    A = (R - sp.diags(d)).tocsr()
    A.sort_indices()
    return A


# ---------------------------------------------------------------------------
# sparse product (A4.1)
# ---------------------------------------------------------------------------
SPMM_CASES = [
    ("fdm2d_7", lambda: wl.fdm2d(7), 1),
    ("fdm2d_23", lambda: wl.fdm2d(23), 5),          # n = 529: ragged vs 64/256
    ("fdm3d_6", lambda: wl.fdm3d(6, 50.0), 17),     # k not a multiple of the panel
    ("random_300", lambda: rand_sparse(300, 0.03, 1), 33),
    ("n1", lambda: sp.csr_matrix(np.array([[-3.0]])), 2),
    ("empty_rows", lambda: sp.csr_matrix(sp.diags(-np.arange(1.0, 201.0))), 4),
    # entries up to 8 (N + 1)^2 = 7.3e5, beyond half precision's range: the
    # FP16 operator holds them under its power-of-two scale
    ("fdm2d_300", lambda: wl.fdm2d(300), 3),
]


@pytest.mark.parametrize("name,make,k", SPMM_CASES)
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 2e-6), ("bf16", 2e-2), ("fp16", 2e-3)])
@pytest.mark.parametrize("shift", [0.0, -7.5, -3.0 + 4.0j])
def test_spmm_parity(ctx, pk, name, make, k, prec, tol, shift):
    A = make()
    n = A.shape[0]
    X = RNG.standard_normal((n, 2 * k if complex(shift).imag else k))
    Ad = pk.DeviceCSR.from_scipy(A)
    Y = host(pk.spmm(ctx, Ad, dev(X), shift, prec))
    if complex(shift).imag:
        Xc = X[:, :k] + 1j * X[:, k:]
        Yc = A.T @ Xc + shift * Xc
        ref = np.hstack([Yc.real, Yc.imag])
    else:
        ref = A.T @ X + shift * X
    scale = (abs(A.T) @ abs(X) + abs(shift) * abs(X)).max()
    assert np.abs(Y - ref).max() <= tol * scale


def test_spmm_rejects_bad_csr(ctx, pk):
    A = wl.fdm2d(5)
    Ad = pk.DeviceCSR.from_scipy(A)
    bad = pk.DeviceCSR(Ad.row_ptr, Ad.col_idx.clone(), Ad.val, Ad.n)
    bad.col_idx[3] = 10_000                       # out of range: rejected before any product
    with pytest.raises(pk.CareError) as e:
        pk.spmm(ctx, bad, dev(np.ones((25, 1))), 0.0, "fp64")
    assert e.value.name == "CARE_ERR_ARG"


# ---------------------------------------------------------------------------
# FP64 matrix-core Gram and tall-skinny product (A7, A10 building blocks)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,a,b", [(1, 1, 1), (17, 3, 5), (1000, 33, 31), (70001, 64, 65), (5000, 200, 7)])
def test_gram_parity(ctx, pk, n, a, b):
    X = RNG.standard_normal((n, a))
    Y = RNG.standard_normal((n, b))
    C = host(pk.gram(ctx, dev(X), dev(Y)))
    ref = X.T @ Y
    assert np.abs(C - ref).max() <= 1e-13 * math.sqrt(n) * (np.abs(X).max() * np.abs(Y).max() * n) ** 0.5 + 1e-12
    # X^T X of one buffer with itself: exactly symmetric (the eigen-solvers downstream read one triangle)
    Xd = dev(X)
    Cs = host(pk.gram(ctx, Xd, Xd))
    assert np.allclose(Cs, X.T @ X, rtol=1e-12, atol=1e-10) and np.array_equal(Cs, Cs.T)


@pytest.mark.parametrize("n,q,k", [(1, 1, 1), (19, 4, 3), (1003, 37, 70), (65537, 16, 64), (4096, 130, 5)])
@pytest.mark.parametrize("beta", [0.0, 0.5])
def test_tsgemm_parity(ctx, pk, n, q, k, beta):
    X = RNG.standard_normal((n, q))
    S = RNG.standard_normal((q, k))
    Y0 = RNG.standard_normal((n, k))
    Y = host(pk.tsgemm(ctx, dev(X), dev(S), -1.5, beta, dev(Y0)))
    ref = -1.5 * X @ S + beta * Y0
    assert np.abs(Y - ref).max() <= 1e-12 * (np.abs(X) @ np.abs(S)).max() + 1e-14


@pytest.fixture(scope="module")
def ctx_gram128(pk):
    """A context whose large FP64 Grams run on the library's 128 x 128-tile
    MFMA kernel (MPCARE_GRAM=1 at context creation)."""
    import os
    old = os.environ.get("MPCARE_GRAM")
    os.environ["MPCARE_GRAM"] = "1"
    try:
        c = pk.Context(0)
    finally:
        if old is None:
            del os.environ["MPCARE_GRAM"]
        else:
            os.environ["MPCARE_GRAM"] = old
    yield c
    c.close()


@pytest.mark.parametrize("n,a,b", [(1, 40, 40), (17, 33, 100), (1000, 129, 300), (70001, 64, 65), (5000, 256, 128),
                                   (40000, 417, 417)])
def test_gram128_parity(ctx_gram128, pk, n, a, b):
    """The 128 x 128-tile FP64 MFMA Gram against the FP64 product in numpy:
    ragged tiles, fewer rows than a 16-row slice, one and several tiles;
    X^T X exactly symmetric and run-to-run identical."""
    X = RNG.standard_normal((n, a))
    Y = RNG.standard_normal((n, b))
    C = host(pk.gram(ctx_gram128, dev(X), dev(Y)))
    ref = X.T @ Y
    assert np.abs(C - ref).max() <= 1e-13 * math.sqrt(n) * (np.abs(X).max() * np.abs(Y).max() * n) ** 0.5 + 1e-12
    Xd = dev(X)
    Cs = host(pk.gram(ctx_gram128, Xd, Xd))
    assert np.allclose(Cs, X.T @ X, rtol=1e-12, atol=1e-10) and np.array_equal(Cs, Cs.T)
    assert np.array_equal(Cs, host(pk.gram(ctx_gram128, Xd, Xd)))


def test_gram_reproducible(ctx, pk):
    X = dev(RNG.standard_normal((50000, 40)))
    C1 = host(pk.gram(ctx, X, X))
    C2 = host(pk.gram(ctx, X, X))
    assert np.array_equal(C1, C2)


# ---------------------------------------------------------------------------
# shifted block solve with SMW (A4)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5), ("fp16", 5e-3)])
@pytest.mark.parametrize("p", [-300.0, -80.0 + 150.0j])
@pytest.mark.parametrize("smw", [False, True])
def test_shifted_solve_parity(ctx, pk, prec, tol, p, smw):
    N = 24
    A = wl.fdm2d(N)
    n = N * N
    m, w = 3, 5
    B = RNG.standard_normal((n, m))
    K = 5.0 * RNG.standard_normal((n, m)) if smw else None
    W = RNG.standard_normal((n, w))
    Ad = pk.DeviceCSR.from_scipy(A)
    V, info = pk.shifted_solve(ctx, Ad, dev(W), p, B=dev(B) if smw else None, K=dev(K) if smw else None, prec=prec,
                               tol=tol)
    V = host(V)
    ref = adi.ShiftedSolver(A, B if smw else None, K).solve(p, W)
    if complex(p).imag:
        ref = np.hstack([ref.real, ref.imag])
    err = np.linalg.norm(V - ref) / np.linalg.norm(ref)
    kappa = 30.0     # ||M^-1|| ||M|| margin for the recursive-residual test at these shifts
    assert err <= kappa * tol, (err, info)
    assert info["iters"] > 0


# ---------------------------------------------------------------------------
# LR-ADI iterate parity (A5, A9)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec,ztol", [("fp64", 1e-8), ("fp32", 1e-4)])
@pytest.mark.parametrize("shifts", [
    "real",
    "complex",
])
@pytest.mark.parametrize("split", [1, 2])    # fused BiCGStab products, or update pass + product
def test_lradi_iterate_parity(ctx, pk, prec, ztol, shifts, split):
    N = 20
    A = wl.fdm2d(N) if shifts == "real" else wl.fdm3d(7, 100.0)
    n = A.shape[0]
    m, w = 2, 3
    B = RNG.standard_normal((n, m))
    K = 2.0 * RNG.standard_normal((n, m))
    W0 = RNG.standard_normal((n, w))
    if shifts == "real":
        lo, hi = wl.fdm2d_spectral_bounds(N)
        s = wl.logspaced_real_shifts(lo, hi, 6)
    else:
        s = np.array([-60 + 40j, -60 - 40j, -400.0, -1500 + 300j, -1500 - 300j, -6000.0])
    jmax = 8
    Ad = pk.DeviceCSR.from_scipy(A)
    opts = pk.default_opts(prec, j_max=jmax, krylov_tol=1e-12 if prec == "fp64" else 1e-6, spmm_split=split)
    Z, stats, st = pk.lyap_lradi(ctx, Ad, dev(W0), s, B=dev(B), K=dev(K), tol=1e-30, opts=opts)
    Z = host(Z)
    Zr, Wr, info = adi.lradi(A, B, K, W0, s, tol=1e-30, jmax=jmax)
    assert stats["iter_inner"] == info["steps"]
    assert Z.shape[1] == Zr.shape[1]
    d = lowrank.factored_diff_norm(Z, Zr) / lowrank.factored_norm(Zr)
    assert d <= ztol
    assert abs(stats["res_rel"] - info["hist"][-1]) <= max(ztol, 1e-3 * info["hist"][-1]) * 10


def test_lradi_converges_to_bartels_stewart(ctx, pk):
    N = 12
    A = wl.fdm2d(N)
    n = N * N
    B = RNG.standard_normal((n, 2))
    K = RNG.standard_normal((n, 2))
    W0 = RNG.standard_normal((n, 2))
    lo, hi = wl.fdm2d_spectral_bounds(N)
    s = wl.logspaced_real_shifts(lo, hi, 8)
    Ad = pk.DeviceCSR.from_scipy(A)
    Z, stats, st = pk.lyap_lradi(ctx, Ad, dev(W0), s, B=dev(B), K=dev(K), tol=1e-13,
                                 opts=pk.default_opts("fp64", j_max=200, krylov_tol=1e-13))
    Z = host(Z)
    Ak = A.toarray() - B @ K.T
    X = riccati.lyap_bartels_stewart(Ak.T, -(W0 @ W0.T))
    assert np.linalg.norm(Z @ Z.T - X) <= 1e-9 * np.linalg.norm(X)


# ---------------------------------------------------------------------------
# Algorithm 1 and Algorithm 2 (A7, A10)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("eta", [0.0, 1e-4])
@pytest.mark.parametrize("shape", [(6, 10, 2, 3), (200, 40, 4, 5)])
def test_residual_factor_parity(ctx, pk, eta, shape):
    N, r, m, p = shape
    A = wl.fdm2d(N) if N > 10 else rand_sparse(N * N, 0.1, 7)
    n = A.shape[0]
    B = RNG.standard_normal((n, m))
    C = RNG.standard_normal((p, n))
    Z = 0.05 * RNG.standard_normal((n, r)) @ np.diag(np.logspace(0, -6, r))
    Ad = pk.DeviceCSR.from_scipy(A)
    Cp, Cm, res = pk.residual_factor(ctx, Ad, dev(B), dev(C), dev(Z), eta)
    Cp, Cm = host(Cp), host(Cm)
    ref = lowrank.residual_factor(A, B, C, Z, eta, full=True)
    assert abs(res - ref["res_fro"]) <= 1e-10 * ref["res_fro"]
    nrm = ref["res_fro"]
    assert lowrank.factored_diff_norm(Cp, ref["Cp"]) <= 1e-9 * nrm
    assert lowrank.factored_diff_norm(Cm, ref["Cm"]) <= 1e-9 * nrm
    if n <= 400:
        R = riccati.riccati_residual(A, B, C, Z @ Z.T)
        err = np.linalg.norm(Cp @ Cp.T - Cm @ Cm.T - R)
        assert err <= (1e-9 if eta == 0 else 2 * math.sqrt(n) * eta) * np.linalg.norm(R) + 1e-12


def test_residual_factor_rank_deficient_and_zero(ctx, pk):
    """Z with exactly repeated columns (F rank deficient) and Z = 0."""
    N = 15
    A = wl.fdm2d(N)
    n = N * N
    B = RNG.standard_normal((n, 2))
    C = RNG.standard_normal((3, n))
    z = 0.01 * RNG.standard_normal((n, 3))
    Z = np.hstack([z, z, z[:, :1] * 2.0])
    Ad = pk.DeviceCSR.from_scipy(A)
    Cp, Cm, res = pk.residual_factor(ctx, Ad, dev(B), dev(C), dev(Z), 0.0)
    R = riccati.riccati_residual(A, B, C, Z @ Z.T)
    Cp, Cm = host(Cp), host(Cm)
    assert np.linalg.norm(Cp @ Cp.T - Cm @ Cm.T - R) <= 1e-10 * np.linalg.norm(R)
    Cp, Cm, res = pk.residual_factor(ctx, Ad, dev(B), dev(C), dev(np.zeros((n, 0))), 0.0)
    assert abs(res - np.linalg.norm(C.T @ C)) <= 1e-12 * res


@pytest.mark.parametrize("case", ["psd", "indefinite", "collinear"])
def test_lowrank_truncate_parity(ctx, pk, case):
    n = 3000
    Z = RNG.standard_normal((n, 20)) @ np.diag(np.logspace(0, -7, 20))
    if case == "psd":
        Zp = 1e-3 * RNG.standard_normal((n, 6))
        Zm = 0.5 * Z[:, :3]
    elif case == "indefinite":
        Zp = 1e-2 * RNG.standard_normal((n, 4))
        Zm = RNG.standard_normal((n, 3))
    else:   # nearly collinear ADI-like blocks
        base = RNG.standard_normal((n, 4))
        Zp = np.hstack([base * (0.5 ** j) + 1e-9 * RNG.standard_normal((n, 4)) for j in range(6)])
        Zm = 1e-4 * base
    G = np.hstack([Z, Zp, Zm])
    sign = np.r_[np.ones(Z.shape[1] + Zp.shape[1]), -np.ones(Zm.shape[1])]
    for eta in (0.0, 1.1102230246251565e-15, 1e-6):
        Zg, eta_n = pk.lowrank_truncate(ctx, dev(G), sign, eta)
        Zg = host(Zg)
        ref = lowrank.signed_truncate(G, sign, eta, full=True)
        nrm = lowrank.factored_norm(ref["Z"])
        tol = 1e-10 if eta < 1e-9 else 10 * eta
        assert lowrank.factored_diff_norm(Zg, ref["Z"]) <= tol * nrm
        assert abs(eta_n - ref["eta_n"]) <= 1e-8 + 1e-6 * ref["eta_n"]


# ---------------------------------------------------------------------------
# Framework 1 end to end (A6, A8, A9, A10)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_care_solve_config1_vs_schur(ctx, pk, prec):
    P = wl.config1()
    Ad = pk.DeviceCSR.from_scipy(P.A)
    Z, stats, st = pk.care_solve(ctx, Ad, dev(P.B), dev(P.C), tol=1e-12, shifts=P.shifts, prec=prec)
    assert st == 0, stats
    Z = host(Z)
    Xs = riccati.care_schur(P.A, P.B, P.C)
    assert np.linalg.norm(Z @ Z.T - Xs) <= 1e-8 * np.linalg.norm(Xs)
    rel = lowrank.residual_norm(P.A, P.B, P.C, Z) / np.linalg.norm(P.C @ P.C.T)
    assert rel <= 1e-10
    # the library's FP64 residual agrees with the oracle's down to the
    # rounding floor of the two residual evaluations (both are summed
    # differently; here ||A^T X||_F / ||C^T C||_F ~ 1e3, so ~1e-13)
    assert abs(rel - stats["res_rel"]) <= 1e-3 * rel + 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("split", [0, 2])    # automatic choice (fused at this size), forced split
def test_care_solve_fdm_vs_oracle(ctx, pk, prec, split):
    P = wl.fdm2d_problem(40, 3, 4)
    Ad = pk.DeviceCSR.from_scipy(P.A)
    Z, stats, st = pk.care_solve(ctx, Ad, dev(P.B), dev(P.C), tol=1e-12, shifts=P.shifts, prec=prec,
                                 spmm_split=split)
    assert st == 0, stats
    Z = host(Z)
    Zr, info = ocare.framework1(P.A, P.B, P.C, P.shifts, tol=1e-13)
    d = lowrank.factored_diff_norm(Z, Zr) / lowrank.factored_norm(Zr)
    assert d <= 1e-8
    rel = lowrank.residual_norm(P.A, P.B, P.C, Z) / np.linalg.norm(P.C @ P.C.T)
    assert rel <= 1e-10
    # closed-loop stability of A - B B^T X
    Acl = P.A.toarray() - P.B @ ((P.B.T @ Z) @ Z.T)
    assert np.linalg.eigvals(Acl).real.max() < 0


def test_spmm_fp16_entries_over_nine_decades(ctx, pk):
    # entries from 1e-3 to 1e6 in one operator: the power-of-two scale keeps
    # the largest within half's range, the smallest fall to half's subnormal
    # range, where they carry little weight in any row's sum
    rng = np.random.default_rng(23)
    n = 3000
    A = sp.random(n, n, density=0.003, random_state=np.random.RandomState(4), format="csr")
    A.data = np.sign(rng.standard_normal(A.nnz)) * 10.0 ** rng.uniform(-3.0, 6.0, A.nnz)
    A = (A - 2e6 * sp.identity(n)).tocsr()
    X = rng.standard_normal((n, 6))
    Y = host(pk.spmm(ctx, pk.DeviceCSR.from_scipy(A), dev(X), -5.0, "fp16"))
    ref = A.T @ X - 5.0 * X
    scale = abs(A.T) @ abs(X) + 5.0 * abs(X)
    assert np.all(np.isfinite(Y))
    assert np.abs(Y - ref).max() <= 2e-3 * scale.max()
    # row by row: each within half's relative accuracy of its own magnitude sum
    assert np.all(np.abs(Y - ref) <= 2e-3 * scale + 1e-12)
