"""The Toeplitz example of Sec. 5.2 (5-diagonal Toeplitz A, B n x 10 with
||B||_F = 1, C 5 x n, heuristic shifts): GPU solves against the dense
Schur solution at n = 400, and at the paper's sizes against the CPU oracle's
FP64 residual of the returned factor and the other precision's result."""
import numpy as np
import pytest

import workloads as wl
from oracle import lowrank, riccati

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


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_toeplitz_small_vs_schur(pk, ctx, prec):
    P = wl.toeplitz_problem(400)
    print(f"toeplitz n=400 prec={prec}", flush=True)
    Z, stats, st = pk.care_solve(ctx, pk.DeviceCSR.from_scipy(P.A), dev(P.B), dev(P.C), tol=1e-12, shifts=None,
                                 prec=prec)
    assert st == 0, stats
    Z = Z.cpu().numpy()
    Xs = riccati.care_schur(P.A, P.B, P.C)
    assert lowrank.residual_norm(P.A, P.B, P.C, Z) <= 1e-10 * np.linalg.norm(P.C @ P.C.T)
    assert np.linalg.norm(Z @ Z.T - Xs) <= 1e-8 * np.linalg.norm(Xs)


@pytest.mark.parametrize("n", [32768, 131072])
def test_toeplitz_paper_sizes(pk, ctx, n):
    # the smallest and largest sizes of the paper's table: both precisions
    # with one heuristic shift set; the returned factors' residuals evaluated
    # by the CPU oracle, and the two results against each other
    P = wl.toeplitz_problem(n)
    A = pk.DeviceCSR.from_scipy(P.A)
    sh = pk.penzl_shifts(ctx, A)
    Zs = {}
    for prec in ("fp64", "fp32"):
        print(f"toeplitz n={n} prec={prec}", flush=True)
        Z, stats, st = pk.care_solve(ctx, A, dev(P.B), dev(P.C), tol=1e-10, shifts=sh, prec=prec)
        assert st == 0, stats
        Zs[prec] = Z.cpu().numpy()
        rel = lowrank.residual_norm(P.A, P.B, P.C, Zs[prec]) / np.linalg.norm(P.C @ P.C.T)
        assert rel <= 1e-10, (prec, rel)
        assert abs(rel - stats["res_rel"]) <= 1e-2 * rel + 1e-14, (rel, stats["res_rel"])
    d = lowrank.factored_diff_norm(Zs["fp32"], Zs["fp64"]) / lowrank.factored_norm(Zs["fp64"])
    assert d <= 1e-8, d
