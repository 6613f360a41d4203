"""Dense CAREs (the dense test problems of Sec. 5.1 and the uneven dense
batch): Framework 1 with LU-based shifted solves against dense Schur
solutions, the batched path against single solves, and honest reporting
where the FP32 inner solves are beyond Theorem 1's conditioning range."""
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


def relres(A, B, C, Z):
    R = A.T @ (Z @ Z.T) + (Z @ Z.T) @ A - (Z @ (Z.T @ B)) @ ((B.T @ Z) @ Z.T) + C.T @ C
    return np.linalg.norm(R) / np.linalg.norm(C @ C.T)


def shifts_for(q, count=16):
    return wl.logspaced_real_shifts(1.0, 10.0 ** q, count)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n,q", [(96, 2.0), (200, 3.0), (256, 4.0)])
def test_dense_care_vs_schur(pk, ctx, prec, n, q):
    _, B, C, _ = wl.dense_instance(0, m=4, p=4, sizes=(n,))
    Q = wl.haar_orthogonal(n, np.random.default_rng(3))
    A = -(Q * np.logspace(0, q, n)) @ Q.T            # kappa_2(A) = 10^q
    print(f"dense n={n} q={q} prec={prec}", flush=True)
    Z, stats, st = pk.care_solve_dense(ctx, dev(A), dev(B), dev(C), tol=1e-12, shifts=shifts_for(q), prec=prec)
    assert st == 0, stats
    Z = Z.cpu().numpy()
    Xs = riccati.care_schur(A, B, C)
    assert relres(A, B, C, Z) <= 1e-10
    assert np.linalg.norm(Z @ Z.T - Xs) <= 1e-8 * np.linalg.norm(Xs)
    assert stats["krylov_iters"] == 0          # direct shifted solves


def test_example1_dense_vs_schur(pk, ctx):
    # the paper's Example 1 family (Sec. 5.1) at n = 300, kappa_2(A) = 1e3
    A, B, C = wl.ex1(300, 10, 5, 3.0)
    Z, stats, st = pk.care_solve_dense(ctx, dev(A), dev(B), dev(C), tol=1e-12, shifts=shifts_for(3.0), prec="fp32")
    assert st == 0, stats
    Z = Z.cpu().numpy()
    Xs = riccati.care_schur(A, B, C)
    assert relres(A, B, C, Z) <= 1e-10
    assert np.linalg.norm(Z @ Z.T - Xs) <= 1e-8 * np.linalg.norm(Xs)


def test_dense_heuristic_shifts(pk, ctx):
    A, B, C, q = wl.dense_instance(3, sizes=(160,))
    Z, stats, st = pk.care_solve_dense(ctx, dev(A), dev(B), dev(C), tol=1e-10, shifts=None, prec="fp64")
    assert st == 0, stats
    assert relres(A, B, C, Z.cpu().numpy()) <= 1e-10


def test_dense_batch_equals_single_solves(pk, ctx):
    idx = [0, 2, 5, 9]
    insts = [wl.dense_instance(i, sizes=(128, 192, 256, 320)) for i in idx]   # q = 2 .. 3.4
    items = [(dev(A), dev(B), dev(C), shifts_for(q)) for A, B, C, q in insts]
    out = pk.care_solve_batch(ctx, items, tol=1e-10, prec="fp32", workers=3)
    for (A, B, C, q), (Zb, sb, st, msg), it in zip(insts, out, items):
        assert st == 0, msg
        Zs, ss, sst = pk.care_solve_dense(ctx, it[0], it[1], it[2], tol=1e-10, shifts=it[3], prec="fp32")
        assert sst == 0
        Zb, Zs = Zb.cpu().numpy(), Zs.cpu().numpy()
        assert lowrank.factored_diff_norm(Zb, Zs) <= 1e-13 * lowrank.factored_norm(Zs)
        assert relres(A, B, C, Zb) <= 1e-10


def test_dense_batch_workload_sample_reports_honestly(pk, ctx):
    # instances of the 64-instance dense batch at their real sizes: kappa from
    # 1e2 to 1e12.  FP32 inner solves may fail for large kappa (Theorem 1);
    # a status of 0 must then still mean a residual within the tolerance.
    idx = [0, 1, 8, 30, 63]
    insts = [wl.dense_instance(i) for i in idx]
    print("dense sample", [(A.shape[0], round(q, 2)) for A, _, _, q in insts], flush=True)
    items = [(dev(A), dev(B), dev(C), shifts_for(q)) for A, B, C, q in insts]
    out = pk.care_solve_batch(ctx, items, tol=1e-10, prec="fp32", workers=4)
    for (A, B, C, q), (Z, stats, st, msg) in zip(insts, out):
        print(f"  n={A.shape[0]} q={q:.2f} status={st} res={stats['res_rel']:.2e} {msg}", flush=True)
        assert st in (0, 1, 2) or st == pk.CARE_ERR_BREAKDOWN or st == pk.CARE_ERR_UNSTABLE, msg
        if st == 0:
            assert relres(A, B, C, Z.cpu().numpy()) <= 1.5e-10
        if q <= 4.0:
            assert st == 0, msg


GOLDEN = __import__("json").load(open(__import__("os").path.join(__import__("os").path.dirname(__file__), "golden",
                                                                   "ex1_table1.json")))


@pytest.mark.parametrize("row", GOLDEN["rows"], ids=lambda r: f"kappa{r['kappa']:.0e}")
def test_example1_against_table1(pk, ctx, row):
    # loose pins from the paper's Table 1: the FP64 result reaches the
    # paper's residual level with a rank of the paper's order; the FP32-inner
    # run converges where the paper's did and does not where it failed
    q = float(np.log10(row["kappa"]))
    A, B, C = wl.ex1(GOLDEN["n"], GOLDEN["m"], GOLDEN["p"], q)
    print(f"Example 1 kappa={row['kappa']:.0e}", flush=True)
    Z, st64, s64 = pk.care_solve_dense(ctx, dev(A), dev(B), dev(C), tol=1e-14, shifts=shifts_for(q), prec="fp64")
    assert s64 in (0, 1), st64
    assert st64["res_paper"] <= 1e-14
    r = st64["rank"]
    assert 0.5 * row["rank_fp64"] <= r <= 2 * row["rank_fp64"] + 4, (r, row)
    try:
        Z32, st32, s32 = pk.care_solve_dense(ctx, dev(A), dev(B), dev(C), tol=1e-14, shifts=shifts_for(q),
                                             prec="fp32", k_max=20)
    except pk.CareError as e:      # e.g. an inner FP32 LR-ADI that diverges
        assert e.name in ("CARE_ERR_UNSTABLE", "CARE_ERR_BREAKDOWN", "CARE_ERR_NONFINITE"), e
        print(f"  fp64 rank {r} res {st64['res_paper']:.2e} | fp32 failed: {e}", flush=True)
        assert not row["fp32_converged"]
        return
    # converged in the paper's sense: its residual measure at the level the
    # table reports (a stop on stagnation at that floor counts)
    ok32 = s32 in (0, 1) and st32["res_paper"] <= 1e-14
    print(f"  fp64 rank {r} res {st64['res_paper']:.2e} | fp32 status {s32} rank {st32['rank']} "
          f"res {st32['res_paper']:.2e} relres {st32['res_rel']:.2e}", flush=True)
    assert ok32 == row["fp32_converged"], (s32, st32["res_paper"], st32["res_rel"])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_example1_dynamic_shifts(pk, ctx, prec):
    # Example 1 at kappa = 10: B = 0.2 ones moves the closed-loop spectrum far
    # from A's, so shifts recomputed for each A - B K^T (shift_update = 1)
    # need far fewer ADI steps than one set from A; both reach the Schur
    # solution
    A, B, C = wl.ex1(300, 10, 5, 1.0)
    Xs = riccati.care_schur(A, B, C)
    steps = {}
    for dyn in (0, 1):
        Z, st, s = pk.care_solve_dense(ctx, dev(A), dev(B), dev(C), tol=1e-12, shifts=None, prec=prec,
                                       shift_update=dyn)
        assert s in (0, 1), st
        Z = Z.cpu().numpy()
        assert relres(A, B, C, Z) <= 1e-11
        assert np.linalg.norm(Z @ Z.T - Xs) <= 1e-8 * np.linalg.norm(Xs)
        steps[dyn] = st["iter0_inner"] + st["iter_inner"]
    print(f"  ADI steps: fixed shifts {steps[0]}, shifts per operator {steps[1]}", flush=True)
    assert 2 * steps[1] <= steps[0], steps
