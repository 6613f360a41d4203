"""The full uneven dense batch: 64 dense CAREs, n in {256, ..., 2048},
kappa_2(A) = 10^q with q = 2 ... 12 (the dense test family of Sec. 5.1, with
the conditioning sweep of Table 1 carried to larger n), m = p = 4, solved in
one batched call and compared with the oracle's solution X (Hamiltonian Schur
method polished by dense Newton-Kleinman; sampled entries X[I, I] and the
sketch X[I, :] Omega stored in tests/golden/config4_x_samples.json).

Beyond kappa ~ 1e6.5 no FP64 method reaches tol 1e-10: the residual of
the rounded exact solution grows like u kappa, and the oracle's own residual
(stored with its samples) is 3e-11 at kappa = 10^6.8 and 3e-6 at 10^12.  The
solver then stops on stagnation (status 1); it must have reached the
oracle's level (within a factor 10).  X must match the oracle to 1e-8 where
kappa_2(A) <= 1e8.  Where the problem is within FP32's conditioning range
(Theorem 1: d_1 kappa_F(L_k) u_s < 1) the FP32-inner result must do the
same; beyond it (kappa >= 1e8, where Table 1's FP32 run fails too) the
solver may stop or report a breakdown, and a status of 0 must still mean a
residual within tolerance."""
import json
import os

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "config4_x_samples.json")))
TOL = 1e-10


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


def x_errors(Z, g):
    """Relative errors of X = Z Z^T against the oracle's samples of
    instance g (rows and Omega drawn as the golden's writer drew them)."""
    rng = np.random.default_rng(GOLDEN["sample_seed"] + g["i"])
    n = Z.shape[0]
    rows = np.sort(rng.choice(n, GOLDEN["nrows"], replace=False))
    assert list(rows) == g["rows"]
    omega = torch.as_tensor(rng.standard_normal((n, GOLDEN["nsketch"])), device=Z.device)
    Zi = Z[torch.as_tensor(rows, device=Z.device)]
    block = (Zi @ Zi.T).cpu().numpy()
    sketch = (Zi @ (Z.T @ omega)).cpu().numpy()
    b0, s0 = np.asarray(g["block"]), np.asarray(g["sketch"])
    return float(np.linalg.norm(block - b0) / np.linalg.norm(b0)), float(np.linalg.norm(sketch - s0) /
                                                                          np.linalg.norm(s0))


def solve_all(pk, ctx, prec):
    items, qs = [], []
    for g in GOLDEN["instances"]:
        A, B, C, q = wl.dense_instance(g["i"], len(GOLDEN["instances"]))
        assert A.shape[0] == g["n"] and abs(q - g["q"]) < 1e-12
        items.append((dev(A), dev(B), dev(C), wl.logspaced_real_shifts(1.0, 10.0 ** q, 16)))
        qs.append(q)
    print(f"dense batch of {len(items)} instances, {prec} inner", flush=True)
    torch.cuda.empty_cache()      # the batch's workers allocate beside this process's cached blocks
    return pk.care_solve_batch(ctx, items, tol=TOL, prec=prec, workers=4), qs


def report(pk, out, qs):
    rows = []
    for g, q, (Z, s, st, msg) in zip(GOLDEN["instances"], qs, out):
        eb = es = float("nan")
        if st in (0, 1, 2) and Z.shape[1] > 0:
            eb, es = x_errors(Z, g)
        rows.append((g, q, st, s, eb, es))
        print(f"  {g['i']:2d} n={g['n']:4d} q={q:5.2f} status={pk.STATUS_NAMES.get(st, st):20s} "
              f"res={s['res_rel']:.2e} rank={s['rank']:4d} X err block {eb:.2e} sketch {es:.2e} "
              f"(oracle relres {g['relres']:.1e}) {msg}", flush=True)
    return rows


def reached_oracle_level(s, g):
    return s["res_rel"] <= max(TOL, 10.0 * g["relres"])


def test_dense_batch_fp64_matches_oracle(pk, ctx):
    out, qs = solve_all(pk, ctx, "fp64")
    for g, q, st, s, eb, es in report(pk, out, qs):
        assert st in (0, 1), (g["i"], st)
        if st == 0:
            assert s["res_rel"] <= TOL
        assert reached_oracle_level(s, g), (g["i"], q, s["res_rel"], g["relres"])
        if q <= 8.0:
            assert max(eb, es) <= 1e-8, (g["i"], q, eb, es)


def test_dense_batch_fp32_inner_matches_oracle_where_fp32_suffices(pk, ctx):
    out, qs = solve_all(pk, ctx, "fp32")
    ok = 0
    for g, q, st, s, eb, es in report(pk, out, qs):
        assert st in (0, 1, 2) or st in (pk.CARE_ERR_BREAKDOWN, pk.CARE_ERR_UNSTABLE, pk.CARE_ERR_NONFINITE), \
            (g["i"], st)
        if st == 0:
            ok += 1
            assert s["res_rel"] <= TOL
        if q <= 6.5:
            # kappa_2(A) <= 10^6.5: both precisions reach tol 1e-10
            assert st == 0, (g["i"], q)
        if q < 8.0:
            # kappa_2(A) < 1e8: FP32 corrections still contract (Theorem 1),
            # ever more slowly towards kappa u_32 ~ 1, so the refinement may
            # end on stagnation or on its step cap (status 1 or 2); either way
            # at the oracle's residual level and with X matching the oracle
            assert st in (0, 1, 2) and reached_oracle_level(s, g), (g["i"], q, st, s["res_rel"], g["relres"])
            assert max(eb, es) <= 1e-8, (g["i"], q, eb, es)
    print(f"fp32 inner: {ok} of {len(qs)} instances converged", flush=True)
