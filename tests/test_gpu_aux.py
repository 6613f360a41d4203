"""Auxiliary behaviour of the solver, forced from the host: resuming from a
saved factor (Z_init) reproduces an uninterrupted run, non-finite inputs are
reported as CARE_ERR_NONFINITE, a forced stagnation returns
CARE_WARN_STAGNATED with the best factor, and an iteration cap of one
returns CARE_WARN_MAXIT without exceeding the cap.  Every kernel exits
normally in each case (the conditions are set on the host)."""
import numpy as np
import pytest

import workloads as wl
from oracle import lowrank

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


@pytest.fixture(scope="module")
def prob():
    return wl.fdm2d_problem(30, 3, 2)


def relres(P, Z):
    return lowrank.residual_norm(P.A, P.B, P.C, Z) / np.linalg.norm(P.C @ P.C.T)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_resume_from_saved_factor(pk, ctx, prob, prec):
    # a run stopped early at tol 1e-6, resumed from its factor to 1e-12, meets
    # the same gate as an uninterrupted run, and the two solutions agree
    # within the first-order reach of their residuals
    P = prob
    A = pk.DeviceCSR.from_scipy(P.A)
    print(f"resume prec={prec}", flush=True)
    Z1, s1, st1 = pk.care_solve(ctx, A, dev(P.B), dev(P.C), tol=1e-6, shifts=P.shifts, prec=prec)
    assert st1 == 0 and s1["res_rel"] <= 1e-6
    Z1 = pk.tight(Z1)                       # column-major, leading dimension n
    Zr, sr, str_ = pk.care_solve(ctx, A, dev(P.B), dev(P.C), tol=1e-12, shifts=P.shifts, prec=prec,
                                 Z_init=Z1.data_ptr(), ldz_init=Z1.stride(1), r_init=Z1.shape[1])
    Zu, su, stu = pk.care_solve(ctx, A, dev(P.B), dev(P.C), tol=1e-12, shifts=P.shifts, prec=prec)
    assert str_ == 0 and stu == 0, (sr, su)
    assert sr["iter0_outer"] == 0 and sr["iter0_inner"] == 0        # the initial solve was skipped
    Zr, Zu = Zr.cpu().numpy(), Zu.cpu().numpy()
    assert relres(P, Zr) <= 1e-11 and relres(P, Zu) <= 1e-11
    d = lowrank.factored_diff_norm(Zr, Zu) / lowrank.factored_norm(Zu)
    print(f"  resumed vs uninterrupted X difference {d:.2e}", flush=True)
    assert d <= 1e-8


@pytest.mark.parametrize("which", ["B", "C", "Z_init"])
def test_nonfinite_inputs(pk, ctx, prob, which):
    P = prob
    A = pk.DeviceCSR.from_scipy(P.A)
    B, C = P.B.copy(), P.C.copy()
    kw = {}
    if which == "B":
        B[7, 1] = np.nan
    elif which == "C":
        C[0, 11] = np.inf
    else:
        Z0 = pk.tight(dev(np.full((P.n, 2), 0.01)))
        Z0[5, 0] = float("nan")
        kw = dict(Z_init=Z0.data_ptr(), ldz_init=P.n, r_init=2)
    with pytest.raises(pk.CareError) as e:
        pk.care_solve(ctx, A, dev(B), dev(C), tol=1e-10, shifts=P.shifts, prec="fp32", **kw)
    assert e.value.name == "CARE_ERR_NONFINITE", e.value


def test_forced_stagnation_returns_best_factor(pk, ctx, prob):
    # stagnation threshold below any attainable residual ratio: the first
    # refinement step counts as stagnating; the status is a warning, the
    # factor the best one met, and its residual is what stats report
    P = prob
    A = pk.DeviceCSR.from_scipy(P.A)
    Z, s, st = pk.care_solve(ctx, A, dev(P.B), dev(P.C), tol=1e-15, shifts=P.shifts, prec="fp32",
                             stagnation=1e-300)
    print(f"  stagnation: status {st} hist {s['res_hist']}", flush=True)
    assert st == 1, s                           # CARE_WARN_STAGNATED
    assert s["stagnated"] == 1
    rel = relres(P, Z.cpu().numpy())
    assert abs(rel - s["res_rel"]) <= 1e-2 * s["res_rel"]
    assert s["res_rel"] <= min(s["res_hist"]) * (1 + 1e-12)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_krylov_cap_of_one(pk, ctx, prob, prec):
    # a shifted solve with an iteration cap of 1 warns and never runs more
    # iterations than the cap (restart rounds share the budget)
    P = prob
    A = pk.DeviceCSR.from_scipy(P.A)
    W = dev(np.random.default_rng(3).standard_normal((P.n, 4)))
    V, info = pk.shifted_solve(ctx, A, W, -100.0, prec=prec, tol=1e-12, maxit=1)
    assert info["status"] == 2, info            # CARE_WARN_MAXIT
    assert 1 <= info["iters"] <= 1
    # the same through lyap_lradi (krylov_maxit = 1)
    opts = pk.default_opts(prec, krylov_maxit=1)
    Z, s, st = pk.lyap_lradi(ctx, A, dev(P.C.T), P.shifts, tol=1e-10, opts=opts)
    assert st == 2, s


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_krylov_cap_on_the_graph_path(pk, ctx, prob, prec):
    # a cap that is not a multiple of the graph chunk (8 iterations) is met
    # exactly on the graph-replay path too
    P = prob
    A = pk.DeviceCSR.from_scipy(P.A)
    W = dev(np.random.default_rng(4).standard_normal((P.n, 3)))
    for cap in (21, 37):
        V, info = pk.shifted_solve(ctx, A, W, -2.0, prec=prec, tol=1e-15, maxit=cap)
        print(f"  cap {cap}: status {info['status']} iters {info['iters']}", flush=True)
        assert info["iters"] <= cap
