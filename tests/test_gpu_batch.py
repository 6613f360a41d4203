"""Batched Framework 1 (independent instances of uneven size on concurrent
worker streams): every instance must come out as its single-instance solve
does, meet the residual gate, agree with the CPU oracle, and report its own
failure without spoiling the others."""
import numpy as np
import pytest

import workloads as wl
from oracle import care as ocare
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


def relres(P, Z):
    return lowrank.residual_norm(P.A, P.B, P.C, Z) / np.linalg.norm(P.C @ P.C.T)


def small_batch():
    # uneven grids and (m, p), seeded per instance like the batch generator
    spec = [(10, 2, 3), (26, 1, 1), (14, 4, 2), (21, 3, 5), (17, 1, 4)]
    return [wl.fdm2d_problem(N, m, p, seed=wl.DEFAULT_SEED + i) for i, (N, m, p) in enumerate(spec)]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_equals_single_instance_solves(pk, ctx, prec):
    probs = small_batch()
    print(f"batch of {len(probs)} prec {prec}", flush=True)
    As = [pk.DeviceCSR.from_scipy(P.A) for P in probs]
    out = pk.care_solve_batch(ctx, [(A, dev(P.B), dev(P.C), P.shifts) for A, P in zip(As, probs)],
                              tol=1e-10, prec=prec, workers=3)
    assert len(out) == len(probs)
    for A, P, (Z, stats, st, msg) in zip(As, probs, out):
        assert st == 0, msg
        Zs, ss, sst = pk.care_solve(ctx, A, dev(P.B), dev(P.C), tol=1e-10, shifts=P.shifts, prec=prec)
        assert sst == 0
        Zb, Zs = Z.cpu().numpy(), Zs.cpu().numpy()
        # same code, same inputs, deterministic reductions: the same factor
        assert lowrank.factored_diff_norm(Zb, Zs) <= 1e-13 * lowrank.factored_norm(Zs)
        assert (stats["iter0_outer"], stats["iter_outer"], stats["rank"]) == \
            (ss["iter0_outer"], ss["iter_outer"], ss["rank"])
        assert relres(P, Zb) <= 1e-10


def test_batch_instances_agree_with_oracle(pk, ctx):
    probs = small_batch()[:2]
    out = pk.care_solve_batch(ctx, [(pk.DeviceCSR.from_scipy(P.A), dev(P.B), dev(P.C), P.shifts) for P in probs],
                              tol=1e-12, prec="fp32", workers=2)
    for P, (Z, stats, st, msg) in zip(probs, out):
        assert st == 0, msg
        Zr, _ = ocare.framework1(P.A, P.B, P.C, P.shifts, tol=1e-13)
        assert lowrank.factored_diff_norm(Z.cpu().numpy(), Zr) <= 1e-8 * lowrank.factored_norm(Zr)


def test_batch_reports_a_failed_instance_and_solves_the_rest(pk, ctx):
    probs = small_batch()[:3]
    items = [(pk.DeviceCSR.from_scipy(P.A), dev(P.B), dev(P.C), P.shifts) for P in probs]
    items[1] = (items[1][0], items[1][1], items[1][2], np.array([-5.0, 3.0]))   # unstable shift
    out = pk.care_solve_batch(ctx, items, tol=1e-10, prec="fp32", workers=2)
    assert out[1][2] == pk.CARE_ERR_ARG and "shift" in out[1][3]
    for k in (0, 2):
        assert out[k][2] == 0
        assert relres(probs[k], out[k][0].cpu().numpy()) <= 1e-10


def test_batch_workload_sample_meets_the_gate(pk, ctx):
    # instances 0, 5 and 12 of the 32-instance uneven FDM batch at their real
    # sizes (N = 100, 135, 204), FP32 inner / FP64 refinement
    idx = [0, 5, 12]
    probs = [wl.fdm_batch_problem(i) for i in idx]
    print("batch sample", [(P.n, P.B.shape[1], P.C.shape[0]) for P in probs], flush=True)
    out = pk.care_solve_batch(ctx, [(pk.DeviceCSR.from_scipy(P.A), dev(P.B), dev(P.C), P.shifts) for P in probs],
                              tol=1e-10, prec="fp32", workers=3)
    for P, (Z, stats, st, msg) in zip(probs, out):
        assert st == 0, msg
        assert stats["res_rel"] <= 1e-10
        assert relres(P, Z.cpu().numpy()) <= 1.5e-10
