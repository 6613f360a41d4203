"""Rotation of the LR-ADI residual factor (option adi_rotate, FP32 inner
solves): W Q with Q orthogonal carries the same residual W W^T, so a solve
with rotations must meet the same gate, and its solution must agree with the
unrotated one to within what the residual gate allows."""
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


@pytest.mark.parametrize("N,m,p", [(80, 3, 4), (120, 2, 6)])
def test_rotation_keeps_the_solution(pk, ctx, N, m, p):
    P = wl.fdm2d_problem(N, m, p)
    print(f"rotation fdm2d N={N} m={m} p={p} fp32", flush=True)
    A = pk.DeviceCSR.from_scipy(P.A)
    out = []
    for rot in (0, 1):
        Z, s, st = pk.care_solve(ctx, A, dev(P.B), dev(P.C), tol=1e-10, shifts=P.shifts, prec="fp32", adi_rotate=rot)
        assert st == 0
        Zh = Z.cpu().numpy()
        rel = lowrank.residual_norm(P.A, P.B, P.C, Zh) / np.linalg.norm(P.C @ P.C.T, "fro")
        print(f"  adi_rotate {rot}: rotations {s['adi_rotations']} relres {rel:.2e} "
              f"krylov iterations {s['krylov_iters']} rank {Zh.shape[1]}", flush=True)
        assert rel <= 1e-10
        out.append((Zh, s, rel))
    (Z0, s0, r0), (Z1, s1, r1) = out
    assert s0["adi_rotations"] == 0 and s1["adi_rotations"] > 0
    # both solutions are within the first-order reach of their residuals of
    # the exact one: ||dX||_F / ||X||_F <~ relres ||C^T C||_F / (2 lambda_min ||X||_F)
    xf = lowrank.factored_norm(Z0)
    bound = (r0 + r1) * np.linalg.norm(P.C @ P.C.T, "fro") / (2.0 * P.meta["lam_lo"] * xf)
    d = lowrank.factored_diff_norm(Z0, Z1) / xf
    print(f"  ||X_rot - X||_F / ||X||_F = {d:.2e} (bound {bound:.1e})", flush=True)
    assert d <= bound
