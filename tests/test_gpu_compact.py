"""Column compaction of the block BiCGStab (option krylov_compact): once at
most half of a block solve's columns still iterate, they are gathered into
fewer panels.  Each column's arithmetic is unchanged, so a solve must give
bit-identical factors and statistics with and without it."""
import numpy as np
import pytest

import workloads as wl
from oracle import shifts as osh

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


def solve_both(pk, ctx, P, shifts, prec, **kw):
    A = pk.DeviceCSR.from_scipy(P.A)
    out = []
    for compact in (0, 1):
        Z, s, st = pk.care_solve(ctx, A, dev(P.B), dev(P.C), tol=1e-10, shifts=shifts, prec=prec,
                                 krylov_compact=compact, **kw)
        assert st == 0
        out.append((Z.cpu().numpy(), s))
    return out


@pytest.mark.parametrize("prec,p", [("fp32", 4), ("fp64", 24)])
@pytest.mark.parametrize("profile", [0, 1])
def test_compaction_leaves_fdm_solve_unchanged(pk, ctx, prec, p, profile):
    # profile = 1 runs every iteration directly, 0 replays captured chunks.
    # FP32: the corrections' wide right-hand sides compact; FP64 has no
    # correction here, so its initial stage gets p + m = 27 columns (2 panels)
    P = wl.fdm2d_problem(60, 3, p)
    print(f"compaction fdm2d N=60 m=3 p={p} {prec} profile {profile}", flush=True)
    (Z0, s0), (Z1, s1) = solve_both(pk, ctx, P, P.shifts, prec, profile=profile)
    print(f"  compactions {s1['krylov_compactions']} krylov iterations {s1['krylov_iters']} rank {Z1.shape[1]}",
          flush=True)
    assert s0["krylov_compactions"] == 0
    assert s1["krylov_compactions"] > 0
    assert Z0.shape == Z1.shape and np.array_equal(Z0, Z1)
    for k in ("krylov_iters", "iter0_outer", "iter0_inner", "iter_outer", "iter_inner", "rank", "res_rel"):
        assert s0[k] == s1[k], k


def test_compaction_leaves_complex_shift_solve_unchanged(pk, ctx):
    # rotating-field 3D problem: complex-conjugate shift pairs (interleaved
    # (re, im) column pairs move together)
    P = wl.fdm3d_problem(8, 1, 10)
    shifts = osh.penzl_shifts(P.A, 16, 20, 10)
    assert np.any(shifts.imag != 0)
    print("compaction fdm3d N=8 fp32 complex shifts", flush=True)
    (Z0, s0), (Z1, s1) = solve_both(pk, ctx, P, shifts, "fp32")
    print(f"  compactions {s1['krylov_compactions']} krylov iterations {s1['krylov_iters']}", flush=True)
    assert Z0.shape == Z1.shape and np.array_equal(Z0, Z1)
    assert s0["krylov_iters"] == s1["krylov_iters"] and s0["res_rel"] == s1["res_rel"]
