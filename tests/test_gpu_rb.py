"""Red-black reduction of the shifted solves (option krylov_rb): for a
two-colourable stencil with a constant diagonal, each shifted solve runs its
Krylov method on the black unknowns of the exactly reduced system.  The
LR-ADI iterates with and without it match the oracle's iterate (sparse LU
per shift) for real shifts and for complex-conjugate pairs; the reduction
needs fewer Krylov column-iterations; matrices it does not apply to (an odd
stencil, a varying diagonal) solve exactly as before; whole CARE solves meet
the gate and agree with and without it."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as wl
from oracle import adi, lowrank

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
RNG = np.random.default_rng(77)


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


def lradi_case(kind):
    if kind == "fdm2d_real":
        N = 24
        A = wl.fdm2d(N)
        lo, hi = wl.fdm2d_spectral_bounds(N)
        s = wl.logspaced_real_shifts(lo, hi, 6)
    elif kind == "fdm3d_complex":
        A = wl.fdm3d(7, 100.0)
        s = np.array([-60 + 40j, -60 - 40j, -400.0, -1500 + 300j, -1500 - 300j, -6000.0])
    elif kind == "toeplitz":            # offsets 1, 2, 3: not two-colourable
        A = wl.toeplitz5(300)
        s = -np.logspace(0, 1, 5)
    else:                               # varying diagonal: no reduction
        A = (wl.fdm2d(16) + sp.diags(np.linspace(-30.0, -1.0, 256))).tocsr()
        s = -np.logspace(1.5, 3.5, 6)
    return A, s


@pytest.mark.parametrize("kind", ["fdm2d_real", "fdm3d_complex", "toeplitz", "varying_diagonal"])
@pytest.mark.parametrize("prec,ztol", [("fp64", 1e-8), ("fp32", 1e-4)])
def test_lradi_iterate_with_and_without_reduction(ctx, pk, kind, prec, ztol):
    A, s = lradi_case(kind)
    n = A.shape[0]
    m, w = 2, 3
    B = RNG.standard_normal((n, m))
    K = 0.5 * RNG.standard_normal((n, m))
    W0 = RNG.standard_normal((n, w))
    jmax = 6
    Zr, Wr, info = adi.lradi(A, B, K, W0, s, tol=1e-30, jmax=jmax)
    Ad = pk.DeviceCSR.from_scipy(A)
    its = {}
    for rb in (0, 1):
        print(f"rb {kind} prec={prec} krylov_rb={rb}", flush=True)
        opts = pk.default_opts(prec, j_max=jmax, krylov_tol=1e-12 if prec == "fp64" else 1e-6, krylov_rb=rb)
        Z, stats, st = pk.lyap_lradi(ctx, Ad, dev(W0), s, B=dev(B), K=dev(K), tol=1e-30, opts=opts)
        Z = Z.cpu().numpy()
        assert stats["iter_inner"] == info["steps"]
        d = lowrank.factored_diff_norm(Z, Zr) / lowrank.factored_norm(Zr)
        print(f"  X difference to the oracle {d:.2e}, Krylov column-iterations {stats['krylov_iters']}", flush=True)
        assert d <= ztol
        its[rb] = stats["krylov_iters"]
    if kind in ("fdm2d_real", "fdm3d_complex"):
        assert its[1] < its[0]
    else:
        assert its[1] == its[0]          # not applicable: the same solve


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_care_solve_with_and_without_reduction(ctx, pk, prec):
    P = wl.fdm2d_problem(40, 3, 2)
    Ad = pk.DeviceCSR.from_scipy(P.A)
    Zs = []
    for rb in (0, 1):
        Z, stats, st = pk.care_solve(ctx, Ad, dev(P.B), dev(P.C), tol=1e-12, shifts=P.shifts, prec=prec, krylov_rb=rb)
        assert st == 0, stats
        Z = Z.cpu().numpy()
        rel = lowrank.residual_norm(P.A, P.B, P.C, Z) / np.linalg.norm(P.C @ P.C.T)
        print(f"  care_solve {prec} krylov_rb={rb}: relres {rel:.2e} Krylov iterations {stats['krylov_iters']} "
              f"t {stats['t_total']:.3f} s", flush=True)
        assert rel <= 1e-11
        Zs.append(Z)
    d = lowrank.factored_diff_norm(Zs[0], Zs[1]) / lowrank.factored_norm(Zs[0])
    assert d <= 1e-9
