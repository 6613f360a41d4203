"""3D convection-diffusion CAREs with a rotating field (complex spectrum,
complex-conjugate shift pairs from the heuristic): FP32 and bf16-product inner
solves with FP64 refinement against the CPU oracle, and the full 64^3 problem
against the residual gate."""
import numpy as np
import pytest

import workloads as wl
from oracle import care as ocare
from oracle import lowrank
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


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16", "fp16"])
def test_3d_rotating_vs_oracle(pk, ctx, prec):
    P = wl.fdm3d_problem(8, 1, 10)
    shifts = osh.penzl_shifts(P.A, 16, 20, 10)          # the same complex pairs on both sides
    assert np.any(shifts.imag != 0)
    print(f"3d n={P.n} prec={prec} shifts={len(shifts)}", flush=True)
    Z, stats, st = pk.care_solve(ctx, pk.DeviceCSR.from_scipy(P.A), dev(P.B), dev(P.C), tol=1e-12, shifts=shifts,
                                 prec=prec)
    assert st == 0, stats
    Z = Z.cpu().numpy()
    Zr, _ = ocare.framework1(P.A, P.B, P.C, shifts, tol=1e-13)
    d = lowrank.factored_diff_norm(Z, Zr) / lowrank.factored_norm(Zr)
    rel = lowrank.residual_norm(P.A, P.B, P.C, Z) / np.linalg.norm(P.C @ P.C.T)
    print(f"  relres {rel:.2e} X-diff {d:.2e} iter0 {stats['iter0_outer']}({stats['iter0_inner']}) "
          f"iter {stats['iter_outer']}({stats['iter_inner']})", flush=True)
    assert rel <= 1e-10
    assert d <= 1e-8


def test_3d_full_size_meets_the_gate(pk, ctx):
    # the 64^3 problem (n = 262,144), FP32 inner solves, heuristic complex shifts
    P = wl.config3()
    Ad = pk.DeviceCSR.from_scipy(P.A)
    Z, stats, st = pk.care_solve(ctx, Ad, dev(P.B), dev(P.C), tol=1e-10, shifts=None, prec="fp32", rmax=2000)
    print(f"3d 64^3 fp32: status {st} relres {stats['res_rel']:.2e} t {stats['t_total']:.2f} s "
          f"iter0 {stats['iter0_outer']}({stats['iter0_inner']}) iter {stats['iter_outer']}({stats['iter_inner']})",
          flush=True)
    assert st == 0
    assert stats["res_rel"] <= 1e-10
