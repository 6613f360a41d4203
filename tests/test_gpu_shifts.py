"""GPU parity of the shift heuristic (GPU Arnoldi with A^T and A^-T, host
Hessenberg QR and greedy choice) against the CPU oracle, and the plain FP64
Newton solve of the 20 x 20 FDM problem with real heuristic shifts against a
dense Schur solution."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as wl
from oracle import lowrank, riccati
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


def _minmax(P, R):
    """max over candidates of prod |(t - p)/(t + p)| (the quantity the greedy
    choice drives down)."""
    s = np.ones(R.size)
    for p in P:
        s *= np.abs((R - p) / (R + p))
    return s.max()


CASES = {
    "fdm2d_30": (lambda: wl.fdm2d(30, 10.0), False),
    "fdm2d_30_real": (lambda: wl.fdm2d(30, 10.0), True),
    "fdm3d_8_rotating": (lambda: wl.fdm3d(8, 100.0, "rotating"), False),
    "diag_4_values": (lambda: sp.diags(np.repeat([-2.0, -11.0, -60.0, -400.0], [60, 50, 70, 40])).tocsr(), False),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_penzl_shifts_match_oracle(pk, ctx, case):
    make, real = CASES[case]
    A = make()
    print(f"penzl case {case} n={A.shape[0]}", flush=True)
    got = pk.penzl_shifts(ctx, pk.DeviceCSR.from_scipy(A), l0=16, kp=20, km=10, real_only=real)
    ref = osh.penzl_shifts(A, 16, 20, 10, real_only=real)
    assert np.all(got.real < 0)
    # pairs adjacent, Im > 0 first
    i = 0
    while i < got.size:
        if got[i].imag != 0:
            assert got[i].imag > 0 and got[i + 1] == np.conj(got[i])
            i += 2
        else:
            i += 1
    assert got.shape == ref.shape
    if case == "diag_4_values":
        # the forward and inverse runs both find the 4 eigenvalues exactly, so
        # after the first four choices the candidates left are rounding-level
        # duplicates whose order is not unique: compare the sets
        assert np.allclose(np.sort_complex(got), np.sort_complex(ref), rtol=1e-10), (got, ref)
        assert np.allclose(np.sort(got[:4].real), [-400.0, -60.0, -11.0, -2.0], rtol=1e-10)
    else:
        assert np.allclose(got, ref, rtol=1e-7, atol=0), (got, ref)
    if real:
        assert np.all(got.imag == 0)
    R = osh.ritz_candidates(A, 20, 10, real)
    assert abs(_minmax(got, R) - _minmax(ref, R)) <= 1e-6


def test_config1_newton_with_real_heuristic_shifts_vs_schur(pk, ctx):
    P = wl.config1()
    Ad = pk.DeviceCSR.from_scipy(P.A)
    Z, stats, st = pk.care_solve(ctx, Ad, dev(P.B), dev(P.C), tol=1e-10, shifts=None, prec="fp64",
                                 penzl_real=1)
    assert st == 0, stats
    Z = Z.cpu().numpy()
    Xs = riccati.care_schur(P.A, P.B, P.C)
    rel = lowrank.residual_norm(P.A, P.B, P.C, Z) / np.linalg.norm(P.C @ P.C.T)
    assert rel <= 1e-10
    assert np.linalg.norm(Z @ Z.T - Xs) <= 1e-8 * np.linalg.norm(Xs)
