"""Writes config3_x_samples.json: the shift set and sampled entries of the
FP64 oracle's CARE solution X = Z Z^T for the 64^3 rotating-field
convection-diffusion problem (n = 262,144, m = 1, p = 10, seed 1220), for the
full-size GPU parity test.  Calls only the oracle and the input generators.

Shifts: the oracle's Penzl heuristic (16 shifts, 20 Arnoldi steps with A^T,
10 with A^-T; complex-conjugate pairs), applying A^-T with the plane-wise
direct solver.  Solution: oracle NLR-ADI to relres 1e-13, every shifted solve
done by oracle.adi.KronZShiftedSolver (the matrix is I (x) A_xy + T_z (x) I:
a sine transform along z and 64 sparse LU solves of order 4096 per shift,
exact up to rounding; a sparse LU of the whole 3D matrix has ~1e9 nonzeros).

Stored (rows I: 32 distinct indices, Omega: n x 16 standard normal, both
drawn in this order from numpy.random.default_rng(SAMPLE_SEED)):
  block  = X[I, I];  sketch = X[I, :] Omega;  x_fro = ||X||_F;
  relres = ||R(X)||_F / ||C^T C||_F of the oracle's Z;  shifts (re, im).

Run from the repository root:  python tests/golden/make_config3_x_samples.py"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import adi, care, lowrank  # noqa: E402
from oracle import shifts as osh  # noqa: E402

SAMPLE_SEED = 20263
NROWS, NSKETCH = 32, 16
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config3_x_samples.json")


def sample_rows_and_sketch(n):
    rng = np.random.default_rng(SAMPLE_SEED)
    rows = np.sort(rng.choice(n, NROWS, replace=False))
    omega = rng.standard_normal((n, NSKETCH))
    return rows, omega


def main():
    P = wl.config3()
    t0 = time.time()
    cache = {}

    def factory(A, B, K):
        return adi.KronZShiftedSolver(A, B, K, cache=cache)
    base = factory(P.A, None, None)
    shifts = osh.penzl_shifts(P.A, 16, 20, 10, inv_apply=lambda v: base.solve_base(0.0, v))
    t_sh = time.time() - t0
    print(f"shifts ({t_sh:.1f} s): {shifts}", flush=True)
    Z, info = care.nlradi(P.A, P.B, P.C, shifts, tol=1e-13, adi_tol=1e-13, solver_factory=factory)
    nrm = np.linalg.norm(P.C @ P.C.T, "fro")
    rel = lowrank.residual_norm(P.A, P.B, P.C, Z) / nrm
    rows, omega = sample_rows_and_sketch(P.n)
    Zi = Z[rows]
    out = dict(
        problem=dict(name=P.name, N=64, m=1, p=10, seed=wl.DEFAULT_SEED, nu=100.0, field="rotating"),
        shifts=dict(re=[float(s.real) for s in shifts], im=[float(s.imag) for s in shifts],
                    routine="oracle.shifts.penzl_shifts(l0=16, kp=20, km=10)"),
        oracle=dict(routine="oracle.care.nlradi with oracle.adi.KronZShiftedSolver (FP64)", tol=1e-13,
                    adi_tol=1e-13, outer=info["outer"], inner=info["inner"],
                    hist=[float(h) for h in info["hist"]], rank=int(Z.shape[1]),
                    seconds=round(time.time() - t0, 1)),
        sample_seed=SAMPLE_SEED, rows=[int(r) for r in rows],
        block=(Zi @ Zi.T).tolist(), sketch=(Zi @ (Z.T @ omega)).tolist(),
        x_fro=lowrank.factored_norm(Z), relres=float(rel))
    with open(OUT, "w") as f:
        json.dump(out, f)
    print(f"wrote {OUT}: rank {Z.shape[1]}, relres {rel:.3e}, ||X||_F {out['x_fro']:.6e}, "
          f"{out['oracle']['seconds']} s", flush=True)


if __name__ == "__main__":
    main()
