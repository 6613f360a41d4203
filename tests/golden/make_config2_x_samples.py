"""Writes config2_x_samples.json: sampled entries of the FP64 oracle's CARE
solution X = Z Z^T for the 500 x 500 convection-diffusion problem (n =
250,000, m = p = 5, seed 1220, 12 Wachspress shifts), for the full-size GPU
parity test.  Calls only the oracle and the input generators.

Stored (rows I: 32 distinct indices, Omega: n x 16 standard normal, both
drawn in this order from numpy.random.default_rng(SAMPLE_SEED)):
  block  = X[I, I]          (32 x 32 entries, computed one by one from Z)
  sketch = X[I, :] Omega    (32 x 16; a Gaussian sketch of the 32 rows)
  x_fro  = ||X||_F, relres = ||R(X)||_F / ||C^T C||_F of the oracle's Z;
  the oracle's work: sparse LU factorizations and column solves with the
  seconds spent in each, residual evaluations (the CPU baseline of the
  benchmark scales its timed sample by these counts).

Run from the repository root:  python tests/golden/make_config2_x_samples.py
(about four minutes on 8 CPU threads; the SuperLU factorisations of the
shifted matrices and the column steps dominate)."""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import adi, care, lowrank  # noqa: E402

SAMPLE_SEED = 20260
NROWS, NSKETCH = 32, 16
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config2_x_samples.json")


def sample_rows_and_sketch(n):
    rng = np.random.default_rng(SAMPLE_SEED)
    rows = np.sort(rng.choice(n, NROWS, replace=False))
    omega = rng.standard_normal((n, NSKETCH))
    return rows, omega


def main():
    P = wl.config2()
    solvers = []

    def factory(A, B, K):
        s = adi.ShiftedSolver(A, B, K)
        solvers.append(s)
        return s
    t0 = time.time()
    Z, info = care.nlradi(P.A, P.B, P.C, P.shifts, tol=1e-13, adi_tol=1e-13, solver_factory=factory)
    t_solve = time.time() - t0
    nrm = np.linalg.norm(P.C @ P.C.T, "fro")
    t1 = time.time()
    rel = lowrank.residual_norm(P.A, P.B, P.C, Z) / nrm
    t_res = time.time() - t1
    work = dict(factorizations=sum(s.counts["factorizations"] for s in solvers),
                factor_s=round(sum(s.counts["factor_s"] for s in solvers), 2),
                columns=sum(s.counts["columns"] for s in solvers),
                solve_s=round(sum(s.counts["solve_s"] for s in solvers), 2),
                residual_evaluations=info["outer"], residual_s_final_rank=round(t_res, 2),
                nlradi_s=round(t_solve, 1), threads=os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count()))
    rows, omega = sample_rows_and_sketch(P.n)
    Zi = Z[rows]
    block = Zi @ Zi.T
    sketch = Zi @ (Z.T @ omega)
    out = dict(
        problem=dict(name=P.name, N=500, m=5, p=5, seed=wl.DEFAULT_SEED,
                     shift_set=P.meta["shift_set"], nshifts=int(P.shifts.size)),
        oracle=dict(routine="oracle.care.nlradi (sparse LU per shift, FP64)", tol=1e-13, adi_tol=1e-13,
                    outer=info["outer"], inner=info["inner"], hist=[float(h) for h in info["hist"]],
                    rank=int(Z.shape[1]), seconds=round(time.time() - t0, 1), work=work),
        sample_seed=SAMPLE_SEED, rows=[int(r) for r in rows],
        block=block.tolist(), sketch=sketch.tolist(),
        x_fro=lowrank.factored_norm(Z), relres=float(rel))
    with open(OUT, "w") as f:
        json.dump(out, f)
    print(f"wrote {OUT}: rank {Z.shape[1]}, relres {rel:.3e}, ||X||_F {out['x_fro']:.6e}, "
          f"{out['oracle']['seconds']} s", flush=True)


if __name__ == "__main__":
    main()
