"""Writes config4_x_samples.json: for each of the 64 dense CAREs of the
uneven dense batch (n in {256, ..., 2048}, kappa_2(A) = 10^q, q = 2 ... 12,
m = p = 4, seed 1220 + i), sampled entries of the oracle's stabilizing
solution X by the Hamiltonian Schur method (oracle.riccati.care_hamiltonian)
polished by dense Newton-Kleinman steps (oracle.riccati.newton_kleinman_dense,
kept only if they lower the residual), for the full-batch GPU test.  Calls only the oracle and the input generators.

Per instance (rows I: 8 distinct indices, Omega: n x 8 standard normal, drawn
in this order from numpy.random.default_rng(SAMPLE_SEED + i)):
  block = X[I, I];  sketch = X[I, :] Omega;  x_fro = ||X||_F;
  relres = ||R(X)||_F / ||C^T C||_F of the oracle's X (its own accuracy),
  relres_schur the same before the polish.

Run from the repository root:  python tests/golden/make_config4_x_samples.py"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import riccati  # noqa: E402

SAMPLE_SEED = 20264
NROWS, NSKETCH = 8, 8
COUNT = 64
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config4_x_samples.json")


def sample_rows_and_sketch(n, i):
    rng = np.random.default_rng(SAMPLE_SEED + i)
    rows = np.sort(rng.choice(n, NROWS, replace=False))
    omega = rng.standard_normal((n, NSKETCH))
    return rows, omega


def main():
    insts = []
    t_all = time.time()
    for i in range(COUNT):
        A, B, C, q = wl.dense_instance(i, COUNT)
        t0 = time.time()
        Xh = riccati.care_hamiltonian(A, B, C)
        rel_h = float(np.linalg.norm(riccati.riccati_residual(A, B, C, Xh)) / np.linalg.norm(C @ C.T))
        # Newton-Kleinman polish from the Schur solution (quadratic
        # convergence; stops when the residual no longer drops)
        X, hist = riccati.newton_kleinman_dense(A, B, C, X0=Xh, tol=1e-15, kmax=4)
        rel = float(hist[-1]) if hist else rel_h
        if rel > rel_h:
            X, rel = Xh, rel_h
        dt = time.time() - t0
        rows, omega = sample_rows_and_sketch(A.shape[0], i)
        insts.append(dict(i=i, n=int(A.shape[0]), q=float(q), rows=[int(r) for r in rows],
                          block=X[np.ix_(rows, rows)].tolist(), sketch=(X[rows] @ omega).tolist(),
                          x_fro=float(np.linalg.norm(X)), relres=rel, relres_schur=rel_h, seconds=round(dt, 2)))
        print(f"{i:2d} n={A.shape[0]} q={q:.2f} relres {rel:.2e} (Schur {rel_h:.2e}) {dt:.1f} s", flush=True)
    with open(OUT, "w") as f:
        json.dump(dict(routine="oracle.riccati.care_hamiltonian (FP64)", sample_seed=SAMPLE_SEED,
                       nrows=NROWS, nsketch=NSKETCH, instances=insts,
                       seconds=round(time.time() - t_all, 1)), f)
    print(f"wrote {OUT}", flush=True)


if __name__ == "__main__":
    main()
