"""Benchmark: CARE solve time and sparse-product HBM bandwidth, FP32-inner
mixed-precision refinement vs the all-FP64 path, at relative residual
||R||_F / ||C^T C||_F <= 1e-10, on the 500 x 500 2D convection-diffusion FDM
problem (n = 250,000, 1,248,000 nonzeros, m = p = 5, Gaussian B and C from
seed 1220, 12 Wachspress (minimax) real shifts for the closed-form spectral
interval, largest magnitude first).

Prints ONE JSON line (see the keys below).  A step is one full care_solve
(initial NLR-ADI solve + refinement) with inputs resident in HBM.

Timed solves run the production path (no per-launch events, HIP-graph replay
of the Krylov chunks).  After them:
  * both precisions are timed again at tol 1e-12, the tolerance at which the
    solution meets ||X - X_ref||_F / ||X_ref||_F <= 1e-8 on this problem, and
    every solution is compared with sampled rows of the FP64 oracle's solution
    (tests/golden/config2_x_samples.json);
  * one extra FP32-inner solve in which every sparse-product launch records
    HIP events at its own start and end (hipExtLaunchKernelGGL, on the
    library's stream) gives the roofline object;
  * both precisions are timed once more with the paper's inner solver,
    restarted GMRES right-preconditioned by ILU(0) of A^T + p I
    ("paper_inner_solver"; the production path runs BiCGStab on the exact
    red-black reduction instead);
  * the CPU oracle is timed on a bounded sample of the same workload.

`--workload fdm3d` times the 64^3 rotating-field problem (n = 262,144, m = 1,
p = 10, the oracle golden's shift set with one conjugate pair), FP32 inner vs
FP64, and adds one solve each with bf16 and scaled fp16 operator values, all
against the oracle's samples of X.

`--workload toeplitz --n N` times the Toeplitz example of Sec. 5.2 instead
(B n x 10 with ||B||_F = 1, C 5 x n, one heuristic shift set shared by both
precisions); its line carries no CPU baseline, no oracle X samples and no
counter traffic.

`--workload fdm_batch` times the uneven batch of 32 2D FDM CAREs (grids
N = 100 ... 632, n = 1e4 ... 4e5, (m, p) from {1..8}) solved in one batched
call on concurrent worker streams, FP32 inner vs FP64, and prints its own
line (a step is one batched solve of all 32).  `--workload dense_batch` does
the same for the 64 dense CAREs (n = 256 ... 2048, kappa_2(A) = 1e2 ... 1e12,
LU shifted solves), with the count of instances that met the tolerance.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CARE solve time & SpMM HBM GB/s: FP32-inner vs FP64, at rel residual <=1e-10"
# HBM bytes per k_spmm launch measured with rocprofv3 counters (FETCH_SIZE,
# WRITE_SIZE, calibrated on a 1 GiB copy) for this workload; used only while
# the kernel source it was measured on is unchanged
PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_spmm_fdm2d_500_fp32_hbm_counters.md")
KERNEL_SOURCES = ("paper_2607_14742_amd/csrc/spmm_kernel.hpp", "paper_2607_14742_amd/csrc/sparse.hip")
GOLDEN = os.path.join(ROOT, "tests", "golden", "config2_x_samples.json")
GOLDEN3 = os.path.join(ROOT, "tests", "golden", "config3_x_samples.json")
HBM_PEAK_GBS = 8000.0
TOL = 1e-10
TOL_XGATE = 1e-12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=("fdm2d", "fdm3d", "toeplitz", "fdm_batch", "dense_batch"), default="fdm2d",
                    help="fdm2d: the 2D FDM problem (default); fdm3d: the 64^3 rotating-field problem "
                         "(FP32 inner vs FP64, and bf16 / fp16 products); toeplitz: the Toeplitz example of Sec. 5.2; "
                         "fdm_batch: the 32-instance uneven FDM batch; dense_batch: the 64-instance dense batch")
    ap.add_argument("--N", type=int, default=500, help="fdm2d grid size (500 -> n = 250000)")
    ap.add_argument("--batch-workers", type=int, default=4, help="fdm_batch: concurrent worker streams")
    ap.add_argument("--n", type=int, default=131072, help="toeplitz matrix size")
    ap.add_argument("--no-fp64", action="store_true", help="skip the all-FP64 comparison solves")
    ap.add_argument("--no-xgate", action="store_true", help="skip the tol 1e-12 solves")
    ap.add_argument("--no-paper-solver", action="store_true",
                    help="skip the two solves with the paper's inner solver (GMRES + ILU(0)); "
                         "--no-fp64 skips them too")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-shifts", type=int, default=12)
    ap.add_argument("--dense-sweep", action="store_true",
                    help="time the batched shifted LU (16 shifts, n = 256..2048, FP32 and FP64) with its solves, "
                         "and the FP64 Grams of the refinement's shapes on both implementations, and print that "
                         "table instead")
    ap.add_argument("--spmm-sweep", action="store_true",
                    help="time the shifted sparse product alone over k = 1..128 on the 500 x 500 2D and 64^3 3D "
                         "operators with rotated operand sets of more than 1 GiB, and print that table instead")
    return ap.parse_args()


def spmm_sweep(pk, wl, torch):
    """Standalone sweep of the shifted SELL product Y = (A^T + p I) X: for
    each operator, precision and column count k, enough rotated copies of
    (operator, X, Y) that one round moves more than 1 GiB (so the 256 MB
    Infinity Cache cannot hold the operands), mean time per product over the
    rounds, algorithmic bytes nnz (s_v + 4) + 4 (n + 1) + 2 n k s_x."""
    ctx = pk.Context(0)
    rows = []
    cases = [("fdm2d 500x500", wl.fdm2d(500), -1e3), ("fdm3d 64^3 rotating", wl.fdm3d(64, 100.0), -1e3)]
    for name, A, shift in cases:
        Ad = pk.DeviceCSR.from_scipy(A, "cuda:0")
        for prec in ("fp32", "fp64", "bf16", "fp16"):
            for k in (1, 2, 4, 8, 16, 32, 64, 128):
                _, nb = pk.spmm_timing(ctx, Ad, k, shift, prec, nsets=1, reps=1)
                per_set = nb + A.nnz * 4          # the SELL index padding is within the operator copy
                nsets = int(min(64, max(4, -(-(1 << 30) // per_set))))
                us, nb = pk.spmm_timing(ctx, Ad, k, shift, prec, nsets=nsets, reps=3)
                gbs = nb / (us * 1e-6) / 1e9
                rows.append({"operator": name, "prec": prec, "k": k, "nsets": nsets, "us": round(us, 2),
                             "bytes": int(nb), "GB/s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)})
                print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
        del Ad
    ctx.close()
    return rows


def dense_sweep(pk, wl, torch, np):
    """Host-timed sweep of the dense kernels (each call synchronises; kernel
    durations come from a profiler run of this sweep):
    * the batched LU of A^T + p_s I for 16 log-spaced shifts of the dense test
      family (A = -Q diag(logspace(0, 2, n)) Q^T), n = 256, 512, 1024, 2048,
      FP32 and FP64, then 10 solves with 16 right-hand sides;
    * the FP64 Grams X^T X at the refinement's widths (n = 250000: 206, 417,
      1026 columns; n = 125000: 1218) with the library's rule (own
      128 x 128-tile kernel where faster) and with rocBLAS only."""
    import os
    rows = []
    ctx = pk.Context(0)
    for prec in ("fp32", "fp64"):
        for n in (256, 512, 1024, 2048):
            rng = np.random.default_rng(n)
            Q = wl.haar_orthogonal(n, rng)
            At = torch.as_tensor((-(Q * np.logspace(0.0, 2.0, n)) @ Q.T).T.copy(), device="cuda:0")
            shifts = wl.logspaced_real_shifts(1.0, 100.0, 16).real
            tf = []
            for rep in range(3):
                torch.cuda.synchronize()
                t = time.perf_counter()
                F, perm, info = pk.shifted_lu_factor(ctx, At, shifts, prec=prec)
                torch.cuda.synchronize()
                tf.append(time.perf_counter() - t)
            W = torch.as_tensor(rng.standard_normal((n, 16)), device="cuda:0")
            pk.shifted_lu_solve(ctx, F[0], perm[0], W, prec=prec)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(10):
                pk.shifted_lu_solve(ctx, F[0], perm[0], W, prec=prec)
            torch.cuda.synchronize()
            ts = (time.perf_counter() - t) / 10
            fl = 16 * 2.0 / 3.0 * n ** 3
            rows.append({"kernel": "lu", "prec": prec, "n": n, "shifts": 16, "factor_ms": round(1e3 * min(tf[1:]), 3),
                         "factor_GFLOPs": round(fl / min(tf[1:]) * 1e-9, 1), "solve16_us": round(1e6 * ts, 1),
                         "info": int(sum(info))})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    ctx.close()
    for impl in ("2", "0"):
        os.environ["MPCARE_GRAM"] = impl        # read at context creation
        ctx = pk.Context(0)
        for n, q in ((250000, 206), (250000, 417), (250000, 1026), (125000, 1218)):
            X = torch.as_tensor(np.random.default_rng(q).standard_normal((n, q)), device="cuda:0")
            pk.gram(ctx, X, X)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(5):
                pk.gram(ctx, X, X)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t) / 5
            rows.append({"kernel": "gram", "impl": "rule" if impl == "2" else "rocblas", "n": n, "q": q,
                         "ms": round(1e3 * dt, 3), "TFLOPs_full_square": round(2.0 * n * q * q / dt * 1e-12, 1)})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
            del X
        ctx.close()
    os.environ.pop("MPCARE_GRAM", None)
    return rows


def fdm_batch_bench(args, pk, wl, torch, np):
    """One JSON line for the 32-instance uneven FDM batch: wall time of one
    batched care_solve_batch call (--batch-workers worker streams) per
    precision."""
    count = 32
    probs = [wl.fdm_batch_problem(i, count) for i in range(count)]
    dev = "cuda:0"
    items = [(pk.DeviceCSR.from_scipy(P.A, dev), torch.as_tensor(P.B, device=dev), torch.as_tensor(P.C, device=dev),
              P.shifts) for P in probs]
    ctx = pk.Context(0)

    def run(prec):
        times, last = [], None
        for it in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            out = pk.care_solve_batch(ctx, items, tol=TOL, prec=prec, workers=args.batch_workers)
            torch.cuda.synchronize()
            if it >= args.warmup:
                times.append(time.perf_counter() - t)
            last = out
        worst = max(s["res_rel"] for _, s, _, _ in last)
        bad = sum(1 for _, _, st, _ in last if st != 0)
        its = sum(s["krylov_iters"] for _, s, _, _ in last)
        print(f"[bench] fdm_batch {prec}: {np.mean(times):.3f} s, worst relres {worst:.2e}", file=sys.stderr,
              flush=True)
        return {"mean_s": round(float(np.mean(times)), 4), "solve_s": [round(t, 4) for t in times],
                "worst_relres": worst, "failed_instances": bad, "krylov_column_iters": its}

    r32 = run("fp32")
    res = {"metric": "CARE batch solve time, 32 uneven FDM instances, at rel residual <=1e-10",
           "value": r32["mean_s"], "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(1e3 * r32["mean_s"], 2), "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"uneven 2D FDM batch: {count} instances, n {probs[0].n}..{probs[-1].n}, "
                                  f"{sum(P.A.nnz for P in probs)} nonzeros in all, (m, p) in 1..8, "
                                  f"12 Wachspress shifts each, {args.batch_workers} worker streams, FP32 inner / FP64 refine, "
                                  f"tol {TOL:g}"},
           "fp32_inner": r32}
    if not args.no_fp64:
        r64 = run("fp64")
        res["fp64"] = r64
        res["speedup_fp32_inner_vs_fp64"] = round(r64["mean_s"] / r32["mean_s"], 3)
    ctx.close()
    print(json.dumps(res))


def dense_batch_bench(args, pk, wl, torch, np):
    """One JSON line for the 64-instance uneven dense batch (n 256 ... 2048,
    kappa_2(A) = 1e2 ... 1e12, m = p = 4, 16 log-spaced real shifts each):
    wall time of one batched care_solve_batch call per precision, with the
    count of instances that met the tolerance.  Beyond kappa ~ 1e6.5 no FP64
    method reaches tol 1e-10 (the solver stops on stagnation at the oracle's
    level), and from kappa ~ 1e8 the FP32 inner solves fail, as in Table 1."""
    count = 64
    dev = "cuda:0"
    items, kappas = [], []
    for i in range(count):
        A, B, C, q = wl.dense_instance(i, count)
        items.append((torch.as_tensor(A, device=dev), torch.as_tensor(B, device=dev),
                      torch.as_tensor(C, device=dev), wl.logspaced_real_shifts(1.0, 10.0 ** q, 16)))
        kappas.append(10.0 ** q)
    ctx = pk.Context(0)

    def run(prec):
        times, last = [], None
        for it in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            out = pk.care_solve_batch(ctx, items, tol=TOL, prec=prec, workers=args.batch_workers)
            torch.cuda.synchronize()
            if it >= args.warmup:
                times.append(time.perf_counter() - t)
            last = out
        ok = [i for i, (_, s_, st, _) in enumerate(last) if st == 0 and s_["res_rel"] <= TOL]
        stag = sum(1 for _, _, st, _ in last if st == 1)
        worst_ok = max((last[i][1]["res_rel"] for i in ok), default=None)
        print(f"[bench] dense_batch {prec}: {np.mean(times):.3f} s, {len(ok)} of {count} at tol",
              file=sys.stderr, flush=True)
        return {"mean_s": round(float(np.mean(times)), 4), "solve_s": [round(t, 4) for t in times],
                "instances_at_tol": len(ok), "stagnated": stag, "other_status": count - len(ok) - stag,
                "worst_relres_at_tol": worst_ok,
                "largest_kappa_at_tol": max((kappas[i] for i in ok), default=None)}

    r32 = run("fp32")
    res = {"metric": "CARE batch solve time, 64 dense instances, at rel residual <=1e-10",
           "value": r32["mean_s"], "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(1e3 * r32["mean_s"], 2), "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"uneven dense batch: {count} instances, n in {sorted(set(wl.DENSE_SIZES))}, "
                                  "A = -Q diag(logspace(0, q, n)) Q^T with kappa_2 = 10^q, q = 2 ... 12, "
                                  "m = p = 4, 16 log-spaced real shifts each, LU shifted solves, "
                                  f"{args.batch_workers} worker streams, FP32 inner / FP64 refine, tol {TOL:g}"},
           "fp32_inner": r32}
    if not args.no_fp64:
        r64 = run("fp64")
        res["fp64"] = r64
        res["speedup_fp32_inner_vs_fp64"] = round(r64["mean_s"] / r32["mean_s"], 3)
        # the a-priori choice of the inner precision per instance (FP32 where
        # the estimate of kappa_F(L) u_32 allows it, FP64 elsewhere)
        ra = run("auto")
        res["auto"] = ra
        res["speedup_auto_vs_fp64"] = round(r64["mean_s"] / ra["mean_s"], 3)
    ctx.close()
    print(json.dumps(res))


def measured_traffic():
    """(bytes per launch, note) from the committed counter summary, or
    (None, reason) when it is missing or was taken on other kernel source."""
    import hashlib
    import re
    try:
        text = open(PMC_SUMMARY).read()
    except OSError:
        return None, "no counter summary"
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.]+)", text)
    k = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    if not m or not k:
        return None, "counter summary incomplete"
    if k.group(1) != h.hexdigest():
        return None, "kernel changed since the counters were taken"
    return float(m.group(1)), os.path.relpath(PMC_SUMMARY, ROOT)


def oracle_sample_errors(Z, golden, torch):
    """Relative errors of X = Z Z^T against the oracle's sampled rows: the
    entries X[I, I] and the Gaussian sketch X[I, :] Omega (I and Omega drawn
    as the golden's writer drew them)."""
    import numpy as np
    rng = np.random.default_rng(golden["sample_seed"])
    n = Z.shape[0]
    rows = np.sort(rng.choice(n, len(golden["rows"]), replace=False))
    assert list(rows) == golden["rows"]
    omega = torch.as_tensor(rng.standard_normal((n, len(golden["sketch"][0]))), device=Z.device)
    Zi = Z[torch.as_tensor(rows, device=Z.device)]
    block = (Zi @ Zi.T).cpu().numpy()
    sketch = (Zi @ (Z.T @ omega)).cpu().numpy()
    b0, s0 = np.asarray(golden["block"]), np.asarray(golden["sketch"])
    return (float(np.linalg.norm(block - b0) / np.linalg.norm(b0)),
            float(np.linalg.norm(sketch - s0) / np.linalg.norm(s0)))


def cpu_baseline(P, nshift_sample):
    """Time the CPU FP64 oracle on a bounded sample of the same workload and
    scale it by the oracle's own work counts for the complete solve.

    Sample: the first LR-ADI steps of the oracle's first Newton step (W = C^T,
    one step per shift for `nshift_sample` shifts: one SuperLU factorisation
    of A^T + p I and m = 5 column solves each) and one Algorithm-1 residual
    evaluation at the oracle's final rank.  Counts: the factorisations,
    column solves and residual evaluations of the oracle's complete NLR-ADI
    solve to relres 1e-13, recorded by tests/golden/make_config2_x_samples.py
    (which also records the complete solve's own wall time in this
    repository's build container)."""
    import numpy as np

    from oracle import adi, lowrank
    golden = json.load(open(GOLDEN))
    work = golden["oracle"].get("work")
    t0 = time.perf_counter()
    solver = adi.ShiftedSolver(P.A, None, None)
    W = P.C.T.copy()
    for j in range(nshift_sample):
        p = P.shifts[j % len(P.shifts)].real
        V = solver.solve(p, W)
        W = W - 2 * p * V
    c = solver.counts
    t_fac = c["factor_s"] / max(c["factorizations"], 1)
    t_col = c["solve_s"] / max(c["columns"], 1)
    rank = golden["oracle"]["rank"]
    Zs = np.random.default_rng(0).standard_normal((P.n, rank)) * 1e-3
    t1 = time.perf_counter()
    lowrank.residual_norm(P.A, P.B, P.C, Zs)
    t_res = time.perf_counter() - t1
    sample_s = time.perf_counter() - t0
    threads = os.environ.get("OMP_NUM_THREADS") or str(os.cpu_count())
    out = {"unit": "s", "cores": int(threads), "kind": "oracle",
           "sample": (f"oracle (SciPy SuperLU, single-threaded solves; NumPy QR on {threads} threads) on the "
                      f"500 x 500 workload: {c['factorizations']} factorisations of A^T + p I "
                      f"({t_fac:.2f} s each), {c['columns']} column solves ({t_col * 1e3:.1f} ms each), one "
                      f"residual evaluation at rank {rank} ({t_res:.2f} s)"),
           "sample_seconds": round(sample_s, 2)}
    if work:
        est = work["factorizations"] * t_fac + work["columns"] * t_col + work["residual_evaluations"] * t_res
        # the rest of the oracle's work (Kleinman residuals, factor
        # compression, feedback updates) in the proportion the complete solve
        # showed where it was run whole
        whole = work["factor_s"] + work["solve_s"] + work["residual_evaluations"] * work["residual_s_final_rank"]
        ratio = work["nlradi_s"] / whole if whole > 0 else 1.0
        out["value"] = round(est * ratio, 2)
        out["scaled_by"] = (f"the oracle's complete solve (relres {golden['relres']:.1e}): "
                            f"{work['factorizations']} factorisations, {work['columns']} column solves, "
                            f"{work['residual_evaluations']} residual evaluations ({est:.1f} s at the sampled "
                            f"rates), times {ratio:.2f} for the rest of its work: the complete solve took "
                            f"{work['nlradi_s']} s where it was run whole ({work['threads']} threads), of which "
                            f"those three kinds of work took {whole:.1f} s")
    else:
        out["value"] = round(sample_s, 2)
        out["scaled_by"] = "no work counts in the golden: value is the sample itself"
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; runs on several GPUs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2607_14742_amd as pk
    import workloads as wl

    if args.spmm_sweep:
        rows = spmm_sweep(pk, wl, torch)
        best = max(rows, key=lambda r: r["GB/s"])
        print(json.dumps({"metric": "SpMM HBM GB/s (standalone, rotated operands > 1 GiB)", "value": best["GB/s"],
                          "unit": "GB/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
                          "peak": HBM_PEAK_GBS, "rows": rows}))
        return

    if args.dense_sweep:
        rows = dense_sweep(pk, wl, torch, np)
        best = max(r["factor_GFLOPs"] for r in rows if r["kernel"] == "lu" and r["prec"] == "fp32")
        print(json.dumps({"metric": "batched shifted LU GFLOP/s (16 shifts, FP32, best order)", "value": best,
                          "unit": "GFLOP/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
                          "rows": rows}))
        return

    if args.workload == "fdm_batch":
        fdm_batch_bench(args, pk, wl, torch, np)
        return
    if args.workload == "dense_batch":
        dense_batch_bench(args, pk, wl, torch, np)
        return

    dev = "cuda:0"
    # a plain 1 GiB device-to-device copy before anything else: the reference
    # the HBM byte counters of a profiled run are calibrated against
    cal = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    cal.fill_(1.0)
    torch.empty_like(cal).copy_(cal)
    torch.cuda.synchronize()
    del cal

    ctx = pk.Context(0)
    golden = None
    if args.workload == "fdm2d":
        P = wl.fdm2d_problem(args.N, 5, 5, name=f"fdm2d_{args.N}x{args.N}")
        A = pk.DeviceCSR.from_scipy(P.A, dev)
        shifts = P.shifts
        wdesc = (f"2D convection-diffusion FDM {args.N}x{args.N} (n={P.n}, nnz={P.A.nnz}), m=p=5, "
                 f"{len(shifts)} Wachspress real shifts, FP32 inner / FP64 refine, tol {TOL:g}")
        if args.N == 500 and os.path.exists(GOLDEN):
            golden = json.load(open(GOLDEN))
    elif args.workload == "fdm3d":
        # the 64^3 rotating-field problem with the shift set the oracle's
        # golden was computed with (heuristic shifts, one conjugate pair)
        P = wl.config3()
        A = pk.DeviceCSR.from_scipy(P.A, dev)
        golden = json.load(open(GOLDEN3))
        shifts = np.array(golden["shifts"]["re"]) + 1j * np.array(golden["shifts"]["im"])
        wdesc = (f"3D convection-diffusion FDM 64^3 with a rotating field (n={P.n}, nnz={P.A.nnz}), m=1, p=10, "
                 f"{len(shifts)} heuristic shifts (one conjugate pair), FP32 inner / FP64 refine, tol {TOL:g}")
    else:
        # the paper generates its shifts from Krylov subspaces: one heuristic
        # set (GPU Arnoldi, before the timed region) serves both precisions
        P = wl.toeplitz_problem(args.n)
        A = pk.DeviceCSR.from_scipy(P.A, dev)
        shifts = pk.penzl_shifts(ctx, A)
        wdesc = (f"Toeplitz example of Sec. 5.2 (n={P.n}, nnz={P.A.nnz}), m=10, p=5, ||B||_F=1, "
                 f"{len(shifts)} heuristic shifts, FP32 inner / FP64 refine, tol {TOL:g}")
    B = torch.as_tensor(P.B, device=dev)
    C = torch.as_tensor(P.C, device=dev)
    m, p = P.B.shape[1], P.C.shape[0]

    def solve(prec, profile, tol=TOL, **kw):
        torch.cuda.synchronize()
        t = time.perf_counter()
        Z, stats, st = pk.care_solve(ctx, A, B, C, tol=tol, shifts=shifts, prec=prec, profile=profile,
                                     rmax=2048, **kw)
        torch.cuda.synchronize()
        return time.perf_counter() - t, Z, stats, st

    def run(prec, warmup, steps, tol=TOL):
        for _ in range(warmup):
            solve(prec, 0, tol)
        times, last = [], None
        for _ in range(steps):
            el, Z, stats, st = solve(prec, 0, tol)
            times.append(el)
            last = (Z, stats, st)
        return times, last

    def summary(times, st, s, Z):
        d = {"status": st, "relres": s["res_rel"], "res_paper": s["res_paper"],
             "iter0": f"{s['iter0_outer']}({s['iter0_inner']})", "iter": f"{s['iter_outer']}({s['iter_inner']})",
             "rank": s["rank"], "krylov_column_iters": s["krylov_iters"], "mean_s": round(float(np.mean(times)), 4),
             "solve_s": [round(t, 4) for t in times]}
        if golden is not None:
            eb, es = oracle_sample_errors(Z, golden, torch)
            d["xerr_vs_oracle_samples"] = {"block": eb, "sketch": es}
        return d

    t32, (Z32, s32, st32) = run("fp32", args.warmup, args.steps)
    res = {
        "metric": METRIC,
        "value": round(float(np.mean(t32)), 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * float(np.mean(t32)), 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wdesc, "n": P.n, "nnz": int(P.A.nnz), "m": m, "p": p, "tol": TOL},
        "fp32_inner": summary(t32, st32, s32, Z32),
    }
    if not args.no_fp64:
        t64, (Z64, s64, st64) = run("fp64", args.warmup, args.steps)
        res["fp64"] = summary(t64, st64, s64, Z64)
        res["speedup_fp32_inner_vs_fp64"] = round(float(np.mean(t64)) / float(np.mean(t32)), 3)
        # X agreement of the two GPU solutions (factored, cancellation free)
        Y = torch.cat([Z32, Z64], dim=1)
        _, R = torch.linalg.qr(Y)
        T1, T2 = R[:, :Z32.shape[1]], R[:, Z32.shape[1]:]
        res["xdiff_fp32_vs_fp64"] = float(torch.linalg.norm(T1 @ T1.T - T2 @ T2.T) / torch.linalg.norm(T2 @ T2.T))
        del Z64, Y
    if not args.no_xgate:
        # the X-gate tolerance: the first-order reach of a 1e-10 residual in X
        # exceeds 1e-8 on this problem, 1e-12 meets it
        xs = max(1, args.steps // 4)
        xg = {"tol": TOL_XGATE, "steps": xs}
        tx32, (Zx, sx, stx) = run("fp32", 1, xs, TOL_XGATE)
        xg["fp32_inner"] = summary(tx32, stx, sx, Zx)
        if not args.no_fp64:
            tx64, (Zx64, sx64, stx64) = run("fp64", 1, xs, TOL_XGATE)
            xg["fp64"] = summary(tx64, stx64, sx64, Zx64)
            xg["speedup_fp32_inner_vs_fp64"] = round(float(np.mean(tx64)) / float(np.mean(tx32)), 3)
            del Zx64
        del Zx
        res["xgate"] = xg
    if not args.no_paper_solver and not args.no_fp64:
        # the inner solver of the paper's GPU runs: restarted GMRES (30 / 50)
        # right-preconditioned by ILU(0) of A^T + p I (multicolour order, no
        # red-black reduction); one solve per precision, factorisations included
        ps = {"method": "GMRES(30 FP32 / 50 FP64) + ILU(0) of A^T + p I, full system"}
        kw = dict(krylov_method=1, krylov_rb=0, krylov_precond=1)
        for prec in ("fp32", "fp64"):
            el, Zp, sp_, stp = solve(prec, 0, **kw)
            ps["fp32_inner" if prec == "fp32" else "fp64"] = {
                "status": stp, "solve_s": round(el, 4), "relres": sp_["res_rel"],
                "iter": f"{sp_['iter_outer']}({sp_['iter_inner']})", "krylov_column_iters": sp_["krylov_iters"]}
            del Zp
        ps["speedup_fp32_inner_vs_fp64"] = round(ps["fp64"]["solve_s"] / ps["fp32_inner"]["solve_s"], 3)
        res["paper_inner_solver"] = ps
    if args.workload == "fdm3d":
        # FP32 inner solves whose products read A's values in bf16 or in
        # scaled fp16 (one solve each, errors against the oracle's samples)
        for prec in ("bf16", "fp16"):
            el, Zh, sh_, sth = solve(prec, 0)
            res[prec + "_products"] = summary([el], sth, sh_, Zh)
            del Zh

    # roofline: one more FP32-inner solve in which every sparse-product launch
    # records HIP events at its own start and end on the library's stream
    # (outside the timed region; the per-launch events switch graph replay off)
    _, _, sp32, _ = solve("fp32", 1)
    calls, nbytes, tsp = sp32["spmm_calls"], sp32["spmm_bytes"], sp32["t_spmm"]
    spmm_gbs = nbytes / tsp / 1e9 if tsp > 0 else None
    traffic, tnote = measured_traffic() if args.workload == "fdm2d" and args.N == 500 else \
        (None, "counters were taken on the 500 x 500 FDM workload only")
    res["roofline"] = {"bound": "hbm",
                       "kernel": "k_spmm (SELL-64 shifted product of A^T; every launch of one FP32-inner solve: "
                                 "BiCGStab products with their dots, and plain products)",
                       "achieved": round(spmm_gbs, 1) if spmm_gbs else None, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(spmm_gbs / HBM_PEAK_GBS, 4) if spmm_gbs else None,
                       "traffic": round(traffic) if traffic else None, "traffic_source": tnote,
                       "launches": calls, "avg_launch_us": round(1e6 * tsp / calls, 2) if calls else None,
                       "algorithmic_bytes_per_launch": round(nbytes / calls) if calls else None,
                       "profiled_solve_s": round(sp32["t_total"], 4)}
    # FP64 Gram of the residual factor's orthogonalisation (Algorithm 1: F is
    # n x (2 r + p) at the final FP32-inner rank), on the matrix cores:
    # 2 n q^2 flop per call, wall time per call after a warm-up
    q = 2 * s32["rank"] + p
    Fg = torch.randn(q, P.n, dtype=torch.float64, device=dev).t()   # column-major n x q
    for _ in range(2):
        pk.gram(ctx, Fg, Fg)
    torch.cuda.synchronize()
    tg = time.perf_counter()
    reps = 10
    for _ in range(reps):
        pk.gram(ctx, Fg, Fg)
    torch.cuda.synchronize()
    tg = (time.perf_counter() - tg) / reps
    gflop = 2.0 * P.n * q * q / 1e9
    res["gram_fp64"] = {"n": P.n, "q": q, "ms_per_call": round(1e3 * tg, 3),
                        "achieved": round(gflop / tg / 1e3, 1), "peak": 78.6, "unit": "TFLOP/s",
                        "frac": round(gflop / tg / 1e3 / 78.6, 4)}
    del Fg
    ctx.close()
    if args.workload == "toeplitz":
        # context only: the paper's V100 times for this example (n = 131072:
        # FP64 92.07 s, FP32 63.44 s; ILU(0)-GMRES, another machine)
        res["paper_context"] = "Sec. 5.2 Toeplitz table, one V100, n = 131072: FP64 92.07 s, FP32-inner 63.44 s"
    elif args.workload == "fdm2d" and not args.no_cpu_baseline and args.N == 500:
        res["cpu_baseline"] = cpu_baseline(P, args.cpu_sample_shifts)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
