"""Benchmark: right-hand-side solves per second of block CG on one MI355X.

A step is one complete solve A X = B from X = 0 to the stop rule (every
column's residual reduced by 1e-8) of the synthetic 3D 7-point Poisson
system on a 256^3 grid (n = 16,777,216) with k = 128 uniform right-hand
sides, hybrid subalgebra with p = 16, in the FP32 + FP64-refinement form
(FP32 block CG whose search direction is kept across FP64 corrections by
residual replacement), with every kernel of the iteration on the GPU and B,
X, A resident in HBM before the timed region. value = k * steps / wall time.

Also reported on the same JSON line:
  compare       the plain FP64 solve of the same system (its rate, the
                speedup of the headline form, the difference of the two
                solutions);
  roofline      the dominant kernel's algorithmic bytes per launch over its
                event-measured average duration (events on the library's
                stream, launches that returned at entry excluded);
  cpu_baseline  the FP64 CPU oracle on this host: a bounded number of its
                iterations (on two sampled column groups for the hybrid
                subalgebra, whose groups are independent block CG solves),
                scaled to the whole solve;
  kernels       per-class time breakdown of the last warm-up solve;
  variants      the other subalgebras of the workload (one timed solve each
                in both forms), when they fit the time budget.
"""
from __future__ import annotations

import argparse
import hashlib
import itertools
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RHS-solves/s to 1e-8 rel residual (FP32+refine vs FP64) + achieved HBM GB/s"
PEAK_HBM_GBS = 8000.0


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def algorithmic_bytes(cls: str, n: int, nnz: int, k: int, precision: str) -> float:
    """Bytes one launch of a kernel class must move (each operand once)."""
    vb = 8 if precision == "fp64" else 4
    if cls == "spmm":            # A (values + column index + row pointer), P read, Q written
        return vb * nnz + 4 * nnz + 4 * (n + 1) + 2 * vb * n * k
    if cls == "update_r":        # Q, R read; R written
        return 3 * vb * n * k
    if cls == "update_xp":       # X, P, R read; X, P written
        return 5 * vb * n * k
    raise ValueError(cls)


def solve_bytes(kernels: dict, n: int, nnz: int, k: int, precision: str) -> float:
    """Algorithmic bytes of one solve's row passes: launches per class (of a
    profiled solve) times the class's bytes per launch."""
    return sum(algorithmic_bytes(c, n, nnz, k, precision) * kernels[c]["launches"]
               for c in ("spmm", "update_r", "update_xp") if c in kernels)


# sources that determine the HBM traffic of the row kernels: the kernels,
# their launch plan and the stencil row order
TRAFFIC_SOURCES = ("bcg_mfma.hip", "bcg_fast.hip", "bcg_internal.h", "bcg_stencil.hip")


def kernel_hash() -> str:
    """Hash of the row-kernel sources' code: // comments and blank lines are
    dropped (the sources hold no // inside string literals), so a comment edit
    keeps committed counter runs current."""
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_1912_11930_amd", "csrc", f), encoding="utf-8") as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def data_type(precision: str) -> str:
    """Element type of the row kernels: fp64, or fp32 for both mixed forms."""
    return "fp64" if precision == "fp64" else "fp32"


def measured_traffic(kernel: str, workload: str, variant: str, precision: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if current."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))[f"{kernel}/{workload}/{variant}/{data_type(precision)}"]
    except (KeyError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


# row kernels of each class (matrix-core and k-specialised variants)
KERNEL_NAMES = {"spmm": ("k_spmm_mfma", "k_spmm_fast"), "update_r": ("k_update_r_mfma", "k_update_r_fast"),
                "update_xp": ("k_update_xp_mfma", "k_update_xp_fast")}
COPY_BYTES = 2 << 30


def copy_calibration() -> int:
    """A plain device copy of COPY_BYTES (counter calibration for --traffic-from)."""
    import torch
    a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "copies": 3}), flush=True)
    return 0


def _pmc_means(db_path: str, counter: str) -> dict:
    """Per-kernel mean counter value over dispatches that did work, and their
    number: {kernel: (mean, dispatches)}."""
    import sqlite3
    db = sqlite3.connect(db_path)
    cols = [r[1] for r in db.execute("pragma table_info(counters_collection)")]
    ci = {c: i for i, c in enumerate(cols)}
    per = {}
    for r in db.execute("select * from counters_collection"):
        if r[ci["counter_name"]] != counter:
            continue
        per.setdefault(r[ci["kernel_name"]], []).append(float(r[ci["value"]]))
    out = {}
    for name, vals in per.items():
        top = max(vals)
        work = [v for v in vals if v > 0.01 * top]  # launches that returned at entry are dropped
        out[name] = (sum(work) / len(work) if work else 0.0, len(work))
    return out


def _is_fp32_kernel(name: str) -> bool:
    return "_f32" in name or "<float" in name


def traffic_from(directory: str, workload: str, variant: str, path: str | None = None) -> int:
    """Write profiles/traffic.json (or `path`) from four rocprofv3 --pmc
    databases under `directory`: copy_fetch, copy_write (bench.py
    --copy-calibration) and fetch, write (the benchmark, both precisions).
    FETCH_SIZE / WRITE_SIZE are KiB per dispatch; each is scaled so that the
    plain copy reads and writes COPY_BYTES."""
    import glob

    def db(sub):
        return glob.glob(os.path.join(directory, sub, "**", "*_results.db"), recursive=True)[0]

    def copy_kib(sub, counter):
        vals = _pmc_means(db(sub), counter)
        return max(v[0] for v in vals.values())

    f_fetch = (COPY_BYTES / 1024) / copy_kib("copy_fetch", "FETCH_SIZE")
    f_write = (COPY_BYTES / 1024) / copy_kib("copy_write", "WRITE_SIZE")
    fetch = _pmc_means(db("fetch"), "FETCH_SIZE")
    write = _pmc_means(db("write"), "WRITE_SIZE")
    path = path or os.path.join(ROOT, "profiles", "traffic.json")
    rec = json.load(open(path)) if os.path.exists(path) else {}
    for precision in ("fp64", "fp32"):
        want32 = precision != "fp64"
        for cls, knames in KERNEL_NAMES.items():
            def pick(table):
                # the class's kernel of the iteration: the one launched most
                # (the residual modes of the k-specialised product run a few
                # times per solve)
                hits = [v for nm, v in table.items()
                        if any(kn in nm for kn in knames) and _is_fp32_kernel(nm) == want32]
                return max(hits, key=lambda v: v[1])[0] if hits else None
            fk, wk = pick(fetch), pick(write)
            if fk is None or wk is None:
                continue
            rd = fk * 1024 * f_fetch
            wr = wk * 1024 * f_write
            rec[f"{cls}/{workload}/{variant}/{precision}"] = {
                "bytes_per_launch": rd + wr, "read_bytes": rd, "write_bytes": wr,
                "fetch_kib": fk, "write_kib": wk, "fetch_scale": f_fetch, "write_scale": f_write,
                "kernel_hash": kernel_hash(),
            }
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1, sort_keys=True)
    print(json.dumps(rec, indent=1, sort_keys=True))
    return 0


def cpu_baseline_groups(w, p: int, B_groups, gpu_iterations: int, budget_s: float):
    """Hybrid subalgebra: its q = k/p column groups are independent block CG
    solves of width p (Section 2), so the oracle times a bounded number of
    block iterations on sampled groups of the full-size system and the solve
    time is that per-group iteration time x q groups x the GPU's FP64
    iteration count."""
    from threadpoolctl import threadpool_info

    from oracle.bcg import solve as oracle_solve
    from oracle.stencil import stencil_csr
    from workload import coefficients_for

    A = stencil_csr(w.dim, w.N, coefficients_for(w))
    q = w.k // p
    t0 = time.perf_counter()
    oracle_solve(A, B_groups[0][1], "block", p, tol=0.0, maxit=1)
    t1 = time.perf_counter() - t0
    m = max(2, min(gpu_iterations, int(budget_s / len(B_groups) / max(t1, 1e-3))))
    total, its = 0.0, 0
    for _, Bg in B_groups:
        t0 = time.perf_counter()
        oracle_solve(A, Bg, "block", p, tol=0.0, maxit=m)
        total += time.perf_counter() - t0
        its += m
    per_it = total / its
    t_solve = per_it * q * gpu_iterations
    blas = [d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"]
    cores = max(blas + [1])
    groups = ", ".join(str(g) for g, _ in B_groups)
    return {
        "value": w.k / t_solve,
        "unit": "RHS-solves/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"{m} block iterations (p={p}) of the FP64 NumPy/SciPy oracle on each of column groups "
                   f"{groups} of the full {w.name} system ({total:.1f} s, {per_it * 1e3:.0f} ms per group "
                   f"iteration), scaled to {q} groups x the GPU's {gpu_iterations} FP64 iterations; "
                   f"sparse product single-threaded, BLAS on {cores} threads, host has {os.cpu_count()} "
                   f"logical CPUs"),
    }


def cpu_baseline(w, variant: str, p: int, gpu_iterations: int, budget_s: float, precond: str = "none"):
    """Time the oracle's iterations on the full system; scale to the solve."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle.bcg import solve as oracle_solve
    from oracle.stencil import stencil_csr
    from workload import coefficients_for, rhs_for

    A = stencil_csr(w.dim, w.N, coefficients_for(w))
    B = rhs_for(w)
    # one iteration to calibrate, then as many as fit the budget
    t0 = time.perf_counter()
    oracle_solve(A, B, variant, p, tol=0.0, maxit=1, precond=precond)
    t1 = time.perf_counter() - t0
    m = max(2, min(gpu_iterations, int(budget_s / max(t1, 1e-3))))
    t0 = time.perf_counter()
    _, info = oracle_solve(A, B, variant, p, tol=0.0, maxit=m, precond=precond)
    tm = time.perf_counter() - t0
    per_it = tm / m
    t_solve = per_it * gpu_iterations
    blas = [d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"]
    cores = max(blas + [1])
    return {
        "value": w.k / t_solve,
        "unit": "RHS-solves/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"{m} iterations of the FP64 NumPy/SciPy oracle ({variant}, p={p}"
                   f"{', Jacobi' if precond != 'none' else ''}) on the full "
                   f"{w.name} system ({tm:.1f} s, {per_it * 1e3:.0f} ms/iteration), scaled to the GPU's "
                   f"{gpu_iterations} iterations; sparse product single-threaded, BLAS on {cores} threads, "
                   f"host has {os.cpu_count()} logical CPUs"),
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="poisson3d_256_k128")
    ap.add_argument("--variant", default="hybrid")
    ap.add_argument("--p", type=int, default=16)
    ap.add_argument("--compare-steps", type=int, default=1,
                    help="timed solves of the other precision (after one profiled solve)")
    ap.add_argument("--budget-s", type=float, default=420.0,
                    help="wall-time budget (s) past which the optional variant solves are skipped")
    ap.add_argument("--no-variants", action="store_true", help="skip the other subalgebras of the workload")
    ap.add_argument("--precision", default="fp32_reliable", choices=["fp64", "fp32_refine", "fp32_reliable"],
                    help="form of the headline solve: FP32 with FP64 refinement by residual replacement "
                         "(fp32_reliable) or by restarted inner solves (fp32_refine), or plain FP64; the plain "
                         "FP64 form (FP32 with residual replacement when the headline is FP64) is timed beside it")
    ap.add_argument("--no-compare", action="store_true", help="skip the solve in the other precision")
    ap.add_argument("--tol", type=float, default=None)
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precond", default="none", choices=["none", "jacobi"],
                    help="preconditioner M of Algorithm 1 (jacobi: M = diag(A))")
    ap.add_argument("--schedule", default="bricks", choices=["bricks", "tiled", "natural"],
                    help="row order of the sparse product (3D): 4x2x2 bricks inside 16x32x2 tiles swept "
                         "through z (bricks), 32x32 x-y tiles swept through z (tiled), or natural")
    ap.add_argument("--sell", type=int, default=0, metavar="SIGMA",
                    help="sparse product on SELL-16-SIGMA storage (SIGMA 1 or a multiple of 16; 0: CSR)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 2 GiB device copy (counter calibration)")
    ap.add_argument("--study", default=None, choices=["repeat128", "gradient", "sell", "paths"],
                    help="repeat128: time to solve 128 right-hand sides in 128/k solves, k = 16..128, p = 16; "
                         "gradient: forward + adjoint backward of the 512^2 diffusion workload")
    ap.add_argument("--study-precisions", default="fp32_refine,fp64")
    ap.add_argument("--traffic-from", default=None,
                    help="write profiles/traffic.json from rocprofv3 --pmc databases in this folder")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration()
    if args.traffic_from:
        return traffic_from(args.traffic_from, args.workload, args.variant)

    if args.study:
        if args.gpus != 1:
            log("bench.py: only --gpus 1 is supported")
            return 2
        studies = {"repeat128": repeat_study, "gradient": gradient_study, "sell": sell_study, "paths": paths_study}
        return studies[args.study](args)
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        log("bench.py: only --gpus 1 is supported; the library has no multi-GPU path")
        return 2

    import torch

    import paper_1912_11930_amd as P
    from paper_1912_11930_amd import _capi
    from workload import WORKLOADS, coefficients_for, rhs_for

    t_start = time.perf_counter()
    w = WORKLOADS[args.workload]
    tol = w.tol if args.tol is None else args.tol
    dev = torch.device("cuda:0")
    kappa = coefficients_for(w)
    rp, ci, va = P.stencil(w.dim, w.N, None if kappa is None else torch.from_numpy(kappa).to(dev), device=dev)
    n, k, nnz = w.n, w.k, w.nnz
    p_eff = {"block": k, "parallel": 1}.get(args.variant, args.p or 1)
    B_host = rhs_for(w)
    B = torch.from_numpy(B_host).to(dev)
    # the oracle's sample (hybrid: the first and the last column group)
    sample_groups = None
    if not args.no_cpu_baseline and args.variant == "hybrid" and k // p_eff > 1:
        q = k // p_eff
        sample_groups = [(g, B_host[:, g * p_eff:(g + 1) * p_eff].copy()) for g in (0, q - 1)]
    del B_host
    order = None
    schedule = "natural"
    if args.schedule == "tiled" and w.dim == 3:
        order = P.stencil_schedule(w.dim, w.N, 32, device=dev)
        schedule = "tiled 32x32 (x,y) swept through z"
    elif args.schedule == "bricks" and w.dim == 3:
        order = P.stencil_brick_schedule(w.N, (16, 32, 2), (4, 2, 2), device=dev)
        schedule = "4x2x2 bricks in 16x32x2 tiles swept through z"

    def make_solver(variant: str, p: int):
        sv = P.BCG(rp, ci, va, k=k, subalgebra=variant, p=p)
        if args.precond != "none":
            sv.set_preconditioner(args.precond)
        if order is not None:
            sv.set_row_schedule(order)
        if args.sell:
            sv.set_sell(True, args.sell)
        return sv

    solver = make_solver(args.variant, p_eff)
    matrix_format = f"sell-16-{args.sell}" if args.sell else "csr"
    torch.cuda.synchronize()
    log(f"bench: set-up {time.perf_counter() - t_start:.1f} s")

    def run(precision: str, steps: int, warmup: int) -> dict:
        """Warm-up solves, the last of them with every kernel class profiled
        (the breakdown; after the first warm-up, when there is one, so
        first-launch costs stay out of it), then `steps` timed solves with
        events only around the dominant class."""
        solver.set_precision(precision)
        X = torch.empty_like(B)
        log(f"bench: {w.name} n={n} nnz={nnz} k={k} variant={args.variant} p={p_eff} precision={precision}")
        info = None
        for i in range(max(warmup, 1)):
            profiled = i == max(warmup, 1) - 1
            if profiled:
                solver.set_profiling(True)
            X.zero_()
            _, info = solver.solve(B, X, tol=tol, maxit=100000)
            log(f"{'profiled warmup' if profiled else 'warmup'} {i}: status={info['status_name']} "
                f"iterations={info['iterations']} {info['solve_ms']:.1f} ms true_rel_res={info['true_rel_res']:.2e}")
        breakdown = solver.kernel_times()
        solver.set_profiling(False)
        cand = {c: breakdown[c][1] for c in ("spmm", "update_r", "update_xp")}
        dominant = max(cand, key=cand.get)
        solver.set_profiling(True, classes=[dominant])
        its = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            X.zero_()
            _, info = solver.solve(B, X, tol=tol, maxit=100000)
            its.append(info["iterations"])
            log(f"step {i}: status={info['status_name']} iterations={info['iterations']} "
                f"{info['solve_ms']:.1f} ms")
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        launches, total_ms = solver.kernel_times()[dominant]
        solver.set_profiling(False)
        kernels = {c: {"launches": breakdown[c][0], "total_ms": round(breakdown[c][1], 3),
                       "avg_us": round(1e3 * breakdown[c][1] / max(breakdown[c][0], 1), 2)}
                   for c in _capi.KERNEL_CLASSES if breakdown[c][0]}
        for c in ("spmm", "update_r", "update_xp"):
            if c in kernels:
                bts = algorithmic_bytes(c, n, nnz, k, precision)
                kernels[c]["GBps"] = round(bts / (kernels[c]["avg_us"] * 1e-6) / 1e9, 1)
        return {"precision": precision, "elapsed": elapsed, "steps": steps, "X": X, "info": info,
                "iterations": its[-1] if its else None, "dominant": dominant, "launches": launches,
                "avg_ms": total_ms / max(launches, 1), "kernels": kernels,
                "kernels_total_ms": round(sum(v[1] for v in breakdown.values()), 3)}

    head = run(args.precision, args.steps, args.warmup)
    ms_per_step = 1e3 * head["elapsed"] / args.steps
    value = k * args.steps / head["elapsed"]
    dominant = head["dominant"]
    bytes_launch = algorithmic_bytes(dominant, n, nnz, k, args.precision)
    achieved = bytes_launch / (head["avg_ms"] * 1e-3) / 1e9
    # the counter figures were taken with CSR storage
    traffic = measured_traffic(dominant, w.name, args.variant, args.precision) if not args.sell else None
    info = head["info"]

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "RHS-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": f"{w.N}^{w.dim}", "n": n, "nnz": nnz, "k": k,
                   "variant": args.variant, "p": p_eff, "precision": args.precision, "tol": tol,
                   "rhs": w.rhs, "row_schedule": schedule, "precond": args.precond,
                   "format": matrix_format},
        "iterations": head["iterations"],
        "outer_iterations": info["outer_iterations"] if info else None,
        "true_rel_res": info["true_rel_res"] if info else None,
        "roofline": {"bound": "hbm", "kernel": dominant, "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "bytes_per_launch": bytes_launch, "avg_launch_us": 1e3 * head["avg_ms"],
                     "launches": head["launches"]},
        "kernels": head["kernels"],
        "kernels_total_ms": head["kernels_total_ms"],
        # the row passes' algorithmic bytes of one solve over the timed solve time
        "solve_GBps": solve_bytes(head["kernels"], n, nnz, k, args.precision) / (ms_per_step * 1e-3) / 1e9,
        "cpu_baseline": None,
    }
    if not args.no_compare:
        other = "fp64" if args.precision != "fp64" else "fp32_reliable"
        cmp_ = run(other, args.compare_steps, 1)
        diff = float(torch.linalg.norm(head["X"] - cmp_["X"]) / torch.linalg.norm(cmp_["X"]))
        cs = args.compare_steps
        out["compare"] = {
            "precision": other,
            "value": k * cs / cmp_["elapsed"],
            "ms_per_step": 1e3 * cmp_["elapsed"] / cs,
            "steps": cs,
            "iterations": cmp_["iterations"],
            "true_rel_res": cmp_["info"]["true_rel_res"],
            "speedup_of_headline": (k * args.steps / head["elapsed"]) / (k * cs / cmp_["elapsed"]),
            "rel_diff_solutions": diff,
            "kernels": cmp_["kernels"],
        }
        del cmp_
    del head
    if not args.no_cpu_baseline:
        log("cpu_baseline: timing the oracle ...")
        if sample_groups is not None:
            out["cpu_baseline"] = cpu_baseline_groups(w, p_eff, sample_groups, head_fp64_iterations(out),
                                                      args.cpu_budget)
        else:
            out["cpu_baseline"] = cpu_baseline(w, args.variant, p_eff, head_fp64_iterations(out), args.cpu_budget,
                                               args.precond)
        sample_groups = None
    if not args.no_variants and w.variants:
        solver.close()
        torch.cuda.empty_cache()
        out["variants"] = variant_solves(args, w, tol, B, make_solver, t_start, out)
    log(f"bench: total {time.perf_counter() - t_start:.1f} s")
    print(json.dumps(out), flush=True)
    return 0


def variant_solves(args, w, tol, B, make_solver, t_start: float, out: dict) -> list:
    """One timed solve in each precision of every other subalgebra the
    workload lists (after one untimed solve that also warms its kernels),
    while the wall time stays inside the budget; a variant whose estimated
    cost would overrun it is listed as skipped."""
    import torch

    res = []
    head_p = {"block": w.k, "parallel": 1}.get(args.variant, args.p or 1)
    per_rhs_s = out["ms_per_step"] / 1e3
    for variant, p in w.variants:
        if variant == args.variant and p == head_p:
            continue
        # a cost guess from the headline: the other forms iterate up to ~2x longer
        need = 4 * 2.5 * per_rhs_s
        if time.perf_counter() - t_start + need > args.budget_s:
            res.append({"variant": variant, "p": p, "skipped": "time budget"})
            continue
        sv = make_solver(variant, p)
        X = torch.empty_like(B)
        rec = {"variant": variant, "p": p}
        for precision in (args.precision, "fp64" if args.precision != "fp64" else "fp32_reliable"):
            sv.set_precision(precision)
            X.zero_()
            sv.solve(B, X, tol=tol, maxit=100000)
            X.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = sv.solve(B, X, tol=tol, maxit=100000)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            log(f"variant {variant} p={p} {precision}: status={info['status_name']} "
                f"iterations={info['iterations']} {1e3 * dt:.1f} ms")
            rec[precision] = {"value": w.k / dt, "ms_per_step": 1e3 * dt, "iterations": info["iterations"],
                              "outer_iterations": info["outer_iterations"], "status": info["status_name"],
                              "true_rel_res": info["true_rel_res"]}
        res.append(rec)
        sv.close()
        del X
        torch.cuda.empty_cache()
    return res


def repeat_study(args) -> int:
    """Time to solve 128 right-hand sides of the 128^3 Poisson system in
    r = 128/k solves of k columns each, k = 16, 32, 64, 128 with p = 16
    (block at k = 16, hybrid above): the paper's third experiment (Section 5),
    on this GPU. One JSON line per (precision, k): the wall time of the r
    solves after one warm-up solve, iterations and the worst true relative
    residual of the r solves, and from one more solve with per-class events
    the sparse product's and the updates' average time and algorithmic GB/s."""
    import torch

    import paper_1912_11930_amd as P
    from workload import WORKLOADS, rhs

    w = WORKLOADS["poisson3d_128_k16"]
    total = 128
    dev = torch.device("cuda:0")
    rp, ci, va = P.stencil(w.dim, w.N, None, device=dev)
    sched = P.stencil_schedule(w.dim, w.N, 32, device=dev)
    B_all = torch.from_numpy(rhs(w.n, total, "uniform")).to(dev)
    n, nnz = w.n, w.nnz
    for precision in args.study_precisions.split(","):
        for k in (16, 32, 64, 128):
            variant, p = ("block", 0) if k == 16 else ("hybrid", 16)
            solver = P.BCG(rp, ci, va, k=k, subalgebra=variant, p=p)
            solver.set_row_schedule(sched)
            solver.set_precision(precision)
            batches = [B_all[:, j * k:(j + 1) * k].contiguous() for j in range(total // k)]
            X = torch.zeros_like(batches[0])
            _, info = solver.solve(batches[0], X, tol=w.tol, maxit=100000)  # warm-up
            X.zero_()
            solver.set_profiling(True)
            solver.solve(batches[0], X, tol=w.tol, maxit=100000)
            times = solver.kernel_times()
            solver.set_profiling(False)
            its, worst = [], 0.0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for Bj in batches:
                X.zero_()
                _, info = solver.solve(Bj, X, tol=w.tol, maxit=100000)
                if info["status_name"] != "OK":
                    log(f"study: k={k} {precision}: status {info['status_name']}")
                    return 1
                its.append(info["iterations"])
                worst = max(worst, info["true_rel_res"])
            torch.cuda.synchronize()
            elapsed = time.perf_counter() - t0
            kernels = {}
            for c in ("spmm", "update_r", "update_xp"):
                launches, ms = times[c]
                if launches:
                    us = 1e3 * ms / launches
                    kernels[c] = {"avg_us": round(us, 2),
                                  "GBps": round(algorithmic_bytes(c, n, nnz, k, precision) / (us * 1e-6) / 1e9, 1)}
            line = {"study": "repeat128", "workload": f"{w.name.rsplit('_k', 1)[0]}_rhs128", "total_rhs": total,
                    "k": k, "p": 16, "variant": variant, "solves": len(batches), "precision": precision,
                    "seconds": round(elapsed, 4), "rhs_per_s": round(total / elapsed, 2),
                    "iterations": its, "max_true_rel_res": worst, "kernels": kernels}
            print(json.dumps(line), flush=True)
            del solver, X, batches
            torch.cuda.empty_cache()
    return 0


def gradient_study(args) -> int:
    """Forward solve plus adjoint backward of the 512^2 diffusion workload
    (k = 32, block): L = sum(W * X) with X = A(kappa)^{-1} B, gradients with
    respect to B and to the cell coefficients kappa through the library's
    autograd functions (assembly, solve, adjoint solve, sampled outer
    product, coefficient VJP). One JSON line per precision: wall times of
    the forward and the backward after one warm-up pass, medians of
    `steps` passes."""
    import torch

    import paper_1912_11930_amd as P
    from workload import WORKLOADS, cell_coefficients, loss_weights, rhs

    w = WORKLOADS["diffusion2d_512_k32"]
    dim, N, k = w.dim, w.N, w.k
    dev = torch.device("cuda:0")
    kappa0 = torch.tensor(cell_coefficients(dim, N, w.sigma), dtype=torch.float64, device=dev)
    B = torch.from_numpy(rhs(w.n, k, w.rhs)).to(dev)
    W = torch.from_numpy(loss_weights(w.n, k)).to(dev)
    rp, ci, v0 = P.stencil(dim, N, kappa0)
    tol = w.tol if args.tol is None else args.tol
    for precision in args.study_precisions.split(","):
        solver = P.BCG(rp, ci, v0, k=k, subalgebra="block")
        solver.set_precision(precision)
        fw, bw, its = [], [], None
        for rep_i in range(args.warmup + max(args.steps, 1)):
            kt = kappa0.clone().requires_grad_(True)
            Bt = B.clone().requires_grad_(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            vals = P.StencilValues.apply(kt, dim, N)
            X = P.BCGSolve.apply(vals, Bt, solver, tol, 100000)
            loss = (W * X).sum()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            its_fwd = solver.info()["iterations"]
            loss.backward()
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            its = (its_fwd, solver.info()["iterations"])
            if rep_i >= args.warmup:
                fw.append(t1 - t0)
                bw.append(t2 - t1)
        fw.sort()
        bw.sort()
        f_ms, b_ms = 1e3 * fw[len(fw) // 2], 1e3 * bw[len(bw) // 2]
        line = {"study": "gradient", "workload": w.name, "variant": "block", "k": k, "precision": precision,
                "tol": tol, "forward_ms": round(f_ms, 3), "backward_ms": round(b_ms, 3),
                "total_ms": round(f_ms + b_ms, 3), "iterations_forward": its[0], "iterations_adjoint": its[1],
                "grad_kappa_norm": float(torch.linalg.norm(kt.grad)), "grad_B_norm": float(torch.linalg.norm(Bt.grad)),
                "passes": len(fw)}
        print(json.dumps(line), flush=True)
        del solver
        torch.cuda.empty_cache()
    return 0


def sell_study(args) -> int:
    """CSR against SELL-16-sigma storage of the sparse product (sigma 1 and
    256), k = 16 (block) and k = 64 (hybrid, p = 16; the paper suggests the
    format for the product's cache behaviour at larger k), solves to 1e-8 in
    each precision, on two systems:
    the 128^3 Poisson system in the tiled row order, and an irregular one,
    the 2D 1024^2 diffusion system (sigma 0.5) plus symmetric couplings of
    -0.05 between random far rows (3 pairs drawn per row) with the diagonal
    raised by their row sums (rows of 4 to 27 entries, 11 on average). One JSON line per
    system, format and precision: median wall time of `steps` solves after
    `warmup`, and the sparse product's average launch time from one more
    solve with events around that class only."""
    import numpy as np
    import scipy.sparse as sp
    import torch

    import paper_1912_11930_amd as P
    from workload import cell_coefficients, long_range_pairs, rhs

    dev = torch.device("cuda:0")
    systems = [("poisson3d_128", P.stencil(3, 128, None, device=dev), P.stencil_schedule(3, 128, 32, device=dev))]
    N = 1024
    rp, ci, va = P.stencil(2, N, torch.from_numpy(cell_coefficients(2, N, 0.5)).to(dev), device=dev)
    n = N * N
    A = sp.csr_matrix((va.cpu().numpy(), ci.cpu().numpy(), rp.cpu().numpy()), shape=(n, n))
    i, j = long_range_pairs(n, 3)
    C = sp.coo_matrix((np.full(i.size, -0.05), (i, j)), shape=(n, n)).tocsr()
    C = C + C.T
    A = (A + C + sp.diags(np.asarray(abs(C).sum(axis=1)).ravel())).tocsr()
    A.sort_indices()
    systems.append(("longrange2d_1024", tuple(torch.from_numpy(x).to(dev) for x in
                                              (A.indptr.astype(np.int32), A.indices.astype(np.int32),
                                               A.data.astype(np.float64))), None))
    for (name, (rp, ci, va), order), (k, variant, p) in itertools.product(systems, [(16, "block", 0),
                                                                                    (64, "hybrid", 16)]):
        n = rp.numel() - 1
        lens = torch.diff(rp).cpu().numpy()
        B = torch.from_numpy(rhs(n, k, "uniform")).to(dev)
        for sigma in (0, 1, 256):
            solver = P.BCG(rp, ci, va, k=k, subalgebra=variant, p=p)
            if order is not None:
                solver.set_row_schedule(order)
            if sigma:
                solver.set_sell(True, sigma)
            for precision in args.study_precisions.split(","):
                solver.set_precision(precision)
                X = torch.zeros_like(B)
                times = []
                for rep_i in range(args.warmup + max(args.steps, 1)):
                    X.zero_()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    _, info = solver.solve(B, X, tol=1e-8, maxit=100000)
                    torch.cuda.synchronize()
                    if rep_i >= args.warmup:
                        times.append(time.perf_counter() - t0)
                solver.set_profiling(True, classes=["spmm"])
                X.zero_()
                solver.solve(B, X, tol=1e-8, maxit=100000)
                launches, total_ms = solver.kernel_times()["spmm"]
                solver.set_profiling(False)
                times.sort()
                ms = 1e3 * times[len(times) // 2]
                line = {"study": "sell", "system": name, "n": n, "nnz": int(lens.sum()),
                        "row_len_min_max": [int(lens.min()), int(lens.max())], "k": k, "variant": variant,
                        "p": p or k,
                        "format": f"sell-16-{sigma}" if sigma else "csr", "precision": precision,
                        "status": info["status_name"], "iterations": info["iterations"],
                        "true_rel_res": info["true_rel_res"], "ms_per_solve": round(ms, 3),
                        "rhs_solves_per_s": round(k / (ms / 1e3), 2),
                        "spmm_avg_us": round(1e3 * total_ms / max(launches, 1), 2), "solves": len(times)}
                print(json.dumps(line), flush=True)
            del solver
            torch.cuda.empty_cache()
    return 0


def paths_study(args) -> int:
    """Matrix-core against vector kernels for the row passes, by subalgebra
    width (parallel, hybrid 4, 8 and 16), on the 128^3 Poisson system with
    k = 16 and the 256^3 one with k = 128, both in the brick row order.
    Paths: the library's choice; the matrix cores for every row pass
    (BCG_UPDATE_VEC32 = BCG_UPDATE_VEC64 = 0, where the choice differs); the
    k-specialised vector kernels (BCG_NO_MFMA). Each line: per-class average
    launch times and the summed kernel time per iteration of a fixed number of
    iterations (`--steps`, at least 10) after one untimed solve, FP64 and the
    FP32 inner iteration (one outer step of exactly that many iterations)."""
    import torch

    import paper_1912_11930_amd as P
    from workload import rhs

    dev = torch.device("cuda:0")
    m = max(args.steps, 10)
    envs = ("BCG_NO_MFMA", "BCG_UPDATE_VEC32", "BCG_UPDATE_VEC64")
    for N, k in ((128, 16), (256, 128)):
        n = N ** 3
        rp, ci, va = P.stencil(3, N, None, device=dev)
        nnz = ci.numel()
        order = P.stencil_brick_schedule(N, (16, 32, 2), (4, 2, 2), device=dev)
        B = torch.from_numpy(rhs(n, k, "uniform")).to(dev)
        X = torch.zeros_like(B)
        for (variant, p), precision in itertools.product((("parallel", 1), ("hybrid", 4), ("hybrid", 8),
                                                          ("hybrid", 16)), ("fp32_refine", "fp64")):
            paths = [("default", {}), ("vector", {"BCG_NO_MFMA": "1"})]
            wide = precision == "fp64" or p <= 8
            if k == 128 and wide:  # the library puts some row passes on vector kernels here
                paths.insert(1, ("matrix-core", {"BCG_UPDATE_VEC32": "0", "BCG_UPDATE_VEC64": "0"}))
            for path, env in paths:
                for e in envs:
                    os.environ.pop(e, None)
                os.environ.update(env)
                solver = P.BCG(rp, ci, va, k=k, subalgebra=variant, p=p)
                solver.set_row_schedule(order)
                if precision == "fp64":
                    solver.set_precision("fp64")
                    tol = 0.0
                else:
                    solver.set_precision("fp32_refine", 0.0, m, 1)
                    tol = 1e-8
                X.zero_()
                solver.solve(B, X, tol=tol, maxit=m)
                solver.set_profiling(True)
                X.zero_()
                _, info = solver.solve(B, X, tol=tol, maxit=m)
                times = solver.kernel_times()
                solver.set_profiling(False)
                solver.close()
                del solver
                its = max(info["iterations"], 1)
                line = {"study": "paths", "system": f"poisson3d_{N}", "n": n, "k": k, "variant": variant, "p": p,
                        "precision": "fp64" if precision == "fp64" else "fp32 inner", "path": path,
                        "iterations": info["iterations"]}
                for c in ("spmm", "update_r", "update_xp", "reduce", "small"):
                    launches, total_ms = times[c]
                    if launches:
                        us = 1e3 * total_ms / launches
                        line[f"{c}_us"] = round(us, 1)
                        if c in ("spmm", "update_r", "update_xp"):
                            line[f"{c}_GBps"] = round(
                                algorithmic_bytes(c, n, nnz, k, precision) / (us * 1e-6) / 1e9, 1)
                row_ms = sum(times[c][1] for c in ("spmm", "update_r", "update_xp", "reduce", "small"))
                line["ms_per_iteration"] = round(row_ms / its, 3)
                print(json.dumps(line), flush=True)
            for e in envs:
                os.environ.pop(e, None)
        del B, X
        torch.cuda.empty_cache()
    return 0


def head_fp64_iterations(out: dict) -> int:
    """FP64 iteration count of the benchmark solve (the oracle runs FP64)."""
    if out["config"]["precision"] == "fp64":
        return out["iterations"] or 1
    cmp_ = out.get("compare")
    if cmp_ and cmp_["precision"] == "fp64":
        return cmp_["iterations"] or 1
    return out["iterations"] or 1


if __name__ == "__main__":
    sys.exit(main())
