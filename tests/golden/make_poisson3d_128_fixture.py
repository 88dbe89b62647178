"""Writes poisson3d_128_k16_fp64.npz: the FP64 oracle's converged solves of the
128^3 Poisson workload (k = 16 uniform right-hand sides, tol 1e-8) for the
four subalgebras the workload lists, reduced to what a GPU test compares at
full size: status, iteration count, the final column ratios of the stop rule,
and the solution on 512 sampled rows (drawn once with numpy's PCG64, seed 11).

Only the oracle and the workload's seeded draws are used. Usage (repository
root; about 70 minutes on 8 cores, most of it the hybrid solve):

    python tests/golden/make_poisson3d_128_fixture.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.bcg import solve  # noqa: E402
from oracle.stencil import stencil_csr  # noqa: E402
from workload import WORKLOADS, rhs_for  # noqa: E402

VARIANTS = (("block", 16), ("global", 1), ("parallel", 1), ("hybrid", 4))
SAMPLE_SEED = 11
SAMPLE_ROWS = 512


def main() -> None:
    w = WORKLOADS["poisson3d_128_k16"]
    A = stencil_csr(w.dim, w.N)
    B = rhs_for(w)
    rows = np.sort(np.random.default_rng(SAMPLE_SEED).choice(w.n, SAMPLE_ROWS, replace=False))
    out = {"rows": rows.astype(np.int64), "tol": np.array(w.tol)}
    for variant, p in VARIANTS:
        t0 = time.perf_counter()
        X, info = solve(A, B, variant, p, tol=w.tol, maxit=5000)
        key = f"{variant}{p}"
        out[f"{key}_status"] = np.array(info["status"])
        out[f"{key}_iterations"] = np.array(info["iterations"])
        out[f"{key}_ratios"] = np.asarray(info["ratios"], dtype=np.float64)
        out[f"{key}_x"] = X[rows]
        print(f"{key}: status {info['status']} iterations {info['iterations']} "
              f"max ratio {np.max(info['ratios']):.3e} ({time.perf_counter() - t0:.0f} s)", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "poisson3d_128_k16_fp64.npz")
    np.savez_compressed(path, **out)
    print(path)


if __name__ == "__main__":
    main()
