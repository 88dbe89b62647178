"""Writes diffusion2d_512_k32_gradient.npz: the FP64 oracle's adjoint gradient
of L = sum(W * X), X = A(kappa)^{-1} B, for the 512^2 diffusion workload
(k = 32 standard-normal right-hand sides, log-normal coefficients sigma = 0.5,
block subalgebra, forward and adjoint solves to 1e-12), reduced to what a GPU
test compares at full size: dL/dB = A^{-1} W on 1024 sampled rows, dL/dkappa
on 4096 sampled cells and its largest magnitude over all cells (samples drawn
once with numpy's PCG64, seed 12).

Only the oracle and the workload's seeded draws are used. Usage (repository
root; about 15 minutes on 8 cores):

    python tests/golden/make_diffusion2d_512_gradient_fixture.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.bcg import solve  # noqa: E402
from oracle.grad import kappa_vjp, sampled_outer  # noqa: E402
from oracle.stencil import stencil_csr  # noqa: E402
from workload import WORKLOADS, cell_coefficients, loss_weights, rhs  # noqa: E402

TOL = 1e-12
SAMPLE_SEED = 12


def main() -> None:
    w = WORKLOADS["diffusion2d_512_k32"]
    kappa = cell_coefficients(w.dim, w.N, w.sigma)
    A = stencil_csr(w.dim, w.N, kappa)
    B = rhs(w.n, w.k, w.rhs)
    W = loss_weights(w.n, w.k)
    t0 = time.perf_counter()
    X, ix = solve(A, B, "block", 0, tol=TOL, maxit=100000)
    Y, iy = solve(A, W, "block", 0, tol=TOL, maxit=100000)
    dk = kappa_vjp(w.dim, w.N, kappa, A, sampled_outer(A, Y, X, -1.0))
    rng = np.random.default_rng(SAMPLE_SEED)
    rows = np.sort(rng.choice(w.n, 1024, replace=False))
    cells = np.sort(rng.choice(w.n, 4096, replace=False))
    out = {"tol": np.array(TOL), "rows": rows.astype(np.int64), "cells": cells.astype(np.int64),
           "status_forward": np.array(ix["status"]), "status_adjoint": np.array(iy["status"]),
           "iterations_forward": np.array(ix["iterations"]), "iterations_adjoint": np.array(iy["iterations"]),
           "dB_rows": Y[rows], "dkappa_cells": dk[cells], "dkappa_absmax": np.array(np.abs(dk).max())}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "diffusion2d_512_k32_gradient.npz")
    np.savez_compressed(path, **out)
    print(f"iterations {ix['iterations']} / {iy['iterations']} ({time.perf_counter() - t0:.0f} s)\n{path}")


if __name__ == "__main__":
    main()
