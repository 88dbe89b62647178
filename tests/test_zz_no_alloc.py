"""bcg_solve_noalloc (workspace in the library's fixed per-GPU array, no
allocation) against bcg_create + bcg_solve through the C ABI: same status,
iteration count and solution, on two calls in a row, the second with a
smaller system; oversize and malformed inputs are rejected before any solve."""
import numpy as np
import pytest
import torch

import oracle
from oracle.stencil import stencil_csr
from tests.gpu_helpers import csr_to_dev, dev, host, log, rel
from workload import cell_coefficients, rhs

pytestmark = pytest.mark.gpu


def _P():
    import paper_1912_11930_amd as P
    return P


# (grid N of a 2D diffusion system, k, subalgebra, p, tol, maxit): the first
# takes the matrix-core kernels and runs to convergence, the second (smaller)
# the k-specialised kernels for a fixed number of iterations, the third
# (smaller still) the generic kernels
CALLS = [(61, 32, "hybrid", 8, 1e-8, 5000), (23, 8, "block", 0, 0.0, 7), (9, 3, "global", 3, 1e-10, 500)]


def test_noalloc_matches_handle_solve_on_consecutive_calls():
    P = _P()
    for i, (N, k, variant, p, tol, maxit) in enumerate(CALLS):
        log(f"no-alloc call {i}: N={N} k={k} {variant} p={p} tol={tol}")
        A = stencil_csr(2, N, cell_coefficients(2, N, 0.6))
        B = dev(rhs(A.shape[0], k, "normal", seed=90 + i))
        rp, ci, va = csr_to_dev(A)
        X1 = torch.zeros_like(B)
        i1 = P.solve_noalloc(rp, ci, va, B, X1, variant, p, tol=tol, maxit=maxit)
        s = P.BCG(rp, ci, va, k=k, subalgebra=variant, p=p)
        X2, i2 = s.solve(B, tol=tol, maxit=maxit)
        log(f"  status {i1['status_name']} / {i2['status_name']}, iterations {i1['iterations']} / "
            f"{i2['iterations']}, true_rel_res {i1['true_rel_res']:.3e} / {i2['true_rel_res']:.3e}")
        assert i1["status"] == i2["status"]
        assert i1["status"] == (oracle.OK if tol > 0 else oracle.NOT_CONVERGED)
        assert i1["iterations"] == i2["iterations"]
        assert rel(host(X1), host(X2)) <= 1e-12
        assert abs(i1["true_rel_res"] - i2["true_rel_res"]) <= 1e-6 * i2["true_rel_res"]


def test_noalloc_rejects_oversize_and_malformed():
    P = _P()
    # 3 n k doubles beyond the 128 MiB array: rejected before any device work
    N = 100
    A = stencil_csr(3, N)
    rp, ci, va = csr_to_dev(A)
    B = torch.ones(A.shape[0], 8, dtype=torch.float64, device="cuda")
    X = torch.zeros_like(B)
    with pytest.raises(P.BCGError) as e:
        P.solve_noalloc(rp, ci, va, B, X, "block")
    assert e.value.status == oracle.EINVAL and "workspace" in str(e.value)
    assert torch.count_nonzero(X) == 0
    # a column index out of range: rejected by the device check, X untouched
    A = stencil_csr(2, 9)
    rp, ci, va = csr_to_dev(A)
    bad = ci.clone()
    bad[5] = A.shape[0]
    B = dev(rhs(A.shape[0], 4, "uniform"))
    X = torch.zeros_like(B)
    with pytest.raises(P.BCGError) as e:
        P.solve_noalloc(rp, bad, va, B, X, "block")
    assert e.value.status == oracle.EINVAL
    assert torch.count_nonzero(X) == 0
    # and the array still serves a well-formed solve afterwards
    info = P.solve_noalloc(rp, ci, va, B, X, "block", tol=1e-10, maxit=500)
    assert info["status"] == oracle.OK and info["true_rel_res"] <= 1e-9
