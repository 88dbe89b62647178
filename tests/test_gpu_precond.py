"""Jacobi-preconditioned block CG (M = diag(A)) on the GPU, through the C ABI.

The library runs block CG on the symmetrically scaled system D^{-1/2} A
D^{-1/2}; the oracle runs Algorithm 1 with Z = M^{-1} R directly. The two
produce the same iterates up to rounding: fixed-iteration iterates agree to
1e-10 relative (Frobenius), converged solutions to 1e-8, the stop-rule ratios
(M^{-1}-norms) to 1e-8 relative.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle.bcg import solve as oracle_solve
from oracle.grad import sampled_outer as oracle_sampled_outer
from oracle.stencil import stencil_csr
from tests.gpu_helpers import csr_to_dev, dev, host, log, rel
from workload import cell_coefficients, loss_weights, rhs

pytestmark = pytest.mark.gpu


def _P():
    import paper_1912_11930_amd as P
    return P


def _problem(dim, N, k, sigma=1.0, seed=11):
    A = stencil_csr(dim, N, cell_coefficients(dim, N, sigma))
    return A, rhs(A.shape[0], k, "normal", seed)


def _jacobi_solver(A, k, variant, p):
    P = _P()
    s = P.BCG(*csr_to_dev(A), k=k, subalgebra=variant, p=p)
    s.set_preconditioner("jacobi")
    return s


CASES = [(16, "block", 0), (16, "hybrid", 4), (16, "global", 2), (16, "parallel", 1), (8, "hybrid", 2),
         (32, "block", 0), (12, "hybrid", 3)]


@pytest.mark.parametrize("path", ["default", "generic"])
@pytest.mark.parametrize("k,variant,p", CASES)
def test_jacobi_fixed_iterations(monkeypatch, path, k, variant, p):
    if path == "generic":
        monkeypatch.setenv("BCG_GENERIC_ONLY", "1")
    log(f"jacobi fixed k={k} {variant} p={p} {path}")
    A, B = _problem(2, 23, k)
    m = 8
    Xo, io = oracle_solve(A, B, variant, p, tol=0.0, maxit=m, precond="jacobi")
    s = _jacobi_solver(A, k, variant, p)
    Xg, ig = s.solve(dev(B), tol=0.0, maxit=m)
    assert ig["iterations"] == io["iterations"] == m
    assert ig["status"] == io["status"] == oracle.NOT_CONVERGED
    assert rel(host(Xg), Xo) <= 1e-10
    np.testing.assert_allclose(ig["ratios"], io["ratios"], rtol=1e-8, atol=0)


@pytest.mark.parametrize("variant,p", [("block", 0), ("hybrid", 4), ("parallel", 1), ("global", 4)])
def test_jacobi_converged_3d(variant, p):
    log(f"jacobi converged {variant} p={p}")
    A, B = _problem(3, 16, 16, sigma=1.0)
    tol = 1e-8
    Xo, io = oracle_solve(A, B, variant, p, tol=tol, maxit=5000, precond="jacobi")
    s = _jacobi_solver(A, 16, variant, p)
    Xg, ig = s.solve(dev(B), tol=tol)
    assert io["status"] == ig["status"] == oracle.OK
    assert abs(ig["iterations"] - io["iterations"]) <= 1
    assert rel(host(Xg), Xo) <= 1e-8
    # info.true_rel_res: Euclidean ||B - A X||_j / ||B - A X0||_j of the returned X
    R = B - A @ host(Xg)
    true = np.max(np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0))
    assert abs(ig["true_rel_res"] - true) <= 1e-6 * true
    assert max(ig["ratios"]) <= tol


def test_jacobi_refine_reaches_fp64_accuracy():
    log("jacobi refine")
    P = _P()
    A, B = _problem(3, 20, 16, sigma=1.0)
    tol = 1e-10
    s = _jacobi_solver(A, 16, "hybrid", 4)
    s.set_precision("fp32_refine", inner_tol=1e-4, inner_maxit=2000)
    X, info = s.solve(dev(B), tol=tol)
    assert info["status"] == oracle.OK, info
    assert info["fp64_fallback"] == 0
    s64 = _jacobi_solver(A, 16, "hybrid", 4)
    X64, i64 = s64.solve(dev(B), tol=tol)
    assert i64["status"] == oracle.OK
    assert rel(host(X), host(X64)) <= 1e-7
    Xo, _ = oracle_solve(A, B, "hybrid", 4, tol=tol, maxit=5000, precond="jacobi")
    assert rel(host(X), Xo) <= 1e-7


def test_jacobi_update_values_and_warm_start():
    log("jacobi update values / warm start")
    P = _P()
    A1, B = _problem(2, 21, 8, sigma=0.5, seed=12)
    A2 = stencil_csr(2, 21, cell_coefficients(2, 21, 1.0, seed=5))
    s = _jacobi_solver(A1, 8, "block", 0)
    s.update_values(dev(A2.data.astype(np.float64)))
    X0 = rhs(A2.shape[0], 8, "uniform", 13)
    Xo, io = oracle_solve(A2, B, "block", 0, tol=0.0, maxit=6, X0=X0, precond="jacobi")
    Xg, ig = s.solve(dev(B), X=dev(X0), tol=0.0, maxit=6)
    assert ig["iterations"] == io["iterations"] == 6
    assert rel(host(Xg), Xo) <= 1e-10


def test_jacobi_rejected_and_switched_off():
    log("jacobi input checks")
    P = _P()
    A, B = _problem(2, 9, 4)
    An = A.tolil()
    An[5, 5] = -1.0
    An = An.tocsr()
    s = P.BCG(*csr_to_dev(An), k=4, subalgebra="block")
    with pytest.raises(P.BCGError):
        s.set_preconditioner("jacobi")
    # still unpreconditioned: one iteration as the M = I oracle
    Xo, _ = oracle_solve(An, B, "block", 0, tol=0.0, maxit=1)
    Xg, _ = s.solve(dev(B), tol=0.0, maxit=1)
    assert rel(host(Xg), Xo) <= 1e-10
    # on, then off again
    s2 = _jacobi_solver(A, 4, "block", 0)
    s2.set_preconditioner("none")
    Xo2, _ = oracle_solve(A, B, "block", 0, tol=0.0, maxit=5)
    Xg2, _ = s2.solve(dev(B), tol=0.0, maxit=5)
    assert rel(host(Xg2), Xo2) <= 1e-10


def test_jacobi_gradient_matches_dense():
    # The preconditioner changes the iterates, not the solution: the adjoint
    # gradient of L = sum(W * X) matches the dense FP64 one.
    log("jacobi gradient")
    P = _P()
    A, B = _problem(2, 10, 3, sigma=0.5)
    W = loss_weights(A.shape[0], 3)
    s = _jacobi_solver(A, 3, "block", 0)
    vals = dev(A.data.astype(np.float64)).requires_grad_(True)
    Bt = dev(B).requires_grad_(True)
    X = P.BCGSolve.apply(vals, Bt, s, 1e-13, 10000)
    (dev(W) * X).sum().backward()
    Ad = A.toarray()
    Yd = np.linalg.solve(Ad, W)
    Xd = np.linalg.solve(Ad, B)
    np.testing.assert_allclose(host(Bt.grad), Yd, rtol=0, atol=1e-9 * np.abs(Yd).max())
    dv = oracle_sampled_outer(A, Yd, Xd, -1.0)
    np.testing.assert_allclose(host(vals.grad), dv, rtol=0, atol=1e-9 * np.abs(dv).max())
