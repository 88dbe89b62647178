"""Pins of the oracle's Jacobi-preconditioned block CG (M = diag(A); CPU only).

Each pin comes from outside the oracle: the trace-A-norm Galerkin
characterisation over the preconditioned block Krylov space (every
subalgebra), SciPy's preconditioned CG (k = 1 and the parallel subalgebra), a
dense direct solve, the identity with unpreconditioned block CG when the
diagonal is constant, and the identity with unpreconditioned block CG on the
symmetrically scaled system D^{-1/2} A D^{-1/2} (which also fixes the stop
rule's M^{-1}-norm reading).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from oracle.bcg import solve
from oracle.stencil import stencil_csr
from tests.galerkin import galerkin_iterate
from workload import cell_coefficients, rhs

VARS = [("block", 0), ("global", 1), ("global", 2), ("parallel", 1), ("hybrid", 2), ("hybrid", 4)]


def _problem(dim=2, N=8, k=4, sigma=1.0, seed=1):
    A = stencil_csr(dim, N, cell_coefficients(dim, N, sigma))
    B = rhs(A.shape[0], k, "normal", seed)
    return A, B


@pytest.mark.parametrize("variant,p", VARS)
def test_jacobi_matches_galerkin_characterisation(variant, p):
    A, B = _problem(N=7, k=4, sigma=1.0)
    minv = 1.0 / A.diagonal()
    assert np.ptp(minv) > 0.1 * np.max(minv)  # the diagonal really varies
    X0 = np.zeros_like(B)
    pp = {"block": 4, "parallel": 1}.get(variant, p)
    for m in (1, 2, 4):
        X, info = solve(A, B, variant, p, tol=0.0, maxit=m, precond="jacobi")
        assert info["iterations"] == m
        Xg = galerkin_iterate(A, B, X0, variant, pp, m, minv=minv)
        assert np.linalg.norm(X - Xg) <= 1e-9 * np.linalg.norm(Xg)


@pytest.mark.parametrize("variant,p", [("block", 0), ("global", 0), ("parallel", 0), ("hybrid", 1)])
def test_jacobi_k1_is_scipy_pcg(variant, p):
    A, B = _problem(N=9, k=1, sigma=1.0)
    b = B[:, 0]
    M = sp.diags(1.0 / A.diagonal())
    its = []
    spla.cg(A, b, x0=np.zeros_like(b), rtol=0.0, atol=0.0, maxiter=12, M=M,
            callback=lambda x: its.append(x.copy()))
    for m in (1, 3, 12):
        X, info = solve(A, B, variant, p, tol=0.0, maxit=m, precond="jacobi")
        assert info["iterations"] == m
        np.testing.assert_allclose(X[:, 0], its[m - 1], rtol=0, atol=1e-10 * np.linalg.norm(its[m - 1]))


def test_jacobi_parallel_is_k_independent_pcg_runs():
    A, B = _problem(N=9, k=5, sigma=0.5)
    M = sp.diags(1.0 / A.diagonal())
    m = 7
    X, _ = solve(A, B, "parallel", 1, tol=0.0, maxit=m, precond="jacobi")
    for j in range(B.shape[1]):
        xj, _ = spla.cg(A, B[:, j], x0=np.zeros(A.shape[0]), rtol=0.0, atol=0.0, maxiter=m, M=M)
        np.testing.assert_allclose(X[:, j], xj, rtol=0, atol=1e-10 * np.linalg.norm(xj))


@pytest.mark.parametrize("variant,p", VARS)
def test_jacobi_converged_matches_dense_solve(variant, p):
    A, B = _problem(N=10, k=4, sigma=1.0)
    X, info = solve(A, B, variant, p, tol=1e-10, maxit=2000, precond="jacobi")
    assert info["status"] == oracle.OK
    Xd = np.linalg.solve(A.toarray(), B)
    assert np.linalg.norm(X - Xd) <= np.linalg.cond(A.toarray()) * 1e-9 * np.linalg.norm(Xd)


@pytest.mark.parametrize("variant,p", [("block", 0), ("hybrid", 2), ("global", 2)])
def test_jacobi_with_constant_diagonal_is_unpreconditioned(variant, p):
    # Poisson: diag(A) = 2 dim everywhere, so M^{-1} scales Z and P by one
    # constant that lambda and beta absorb; the iterates and the relative
    # stop-rule ratios are those of M = I.
    A = stencil_csr(2, 9)
    B = rhs(A.shape[0], 4, "normal", 3)
    for m in (1, 5):
        Xj, ij = solve(A, B, variant, p, tol=0.0, maxit=m, precond="jacobi")
        Xn, inn = solve(A, B, variant, p, tol=0.0, maxit=m)
        np.testing.assert_allclose(Xj, Xn, rtol=0, atol=1e-11 * np.linalg.norm(Xn))
        np.testing.assert_allclose(ij["ratios"], inn["ratios"], rtol=1e-10)
    _, cj = solve(A, B, variant, p, tol=1e-8, precond="jacobi")
    _, cn = solve(A, B, variant, p, tol=1e-8)
    assert cj["iterations"] == cn["iterations"]


@pytest.mark.parametrize("variant,p", VARS)
def test_jacobi_is_block_cg_on_scaled_system(variant, p):
    # With S = D^{-1/2}: PCG on (A, B) iterates X = S Xs where Xs is plain
    # block CG on (S A S, S B); the M^{-1}-norm of R is the 2-norm of S R.
    A, B = _problem(N=8, k=4, sigma=1.0)
    s = 1.0 / np.sqrt(A.diagonal())
    S = sp.diags(s)
    As = (S @ A @ S).tocsr()
    Bs = s[:, None] * B
    for m in (3, 8):
        X, info = solve(A, B, variant, p, tol=0.0, maxit=m, precond="jacobi")
        Xs, infos = solve(As, Bs, variant, p, tol=0.0, maxit=m)
        np.testing.assert_allclose(X, s[:, None] * Xs, rtol=0, atol=1e-10 * np.linalg.norm(X))
        np.testing.assert_allclose(info["ratios"], infos["ratios"], rtol=1e-8)
    _, c1 = solve(A, B, variant, p, tol=1e-8, precond="jacobi")
    _, c2 = solve(As, Bs, variant, p, tol=1e-8)
    assert c1["iterations"] == c2["iterations"] and c1["status"] == c2["status"] == oracle.OK


def test_jacobi_input_checks():
    A, B = _problem(N=5, k=2)
    An = A.tolil()
    An[3, 3] = -1.0
    _, info = solve(An.tocsr(), B, "block", 0, precond="jacobi")
    assert info["status"] == oracle.EINVAL
    _, info = solve(A, B, "block", 0, precond="ilu")
    assert info["status"] == oracle.EINVAL
