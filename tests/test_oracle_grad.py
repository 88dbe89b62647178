"""Pins of the oracle's gradients and mixed-precision solve (CPU only).

Gradient pins: a dense FP64 solve of the perturbed (possibly non-symmetric)
system by finite differences, the dense outer-product formula, and finite
differences of the stencil assembly. Mixed precision: the final FP64 true
residual and the distance to a dense solve (the precision policy of its inner
iterations is pinned in tests/test_oracle_refine_policy.py).
"""
import numpy as np
import pytest

import oracle
from oracle import refine
from oracle.bcg import solve
from oracle.grad import assemble_values, kappa_vjp, sampled_outer
from oracle.stencil import stencil_csr
from workload import cell_coefficients, loss_weights, rhs


def _small(dim=2, N=6, k=3, sigma=0.5):
    kappa = cell_coefficients(dim, N, sigma)
    A = stencil_csr(dim, N, kappa)
    B = rhs(A.shape[0], k, "normal")
    W = loss_weights(A.shape[0], k)
    return kappa, A, B, W


def test_sampled_outer_matches_dense_formula():
    _, A, B, W = _small()
    Ad = A.toarray()
    X = np.linalg.solve(Ad, B)
    Y = np.linalg.solve(Ad, W)
    full = -Y @ X.T
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    np.testing.assert_allclose(sampled_outer(A, Y, X, -1.0), full[rows, A.indices], rtol=1e-13, atol=1e-15)


def test_value_gradient_matches_fd_of_dense_solve():
    # perturb one stored entry (A becomes non-symmetric; dense solve is fine)
    _, A, B, W = _small(N=5)
    Ad = A.toarray()
    X = np.linalg.solve(Ad, B)
    Y = np.linalg.solve(Ad.T, W)
    g = sampled_outer(A, Y, X, -1.0)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    rng = np.random.default_rng(7)
    h = 1e-6
    for e in rng.choice(A.nnz, 12, replace=False):
        i, j = rows[e], A.indices[e]
        Ap, Am = Ad.copy(), Ad.copy()
        Ap[i, j] += h
        Am[i, j] -= h
        fd = (np.sum(W * np.linalg.solve(Ap, B)) - np.sum(W * np.linalg.solve(Am, B))) / (2 * h)
        assert abs(fd - g[e]) <= 1e-7 * max(1.0, abs(g[e]))


def test_kappa_vjp_matches_fd_of_assembly():
    for dim, N in [(2, 5), (3, 3)]:
        kappa = cell_coefficients(dim, N, 1.0)
        A = stencil_csr(dim, N, kappa)
        rng = np.random.default_rng(3)
        u = rng.standard_normal(A.nnz)
        v = rng.standard_normal(N ** dim)
        h = 1e-6
        fd = u @ (assemble_values(dim, N, kappa + h * v, A) - assemble_values(dim, N, kappa - h * v, A)) / (2 * h)
        ad = kappa_vjp(dim, N, kappa, A, u) @ v
        assert abs(fd - ad) <= 1e-7 * max(1.0, abs(ad))


def test_coefficient_gradient_chain_matches_fd():
    dim, N = 2, 6
    kappa, A, B, W = _small(dim=dim, N=N)
    X, info = solve(A, B, "block", 0, tol=1e-13, maxit=500)
    Y, info2 = solve(A, W, "block", 0, tol=1e-13, maxit=500)
    assert info["status"] == info2["status"] == oracle.OK
    gk = kappa_vjp(dim, N, kappa, A, sampled_outer(A, Y, X, -1.0))
    h = 1e-6
    for c in [0, 7, 20, 35]:
        kp, km = kappa.copy(), kappa.copy()
        kp[c] += h
        km[c] -= h
        Lp = np.sum(W * np.linalg.solve(stencil_csr(dim, N, kp).toarray(), B))
        Lm = np.sum(W * np.linalg.solve(stencil_csr(dim, N, km).toarray(), B))
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - gk[c]) <= 1e-6 * max(abs(gk[c]), 1e-3 * np.max(np.abs(gk)))


@pytest.mark.parametrize("variant,p", [("block", 0), ("hybrid", 2), ("global", 1), ("parallel", 1)])
def test_refine_reaches_fp64_accuracy(variant, p):
    kappa, A, B, _ = _small(dim=2, N=12, k=4, sigma=1.0)
    tol = 1e-10
    X, info = refine.solve(A, B, variant, p, tol=tol, inner_tol=1e-4, inner_maxit=500)
    assert info["status"] == oracle.OK
    R = B - A @ X
    rel = np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0)
    assert np.max(rel) <= tol
    Xd = np.linalg.solve(A.toarray(), B)
    cond = np.linalg.cond(A.toarray())
    assert np.linalg.norm(X - Xd) / np.linalg.norm(Xd) <= cond * tol
    assert info["outer_iterations"] >= 2          # FP32 alone cannot reach 1e-10
