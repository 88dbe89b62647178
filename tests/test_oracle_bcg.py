"""Pins of the oracle's block CG (CPU only).

Each pin comes from outside the oracle: a dense direct solve, the textbook CG
of SciPy (k = 1 and the parallel subalgebra), the trace-A-norm Galerkin
characterisation of every variant (tests/galerkin.py), the stacked-system
equivalence from the proof of the global-rate lemma (Section 3), the
subspace-inclusion and embedding lemmas (Section 2), closed-form Poisson
eigenvectors, and finite termination.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from oracle.bcg import normalize_p, solve
from oracle.stencil import poisson_eigenvector, stencil_csr
from tests.galerkin import galerkin_iterate, trace_a_error
from workload import cell_coefficients, rhs

VARS = [("block", 0), ("global", 1), ("global", 2), ("parallel", 1), ("hybrid", 2), ("hybrid", 4)]


def _problem(dim=2, N=8, k=4, sigma=0.0, dist="uniform", seed=1):
    kappa = None if sigma == 0 else cell_coefficients(dim, N, sigma)
    A = stencil_csr(dim, N, kappa)
    B = rhs(A.shape[0], k, dist, seed)
    return A, B


def test_normalize_p_table():
    assert normalize_p("block", 0, 8) == 8 and normalize_p("block", 8, 8) == 8
    assert normalize_p("parallel", 0, 8) == 1 and normalize_p("parallel", 1, 8) == 1
    assert normalize_p("global", 0, 8) == 1 and normalize_p("global", 4, 8) == 4
    assert normalize_p("hybrid", 2, 8) == 2
    for bad in [("block", 4, 8), ("parallel", 2, 8), ("hybrid", 3, 8), ("hybrid", 0, 8),
                ("global", 16, 8), ("nope", 1, 8), ("block", 0, 0), ("block", 0, 257)]:
        with pytest.raises(ValueError):
            normalize_p(*bad)


@pytest.mark.parametrize("variant,p", VARS)
def test_converged_matches_dense_solve(variant, p):
    A, B = _problem(dim=2, N=10, k=4, sigma=0.5)
    X, info = solve(A, B, variant, p, tol=1e-10, maxit=2000)
    assert info["status"] == oracle.OK
    Xd = np.linalg.solve(A.toarray(), B)
    cond = np.linalg.cond(A.toarray())
    err = np.linalg.norm(X - Xd) / np.linalg.norm(Xd)
    assert err <= cond * 1e-10 * 10
    assert np.max(info["ratios"]) <= 1e-10


@pytest.mark.parametrize("variant,p", [("block", 0), ("global", 0), ("parallel", 0), ("hybrid", 1)])
def test_k1_is_textbook_cg(variant, p):
    A, B = _problem(dim=2, N=9, k=1, sigma=1.0)
    b = B[:, 0]
    its = []
    spla.cg(A, b, x0=np.zeros_like(b), rtol=0.0, atol=0.0, maxiter=12,
            callback=lambda x: its.append(x.copy()))
    for m in (1, 2, 5, 12):
        X, info = solve(A, B, variant, p, tol=0.0, maxit=m)
        assert info["iterations"] == m
        np.testing.assert_allclose(X[:, 0], its[m - 1], rtol=0, atol=1e-10 * np.linalg.norm(its[m - 1]))


def test_parallel_is_k_independent_cg_runs():
    A, B = _problem(dim=2, N=9, k=5, sigma=0.5)
    m = 7
    X, _ = solve(A, B, "parallel", 1, tol=0.0, maxit=m)
    for j in range(B.shape[1]):
        xj, _ = spla.cg(A, B[:, j], x0=np.zeros(A.shape[0]), rtol=0.0, atol=0.0, maxiter=m)
        np.testing.assert_allclose(X[:, j], xj, rtol=0, atol=1e-10 * np.linalg.norm(xj))


def test_global1_is_cg_on_kronecker_system():
    # S_Gl^1 = R (x) I_k: one scalar per step, i.e. CG on (I_k (x) A) vec(X) = vec(B)
    A, B = _problem(dim=2, N=7, k=3, sigma=1.0)
    n, k = B.shape
    Ak = sp.block_diag([A] * k, format="csr")
    b = B.T.reshape(-1)  # column stacking
    for m in (1, 4, 9):
        x, _ = spla.cg(Ak, b, x0=np.zeros(n * k), rtol=0.0, atol=0.0, maxiter=m)
        X, _ = solve(A, B, "global", 1, tol=0.0, maxit=m)
        np.testing.assert_allclose(X.T.reshape(-1), x, rtol=0, atol=1e-10 * np.linalg.norm(x))


@pytest.mark.parametrize("p", [1, 2, 3])
def test_global_is_classical_on_stacked_system(p):
    # proof of the global-rate lemma: global^p on A == classical BCG with p RHS
    # on diag(A, ..., A) (q copies) with the q column groups stacked as rows
    A, B = _problem(dim=2, N=6, k=6, sigma=0.7)
    n, k = B.shape
    q = k // p
    As = sp.block_diag([A] * q, format="csr")
    Bs = np.vstack([B[:, g * p:(g + 1) * p] for g in range(q)])
    for m in (1, 3, 6):
        X, _ = solve(A, B, "global", p, tol=0.0, maxit=m)
        Xs, _ = solve(As, Bs, "block", 0, tol=0.0, maxit=m)
        Xback = np.hstack([Xs[g * n:(g + 1) * n] for g in range(q)])
        np.testing.assert_allclose(X, Xback, rtol=0, atol=1e-12 * np.linalg.norm(X))


@pytest.mark.parametrize("variant,p", [("block", 4), ("hybrid", 2), ("parallel", 1),
                                       ("global", 1), ("global", 2)])
@pytest.mark.parametrize("m", [1, 2, 3])
def test_iterates_are_trace_a_norm_galerkin(variant, p, m):
    A, B = _problem(dim=2, N=7, k=4, sigma=1.0)
    X0 = 0.1 * rhs(A.shape[0], 4, "normal", seed=11)
    X, _ = solve(A, B, variant, p, tol=0.0, maxit=m, X0=X0)
    Xg = galerkin_iterate(A, B, X0, variant, p, m)
    np.testing.assert_allclose(X, Xg, rtol=0, atol=1e-9 * np.linalg.norm(Xg))


def test_hybrid_is_independent_block_runs_and_aliases():
    A, B = _problem(dim=2, N=8, k=6, sigma=0.5)
    m = 6
    Xh, _ = solve(A, B, "hybrid", 3, tol=0.0, maxit=m)
    for g in range(2):
        Xg, _ = solve(A, B[:, 3 * g:3 * g + 3], "block", 0, tol=0.0, maxit=m)
        np.testing.assert_allclose(Xh[:, 3 * g:3 * g + 3], Xg, rtol=0, atol=1e-13 * np.linalg.norm(Xg))
    Xb, _ = solve(A, B, "block", 0, tol=0.0, maxit=m)
    np.testing.assert_allclose(solve(A, B, "hybrid", 6, tol=0.0, maxit=m)[0], Xb, rtol=0, atol=1e-13)
    np.testing.assert_allclose(solve(A, B, "global", 6, tol=0.0, maxit=m)[0], Xb, rtol=0, atol=1e-13)
    Xp, _ = solve(A, B, "parallel", 1, tol=0.0, maxit=m)
    np.testing.assert_allclose(solve(A, B, "hybrid", 1, tol=0.0, maxit=m)[0], Xp, rtol=0, atol=1e-13)


@pytest.mark.parametrize("m", [2, 4, 8])
def test_subalgebra_inclusion_monotone_error(m):
    # Section 2 lemmas: S1 within S2 => K_S1 within K_S2; with the iterates
    # minimising the trace A-norm error over X0 + K, the richer subalgebra
    # never has the larger error at equal iteration count.
    A, B = _problem(dim=2, N=10, k=8, sigma=1.0, dist="normal")
    Xs = np.linalg.solve(A.toarray(), B)
    E = {}
    for name, v, p in [("Pl", "parallel", 1), ("Hy2", "hybrid", 2), ("Hy4", "hybrid", 4),
                       ("Cl", "block", 8), ("Gl1", "global", 1), ("Gl2", "global", 2),
                       ("Gl4", "global", 4)]:
        X, _ = solve(A, B, v, p, tol=0.0, maxit=m)
        E[name] = trace_a_error(A, Xs, X)
    slack = 1 + 1e-8
    for lo, hi in [("Pl", "Hy2"), ("Hy2", "Hy4"), ("Hy4", "Cl"), ("Gl1", "Gl2"), ("Gl2", "Gl4"),
                   ("Gl4", "Cl"), ("Gl1", "Pl"), ("Gl2", "Hy2"), ("Gl4", "Hy4")]:
        assert E[hi] <= E[lo] * slack, (lo, hi, E[lo], E[hi])


def test_eigenvector_rhs_converges_in_one_block_iteration():
    dim, N = 2, 12
    A = stencil_csr(dim, N)
    modes = [(1, 1), (2, 3), (5, 1), (4, 4)]
    V = np.stack([poisson_eigenvector(dim, N, md) for md in modes], axis=1)
    M = rhs(4, 4, "normal", seed=5)           # mix: span unchanged
    B = V @ M
    X, info = solve(A, B, "block", 0, tol=1e-10, maxit=5)
    assert info["status"] == oracle.OK and info["iterations"] == 1


def test_eigenvector_mixture_parallel_converges_in_m_iterations():
    dim, N = 2, 12
    A = stencil_csr(dim, N)
    modes = [(1, 1), (2, 3), (5, 1)]          # distinct eigenvalues
    V = np.stack([poisson_eigenvector(dim, N, md) for md in modes], axis=1)
    B = np.stack([V[:, 0], V[:, 0] + V[:, 1], V[:, 0] + V[:, 1] + V[:, 2]], axis=1)
    X, info = solve(A, B, "parallel", 1, tol=1e-10, maxit=10)
    assert info["status"] == oracle.OK and info["iterations"] == 3
    for m, j in [(1, 0), (2, 1)]:
        Xm, inf = solve(A, B, "parallel", 1, tol=0.0, maxit=m)
        assert inf["ratios"][j] < 1e-10 and inf["ratios"][j + 1] > 1e-6


def test_finite_termination_classical():
    dim, N, k = 2, 4, 4                       # n = 16, n/k = 4
    A, B = _problem(dim=dim, N=N, k=k, sigma=0.3)
    X, info = solve(A, B, "block", 0, tol=0.0, maxit=N * N // k)
    assert np.max(info["ratios"]) < 1e-9


def test_status_codes():
    A, B = _problem(dim=2, N=6, k=4)
    # invalid p
    assert solve(A, B, "hybrid", 3)[1]["status"] == oracle.EINVAL
    # NaN in B
    Bn = B.copy(); Bn[3, 1] = np.nan
    assert solve(A, Bn, "block")[1]["status"] == oracle.EINVAL
    # zero column: invalid unless decoupled
    Bz = B.copy(); Bz[:, 2] = 0.0
    for v, p in [("block", 0), ("hybrid", 2), ("global", 1)]:
        assert solve(A, Bz, v, p)[1]["status"] == oracle.EINVAL
    Xz, iz = solve(A, Bz, "parallel", 1, tol=1e-10, maxit=500)
    assert iz["status"] == oracle.OK and np.all(Xz[:, 2] == 0.0)
    Xr, _ = solve(A, B[:, [0, 1, 3]], "parallel", 1, tol=0.0, maxit=iz["iterations"])
    np.testing.assert_allclose(Xz[:, [0, 1, 3]], Xr, rtol=0, atol=1e-14)
    # all-zero B: immediate success
    X0, i0 = solve(A, np.zeros_like(B), "block")
    assert i0["status"] == oracle.OK and i0["iterations"] == 0
    # not converged
    assert solve(A, B, "block", tol=1e-12, maxit=2)[1]["status"] == oracle.NOT_CONVERGED
    # breakdown: negative definite operator (negated diagonal)
    An = A.copy(); An.setdiag(-A.diagonal())
    Xb, ib = solve(An, B, "block")
    assert ib["status"] == oracle.EBREAKDOWN and ib["iterations"] == 0 and np.all(Xb == 0)
    # breakdown: rank-deficient block [b, b]
    Bd = np.stack([B[:, 0], B[:, 0]], axis=1)
    assert solve(A, Bd, "block")[1]["status"] == oracle.EBREAKDOWN
    # but parallel handles duplicated columns
    assert solve(A, Bd, "parallel", 1, tol=1e-10, maxit=500)[1]["status"] == oracle.OK


def test_p_update_sign_reading():
    # With the printed '-' sign the k = 1 recursion is not CG: its second
    # iterate differs from SciPy's, which the '+' reading matches.
    A, B = _problem(dim=2, N=9, k=1, sigma=0.5)
    x2, _ = spla.cg(A, B[:, 0], x0=np.zeros(A.shape[0]), rtol=0.0, atol=0.0, maxiter=2)
    X, _ = solve(A, B, "block", 0, tol=0.0, maxit=2)
    np.testing.assert_allclose(X[:, 0], x2, atol=1e-12)
