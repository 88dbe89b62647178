"""Independent characterisation of the block CG iterates (test helper).

For a *-subalgebra S of R^{k x k} with basis {E_t}, the m-th iterate of block
CG over S is the element of X0 + K^m_S(A, R0) (Section 2, block Krylov
subspace definition) that minimises the trace A-norm of the error,
sum_j ||x*_j - x_j||_A^2. Writing X = X0 + sum_{i<m, t} theta_{i,t} A^i R0 E_t,
the minimiser solves the normal equations

    G theta = h,  G_{(i,t),(j,u)} = tr((A^i R0 E_t)^T A (A^j R0 E_u)),
                  h_{(i,t)}      = tr((A^i R0 E_t)^T R0),

because A (X* - X0) = R0. This shares nothing with Algorithm 1 and pins the
oracle's recurrences, projections, signs and transposes.
"""
from __future__ import annotations

import numpy as np


def subalgebra_basis(variant: str, k: int, p: int):
    """Basis matrices of S_Cl, S_Hy^p, S_Pl or S_Gl^p (contiguous groups)."""
    q = k // p
    basis = []
    if variant == "global":
        for a in range(p):
            for b in range(p):
                E = np.zeros((k, k))
                for g in range(q):
                    E[g * p + a, g * p + b] = 1.0
                basis.append(E)
        return basis
    # block (p = k), hybrid, parallel (p = 1): independent entries of each diagonal block
    for g in range(q):
        for a in range(p):
            for b in range(p):
                E = np.zeros((k, k))
                E[g * p + a, g * p + b] = 1.0
                basis.append(E)
    return basis


def galerkin_iterate(A, B, X0, variant, p, m, minv=None):
    """m-th iterate; with a diagonal preconditioner (``minv`` = M^{-1}, one
    value per row) the space is X0 + K^m_S(M^{-1} A, M^{-1} R0), the one the
    preconditioned iteration searches, with the same A-norm criterion."""
    A = np.asarray(A.todense()) if hasattr(A, "todense") else np.asarray(A)
    R0 = B - A @ X0
    k = B.shape[1]
    basis = subalgebra_basis(variant, k, p)
    scale = (lambda V: V) if minv is None else (lambda V: V * np.asarray(minv)[:, None])
    dirs = []
    V = scale(R0)
    for _ in range(m):
        for E in basis:
            dirs.append(V @ E)
        V = scale(A @ V)
    nd = len(dirs)
    G = np.empty((nd, nd))
    h = np.empty(nd)
    AD = [A @ D for D in dirs]
    for i in range(nd):
        h[i] = np.sum(dirs[i] * R0)
        for j in range(i, nd):
            G[i, j] = G[j, i] = np.sum(dirs[i] * AD[j])
    theta = np.linalg.lstsq(G, h, rcond=None)[0]
    X = X0.copy()
    for t, D in zip(theta, dirs):
        X = X + t * D
    return X


def trace_a_error(A, Xstar, X):
    E = Xstar - X
    return float(np.sum(E * (A @ E)))
