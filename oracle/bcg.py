"""Algorithm 1 (stabilised block CG) over the Section 2 *-subalgebras -- oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The iteration follows Algorithm 1 of Section 3 with the preconditioner M = I,
so Z = R. Notation as in the paper: k right-hand sides, block size p dividing
k, q = k/p column groups. Readings of the text that the paper leaves open:

* q is k/p; a group is the contiguous column range [g*p, (g+1)*p)  (Section 2,
  hybrid definition; the Kronecker order printed for the global subalgebra is
  read as I_q (x) S, the only grouping under which the embedding lemma holds);
* the global product sums the q diagonal blocks (index g = 1..q, the printed
  range 0..q being off by one);
* the search-direction update is P <- R + P*beta (the printed minus sign does
  not reduce to CG for k = 1);
* alpha is symmetrised, (alpha + alpha^T)/2, and solved by Cholesky; a
  pivot not above p*eps times its diagonal entry (or non-finite) is a
  breakdown (alpha numerically rank deficient);
* beta solves the recomputed (non-symmetric in floating point) rho of line 6
  by LU with partial pivoting; an exactly zero pivot is a breakdown;
* stop rule (Section 4 only says each column's defect is reduced by 1e-8):
  Euclidean norm of the recursive residual of line 9 relative to the
  column's initial residual, checked right after line 9; all columns must
  pass; the iteration count is the number of products A*P;
* a zero initial-residual column is invalid input unless the subalgebra is
  the diagonal one (parallel, or hybrid with p = 1), where that column's lane
  gets lambda = beta = 0 (1x1 system 0*lambda = 0).

With ``precond="jacobi"`` the preconditioner of Algorithm 1 is M = diag(A)
(lines 2, 10, 11 and 13 use Z = M^{-1} R); reading: the stop rule then
measures each column in the M^{-1}-norm, sqrt(R_j^T M^{-1} R_j), relative to
its initial value (the residual norm preconditioned CG carries), and a
diagonal that is not positive and finite is invalid input.
"""
from __future__ import annotations

import warnings

import numpy as np
import scipy.linalg as sla

from . import EBREAKDOWN, EINVAL, NOT_CONVERGED, OK

VARIANTS = ("block", "global", "parallel", "hybrid")
MAX_K = 256


def normalize_p(variant: str, p: int, k: int) -> int:
    """Block size p of a variant, or ValueError for an invalid combination.

    Section 2: classical = hybrid with p = k; parallel = hybrid with p = 1;
    global and hybrid need p to divide k.
    """
    if not (1 <= k <= MAX_K):
        raise ValueError(f"k={k} outside 1..{MAX_K}")
    if variant == "block":
        if p not in (0, k):
            raise ValueError("block needs p = k (or 0)")
        return k
    if variant == "parallel":
        if p not in (0, 1):
            raise ValueError("parallel needs p = 1 (or 0)")
        return 1
    if variant == "global":
        if p == 0:
            return 1
    elif variant != "hybrid":
        raise ValueError(f"unknown variant {variant!r}")
    if not (1 <= p <= k) or k % p:
        raise ValueError(f"p={p} must divide k={k}")
    return p


def decoupled_columns(variant: str, p: int) -> bool:
    """True when every column is its own 1x1 system (diagonal subalgebra)."""
    return p == 1 and variant in ("parallel", "hybrid")


def block_product(X: np.ndarray, Y: np.ndarray, variant: str, p: int) -> np.ndarray:
    """<<X, Y>>_S of Section 2 in packed form, shape (groups, p, p).

    hybrid/block/parallel: the q diagonal p x p blocks X_g^T Y_g;
    global: their sum (one p x p block, used as I_q (x) S).
    """
    k = X.shape[1]
    q = k // p
    if p == 1:
        d = np.einsum("ij,ij->j", X, Y)[:, None, None]
        return d.sum(axis=0, keepdims=True) if variant == "global" else d
    blocks = np.stack([X[:, g * p:(g + 1) * p].T @ Y[:, g * p:(g + 1) * p] for g in range(q)])
    if variant == "global":
        return blocks.sum(axis=0, keepdims=True)
    return blocks


def apply_coeff(Y: np.ndarray, C: np.ndarray, p: int) -> np.ndarray:
    """Y * c for c in the subalgebra given packed (groups, p, p).

    For the global subalgebra (one block) the same p x p matrix multiplies
    every column group; otherwise group g uses block g.
    """
    n, k = Y.shape
    q = k // p
    out = np.empty_like(Y)
    if p == 1:
        c = C[:, 0, 0]
        return Y * (c if c.shape[0] == k else c[0])
    for g in range(q):
        Cg = C[g] if C.shape[0] == q else C[0]
        out[:, g * p:(g + 1) * p] = Y[:, g * p:(g + 1) * p] @ Cg
    return out


class Breakdown(Exception):
    pass


def cholesky(a: np.ndarray) -> np.ndarray:
    """Lower Cholesky factor of a symmetric block, column by column.

    Breakdown rule: the pivot of column j must exceed p*eps*a[j, j] (and be
    finite); a smaller pivot means alpha is numerically rank deficient, for
    example when two residual columns coincide.
    """
    p = a.shape[0]
    L = np.zeros_like(a)
    eps = np.finfo(np.float64).eps
    for j in range(p):
        d = a[j, j] - L[j, :j] @ L[j, :j]
        if not np.isfinite(d) or not (d > p * eps * a[j, j]) or not (a[j, j] > 0.0):
            raise Breakdown(f"pivot {j} not positive")
        L[j, j] = np.sqrt(d)
        L[j + 1:, j] = (a[j + 1:, j] - L[j + 1:, :j] @ L[j, :j]) / L[j, j]
    return L


def solve_lambda(alpha: np.ndarray, rho: np.ndarray, decoupled: bool) -> np.ndarray:
    """lambda = alpha^{-1} rho per block; alpha symmetrised, then Cholesky."""
    out = np.empty_like(rho)
    for g in range(alpha.shape[0]):
        a = 0.5 * (alpha[g] + alpha[g].T)
        if a.shape[0] == 1:
            if decoupled and a[0, 0] == 0.0 and rho[g, 0, 0] == 0.0:
                out[g] = 0.0
                continue
            if not (a[0, 0] > 0.0) or not np.isfinite(a[0, 0]):
                raise Breakdown("non-positive pivot")
            out[g] = rho[g] / a[0, 0]
            continue
        if not np.all(np.isfinite(a)) or not np.all(np.isfinite(rho[g])):
            raise Breakdown("non-finite block product")
        L = cholesky(a)
        y = sla.solve_triangular(L, rho[g], lower=True, check_finite=False)
        out[g] = sla.solve_triangular(L.T, y, lower=False, check_finite=False)
    return out


def solve_beta(rho_old: np.ndarray, rho_new: np.ndarray, decoupled: bool) -> np.ndarray:
    """beta = rho_old^{-1} rho_new per block, LU with partial pivoting."""
    out = np.empty_like(rho_new)
    for g in range(rho_old.shape[0]):
        r = rho_old[g]
        if r.shape[0] == 1:
            if decoupled and r[0, 0] == 0.0:
                out[g] = 0.0
                continue
            if r[0, 0] == 0.0 or not np.isfinite(r[0, 0]):
                raise Breakdown("zero pivot")
            out[g] = rho_new[g] / r[0, 0]
            continue
        if not np.all(np.isfinite(r)):
            raise Breakdown("non-finite block product")
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            lu, piv = sla.lu_factor(r, check_finite=False)
        if np.any(np.diag(lu) == 0.0):
            raise Breakdown("zero pivot")
        out[g] = sla.lu_solve((lu, piv), rho_new[g], check_finite=False)
    return out


def apply_diag_inverse(V: np.ndarray, minv: np.ndarray | None) -> np.ndarray:
    """M^{-1} V for a diagonal preconditioner given by M^{-1} (one value per
    row); V itself for M = I."""
    return V if minv is None else V * minv[:, None]


def column_norms(R: np.ndarray, minv: np.ndarray | None = None) -> np.ndarray:
    """Euclidean column norms, or the M^{-1}-norms sqrt(R_j^T M^{-1} R_j) for a
    diagonal M given by its inverse ``minv`` (one value per row)."""
    if minv is None:
        return np.sqrt(np.einsum("ij,ij->j", R, R))
    return np.sqrt(np.einsum("ij,ij,i->j", R, R, minv))


def solve(A, B: np.ndarray, variant: str = "block", p: int = 0, tol: float = 1e-8,
          maxit: int = 1000, X0: np.ndarray | None = None, ref_norms: np.ndarray | None = None,
          callback=None, precond: str = "none"):
    """Run Algorithm 1 (M = I, or M = diag(A) with precond="jacobi") and
    return (X, info).

    info: status, iterations, r0 (reference column norms), ratios (final
    ||R_j|| / r0_j of the recursive residual, M^{-1}-norms with Jacobi).
    tol = 0 runs exactly ``maxit`` iterations (fixed-iteration mode).
    ``ref_norms`` replaces the initial residual norms in the stop rule (used
    by the refinement fallback). ``callback(i, X, R)`` is called after each
    iteration's line 9.
    """
    B = np.asarray(B, dtype=np.float64)
    n, k = B.shape
    X = np.zeros_like(B) if X0 is None else np.array(X0, dtype=np.float64, copy=True)
    info = {"status": OK, "iterations": 0, "r0": None, "ratios": None}
    try:
        p = normalize_p(variant, p, k)
    except ValueError:
        info["status"] = EINVAL
        return X, info
    if A.shape != (n, n) or X.shape != (n, k) or maxit < 0 or not (tol >= 0.0) or not np.isfinite(tol):
        info["status"] = EINVAL
        return X, info
    dec = decoupled_columns(variant, p)
    if precond not in ("none", "jacobi"):
        info["status"] = EINVAL
        return X, info
    minv = None  # M^{-1} as one value per row (M = diag(A))
    if precond == "jacobi":
        d = np.asarray(A.diagonal(), dtype=np.float64)
        if not np.all(np.isfinite(d) & (d > 0.0)):
            info["status"] = EINVAL
            return X, info
        minv = 1.0 / d

    def apply_minv(V):
        return apply_diag_inverse(V, minv)

    # line 1: R^0 = B - A X^0 ; line 2: P^1 = M^{-1} R^0
    R = B - A @ X
    r0 = column_norms(R, minv) if ref_norms is None else np.asarray(ref_norms, dtype=np.float64)
    info["r0"] = r0
    if not np.all(np.isfinite(column_norms(R, minv))):
        info["status"] = EINVAL
        return X, info
    if np.all(r0 == 0.0):
        info["ratios"] = np.zeros(k)
        return X, info
    if np.any(r0 == 0.0) and not dec:
        info["status"] = EINVAL
        return X, info
    safe_r0 = np.where(r0 == 0.0, 1.0, r0)
    P = apply_minv(R).copy()
    ratios = column_norms(R, minv) / safe_r0
    for i in range(1, maxit + 1):
        Q = A @ P                                        # line 4
        alpha = block_product(P, Q, variant, p)          # line 5
        rho_old = block_product(P, R, variant, p)        # line 6 (recompute)
        try:
            lam = solve_lambda(alpha, rho_old, dec)      # line 7
        except Breakdown:
            info.update(status=EBREAKDOWN, iterations=i - 1, ratios=ratios)
            return X, info
        X = X + apply_coeff(P, lam, p)                   # line 8
        R = R - apply_coeff(Q, lam, p)                   # line 9
        info["iterations"] = i
        ratios = np.where(r0 == 0.0, 0.0, column_norms(R, minv) / safe_r0)
        if callback is not None:
            callback(i, X, R)
        if np.max(ratios) <= tol:
            info["ratios"] = ratios
            return X, info
        if not np.all(np.isfinite(ratios)):
            info.update(status=EBREAKDOWN, ratios=ratios)
            return X, info
        Z = apply_minv(R)                                # line 10
        rho_new = block_product(Z, R, variant, p)        # line 11
        try:
            beta = solve_beta(rho_old, rho_new, dec)     # line 12
        except Breakdown:
            info.update(status=EBREAKDOWN, ratios=ratios)
            return X, info
        P = Z + apply_coeff(P, beta, p)                  # line 13, sign read as '+'
    info.update(status=NOT_CONVERGED, ratios=ratios)
    return X, info
