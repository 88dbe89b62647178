"""FP32 inner block CG with FP64 outer iterative refinement -- oracle.

TEST INFRASTRUCTURE ONLY. Not in the paper: this is the mixed-precision form
of Algorithm 1 (Section 3, M = I). Pinned on the CPU by
tests/test_oracle_refine_policy.py: its block products against exact sums of
FP32 operands, its coefficient rounding against exact rational updates, whole
parallel inner iterations bit for bit against an exact-arithmetic simulation
of the policy, and the distance of its FP32 iterates from the FP64 iteration
(FP32 level). The GPU's inner iterates agree with it up to the rounding order
of the FP32 sums; the final FP64 accuracy is compared as well.

Inner solve (one restart per outer step, X starts at 0):
  matrix values, the sparse product and all n x k block vectors in FP32;
  the block products accumulated in FP64 from the FP32 inputs; the Cholesky
  and LU solves in FP64; lambda and beta rounded to FP32 before the updates;
  stop when every column's recursive residual fell by ``inner_tol`` relative
  to the inner initial residual, or after ``inner_maxit`` iterations.
Outer loop:
  R = B - A X in FP64; stop when max_j ||R_j|| / ||R0_j|| <= tol;
  scale by the single scalar s = max_j ||R_j|| (a per-column scale is not an
  element of every subalgebra); solve A D = R/s in FP32 to the reduction
  inner_target() (the remaining factor 0.5 tol/ratio, but no deeper than
  inner_tol/4; inner_tol 0 means 4e-6 for groups of p <= 16, 1e-4 for wider
  ones); X += s * D;
  if an outer step does not halve the largest relative residual, finish with
  the FP64 iteration from the current X (flagged in the result).

``solve_reliable`` is the other scheme: one FP32 iteration with the same
inner policy whose search direction is kept across the FP64 corrections
(residual replacement). Pinned by tests/test_oracle_reliable.py: with every
quantity kept in FP64 it reproduces the FP64 iteration (in exact arithmetic
the replaced residual is the recursive one), and with the FP32 policy it
reaches the tolerance in the true residual.
"""
from __future__ import annotations

import numpy as np

from . import EBREAKDOWN, EINVAL, NOT_CONVERGED, OK
from .bcg import (Breakdown, decoupled_columns, normalize_p, solve as solve64, solve_beta,
                  solve_lambda)


def _block_product64(X32, Y32, variant, p):
    X = X32.astype(np.float64)
    Y = Y32.astype(np.float64)
    from .bcg import block_product
    return block_product(X, Y, variant, p)


def _apply32(Y32, C64, p):
    C = C64.astype(np.float32)
    n, k = Y32.shape
    q = k // p
    if p == 1:
        c = C[:, 0, 0]
        return Y32 * (c if c.shape[0] == k else c[0])
    out = np.empty_like(Y32)
    for g in range(q):
        Cg = C[g] if C.shape[0] == q else C[0]
        out[:, g * p:(g + 1) * p] = Y32[:, g * p:(g + 1) * p] @ Cg
    return out


def _norms32(R32):
    R = R32.astype(np.float64)
    return np.sqrt(np.einsum("ij,ij->j", R, R))


def inner_solve32(A32, R32, variant, p, inner_tol, inner_maxit):
    """FP32 block CG from X = 0 on A D = R32; returns (D, iterations, status)."""
    dec = decoupled_columns(variant, p)
    R = R32.copy()
    X = np.zeros_like(R32)
    r0 = _norms32(R)
    if np.any(r0 == 0.0) and not dec:
        return X, 0, EINVAL
    safe = np.where(r0 == 0.0, 1.0, r0)
    P = R.copy()
    for i in range(1, inner_maxit + 1):
        Q = (A32 @ P).astype(np.float32)
        alpha = _block_product64(P, Q, variant, p)
        rho_old = _block_product64(P, R, variant, p)
        try:
            lam = solve_lambda(alpha, rho_old, dec)
        except Breakdown:
            return X, i - 1, EBREAKDOWN
        X = X + _apply32(P, lam, p)
        R = R - _apply32(Q, lam, p)
        ratios = np.where(r0 == 0.0, 0.0, _norms32(R) / safe)
        if np.max(ratios) <= inner_tol:
            return X, i, OK
        if not np.all(np.isfinite(ratios)):
            return X, i, EBREAKDOWN
        rho_new = _block_product64(R, R, variant, p)
        try:
            beta = solve_beta(rho_old, rho_new, dec)
        except Breakdown:
            return X, i, EBREAKDOWN
        P = R + _apply32(P, beta, p)
    return X, inner_maxit, NOT_CONVERGED


def inner_target(inner_tol, tol, ratio):
    """Reduction asked of the next inner solve: the remaining factor tol/ratio
    (with a factor 2 of margin), but no deeper than inner_tol/4."""
    need = 0.5 * tol / ratio
    if not (need > 0.0) or need >= 1.0:
        return inner_tol
    return float(min(max(need, 0.25 * inner_tol), 0.5))


def effective_inner_tol(inner_tol, p):
    """inner_tol 0 selects 4e-6 for groups of p <= 16, 1e-4 for wider ones."""
    return inner_tol if inner_tol > 0.0 else (4e-6 if p <= 16 else 1e-4)


def _rescale_direction(P, rho_old, f, policy32):
    """The search direction and the line-6 product of the last iteration in
    the units of a new residual scale (s_old / s_new = f): both operands of
    rho_old = <<P, R>> scale by f, so P *= f (FP32: the factor and the product
    rounded to FP32) and rho_old *= f^2 (FP64)."""
    P = (P * np.float32(f)).astype(np.float32) if policy32 else P * f
    return P, rho_old * (f * f)


def solve_reliable(A, B, variant="block", p=0, tol=1e-8, delta=1e-2, maxit=100000, X0=None,
                   policy32=True, callback=None):
    """Mixed-precision block CG with residual replacement (not in the paper).

    One FP32 iteration of Algorithm 1 (the inner policy of ``inner_solve32``)
    runs on the scaled system A D = R/s. Its search direction is kept across
    the FP64 corrections instead of being restarted: whenever the recursive
    residual (in units of the current scale s) has fallen to ``delta`` times
    its value at the last correction, or to ``tol``, the correction is applied
    and the residual replaced (residual replacement, van der Vorst and Ye,
    SIAM J. Sci. Comput. 22 (2000); reliable updates, Sleijpen and van der
    Vorst, Computing 56 (1996)):

      X += s D (FP64);  D = 0;  R = B - A X (FP64);  stop if max_j ||R_j|| /
      ||R0_j|| <= tol;  s' = max_j ||R_j||;  R32 = R / s';  P32 *= s / s';
      rho_old *= (s / s')^2;  s = s'

    and the iteration continues with line 10 (rho_new from the replaced
    residual, beta, P = R + P beta). In exact arithmetic the replaced
    residual equals the recursive one, so the iterates are those of the FP64
    iteration (the pin of ``policy32=False``, which keeps every quantity in
    FP64). A correction that does not halve the largest relative residual
    since the previous one ends the solve with the FP64 iteration from the
    current X (``fp64_fallback``). ``maxit`` caps the FP32 iterations.
    Returns (X, info) with FP64 X; info["iterations"] counts FP32 iterations,
    info["replacements"] the corrections.
    """
    B = np.asarray(B, dtype=np.float64)
    n, k = B.shape
    X = np.zeros_like(B) if X0 is None else np.array(X0, dtype=np.float64, copy=True)
    info = {"status": OK, "iterations": 0, "replacements": 0, "fp64_fallback": False}
    try:
        p = normalize_p(variant, p, k)
    except ValueError:
        info["status"] = EINVAL
        return X, info
    dec = decoupled_columns(variant, p)
    if policy32:
        A32, f32 = A.astype(np.float32), np.float32
        gram = _block_product64
        apply = _apply32

        def spmv(M):
            return (A32 @ M).astype(np.float32)
    else:
        f32 = np.float64
        from .bcg import apply_coeff, block_product
        gram = block_product
        apply = apply_coeff

        def spmv(M):
            return A @ M

    def cnorms(M):
        M = M.astype(np.float64)
        return np.sqrt(np.einsum("ij,ij->j", M, M))

    R64 = B - A @ X
    r0 = cnorms(R64)
    if not np.all(np.isfinite(r0)):
        info["status"] = EINVAL
        return X, info
    if np.all(r0 == 0.0):
        info["true_ratio"] = 0.0
        return X, info
    if np.any(r0 == 0.0) and not dec:
        info["status"] = EINVAL
        return X, info
    safe = np.where(r0 == 0.0, 1.0, r0)
    s = float(np.max(r0))
    R = (R64 / s).astype(f32)
    P = R.copy()
    D = np.zeros_like(R)
    last = 1.0   # largest true relative residual at the last correction
    i = 0
    while True:
        if i >= maxit:
            X = X + s * D.astype(np.float64)
            info["status"] = NOT_CONVERGED
            return X, info
        i += 1
        Q = spmv(P)                                    # line 4
        alpha = gram(P, Q, variant, p)                 # line 5
        rho_old = gram(P, R, variant, p)               # line 6
        try:
            lam = solve_lambda(alpha, rho_old, dec)    # line 7
        except Breakdown:
            info.update(status=EBREAKDOWN, iterations=i - 1)
            return X + s * D.astype(np.float64), info
        D = D + apply(P, lam, p)                       # line 8
        R = R - apply(Q, lam, p)                       # line 9
        info["iterations"] = i
        est = float(np.max(np.where(r0 == 0.0, 0.0, s * cnorms(R) / safe)))
        if not np.isfinite(est):
            info["status"] = EBREAKDOWN
            return X + s * D.astype(np.float64), info
        if callback is not None:
            callback(i, X + s * D.astype(np.float64), est)
        if est <= tol or est <= delta * last:
            # correction and residual replacement
            X = X + s * D.astype(np.float64)
            D = np.zeros_like(D)
            R64 = B - A @ X
            c = cnorms(R64)
            true = float(np.max(np.where(r0 == 0.0, 0.0, c / safe)))
            info["replacements"] += 1
            if true <= tol:
                info["true_ratio"] = true
                return X, info
            if not (true <= 0.5 * last):
                X, sub = solve64(A, B, variant, p, tol, maxit=100000, X0=X, ref_norms=r0)
                info["fp64_fallback"] = True
                info["status"] = sub["status"]
                return X, info
            last = true
            s_new = float(np.max(c))
            R = (R64 / s_new).astype(f32)
            P, rho_old = _rescale_direction(P, rho_old, s / s_new, policy32)
            s = s_new
        rho_new = gram(R, R, variant, p)               # line 11
        try:
            beta = solve_beta(rho_old, rho_new, dec)   # line 12
        except Breakdown:
            info["status"] = EBREAKDOWN
            return X + s * D.astype(np.float64), info
        P = R + apply(P, beta, p)                      # line 13


def solve(A, B, variant="block", p=0, tol=1e-8, maxit=50, inner_tol=0.0, inner_maxit=1000,
          X0=None):
    """Mixed-precision solve; returns (X, info) with FP64 X. ``maxit`` caps the
    refinement steps."""
    B = np.asarray(B, dtype=np.float64)
    n, k = B.shape
    X = np.zeros_like(B) if X0 is None else np.array(X0, dtype=np.float64, copy=True)
    info = {"status": OK, "iterations": 0, "outer_iterations": 0, "fp64_fallback": False}
    try:
        p = normalize_p(variant, p, k)
    except ValueError:
        info["status"] = EINVAL
        return X, info
    A32 = A.astype(np.float32)
    R = B - A @ X
    r0 = np.sqrt(np.einsum("ij,ij->j", R, R))
    if not np.all(np.isfinite(r0)):
        info["status"] = EINVAL
        return X, info
    if np.all(r0 == 0.0):
        return X, info
    if np.any(r0 == 0.0) and not decoupled_columns(variant, p):
        info["status"] = EINVAL
        return X, info
    safe = np.where(r0 == 0.0, 1.0, r0)
    prev = np.inf
    outer = 0
    while True:
        c = np.sqrt(np.einsum("ij,ij->j", R, R))
        ratio = float(np.max(np.where(r0 == 0.0, 0.0, c / safe)))
        if ratio <= tol:
            info["true_ratio"] = ratio
            return X, info
        stagnated = ratio > 0.5 * prev
        if not stagnated and outer >= maxit:
            info["status"] = NOT_CONVERGED
            return X, info
        D = None
        if not stagnated:
            outer += 1
            prev = ratio
            s = float(np.max(c))
            D, its, st = inner_solve32(A32, (R / s).astype(np.float32), variant, p,
                                       inner_target(effective_inner_tol(inner_tol, p), tol, ratio), inner_maxit)
            info["iterations"] += its
            info["outer_iterations"] = outer
            if st < 0:
                D = None
        if D is None:
            X, sub = solve64(A, B, variant, p, tol, maxit=100000, X0=X, ref_norms=r0)
            info["fp64_fallback"] = True
            info["iterations"] += sub["iterations"]
            info["status"] = sub["status"]
            return X, info
        X = X + s * D.astype(np.float64)
        R = B - A @ X
