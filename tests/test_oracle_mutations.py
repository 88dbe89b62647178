"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each case monkeypatches one step of the oracle's Algorithm 1 with a plausible
error (wrong sign, transposed coefficient, wrong side of a solve, interleaved
column groups, dropped symmetric half) and checks that the independent
trace-A-norm Galerkin characterisation (or textbook CG) rejects it.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle.bcg as ob
from oracle.stencil import stencil_csr
from tests.galerkin import galerkin_iterate
from workload import cell_coefficients, rhs


def _setup():
    A = stencil_csr(2, 7, cell_coefficients(2, 7, 1.0))
    B = rhs(A.shape[0], 4, "uniform")
    X0 = np.zeros_like(B)
    return A, B, X0


def _galerkin_mismatch(variant, p, m=3):
    A, B, X0 = _setup()
    X, _ = ob.solve(A, B, variant, p, tol=0.0, maxit=m, X0=X0)
    Xg = galerkin_iterate(A, B, X0, variant, p, m)
    return np.linalg.norm(X - Xg) / np.linalg.norm(Xg)


def test_unmutated_passes():
    for v, p in [("block", 4), ("hybrid", 2), ("global", 2), ("parallel", 1)]:
        assert _galerkin_mismatch(v, p) < 1e-9


def _apply_transposed(Y, C, p):
    return _orig_apply(Y, np.transpose(C, (0, 2, 1)).copy(), p)


_orig_apply = ob.apply_coeff
_orig_product = ob.block_product
_orig_beta = ob.solve_beta


def _interleaved_product(X, Y, variant, p):
    k = X.shape[1]
    q = k // p
    perm = np.array([g + q * a for g in range(q) for a in range(p)])  # groups {g, g+q, ...}
    return _orig_product(X[:, perm], Y[:, perm], variant, p)


def _beta_wrong_side(rho_old, rho_new, dec):
    out = np.empty_like(rho_new)
    for g in range(rho_old.shape[0]):
        out[g] = rho_new[g] @ np.linalg.inv(rho_old[g])
    return out


def _product_upper_only(X, Y, variant, p):
    G = _orig_product(X, Y, variant, p)
    return np.triu(G)


@pytest.mark.parametrize("mutation,variant,p", [
    ("transposed_coefficients", "block", 4),
    ("interleaved_groups", "hybrid", 2),
    ("interleaved_groups", "global", 2),
    ("beta_wrong_side", "block", 4),
    ("upper_triangle_gram", "block", 4),
])
def test_mutation_is_caught(monkeypatch, mutation, variant, p):
    if mutation == "transposed_coefficients":
        monkeypatch.setattr(ob, "apply_coeff", _apply_transposed)
    elif mutation == "interleaved_groups":
        monkeypatch.setattr(ob, "block_product", _interleaved_product)
    elif mutation == "beta_wrong_side":
        monkeypatch.setattr(ob, "solve_beta", _beta_wrong_side)
    elif mutation == "upper_triangle_gram":
        monkeypatch.setattr(ob, "block_product", _product_upper_only)
    assert _galerkin_mismatch(variant, p) > 1e-6


def test_minus_sign_update_is_caught(monkeypatch):
    # Replace line 13 by P <- R - P beta through a negated beta.
    def neg_beta(rho_old, rho_new, dec):
        return -_orig_beta(rho_old, rho_new, dec)
    monkeypatch.setattr(ob, "solve_beta", neg_beta)
    A, B, _ = _setup()
    x2, _ = spla.cg(A, B[:, 0], x0=np.zeros(A.shape[0]), rtol=0.0, atol=0.0, maxiter=3)
    X, _ = ob.solve(A, B[:, :1], "block", 0, tol=0.0, maxit=3)
    assert np.linalg.norm(X[:, 0] - x2) > 1e-6 * np.linalg.norm(x2)
    assert _galerkin_mismatch("block", 4) > 1e-6


_orig_minv = ob.apply_diag_inverse


@pytest.mark.parametrize("mutation", ["preconditioner_dropped", "m_instead_of_m_inverse"])
@pytest.mark.parametrize("variant,p", [("block", 4), ("hybrid", 2), ("global", 2)])
def test_jacobi_mutation_is_caught(monkeypatch, mutation, variant, p):
    # Lines 2 and 10 of the preconditioned iteration: Z = R (M ignored) or
    # Z = M R (inverse forgotten) must fail the preconditioned Galerkin pin.
    if mutation == "preconditioner_dropped":
        monkeypatch.setattr(ob, "apply_diag_inverse", lambda V, minv: V)
    else:
        monkeypatch.setattr(ob, "apply_diag_inverse",
                            lambda V, minv: V if minv is None else V / minv[:, None])
    A, B, X0 = _setup()
    minv = 1.0 / A.diagonal()
    X, _ = ob.solve(A, B, variant, p, tol=0.0, maxit=3, X0=X0, precond="jacobi")
    Xg = galerkin_iterate(A, B, X0, variant, p, 3, minv=minv)
    assert np.linalg.norm(X - Xg) > 1e-6 * np.linalg.norm(Xg)


def test_jacobi_unmutated_passes():
    A, B, X0 = _setup()
    minv = 1.0 / A.diagonal()
    for v, p in [("block", 4), ("hybrid", 2), ("global", 2)]:
        X, _ = ob.solve(A, B, v, p, tol=0.0, maxit=3, X0=X0, precond="jacobi")
        Xg = galerkin_iterate(A, B, X0, v, p, 3, minv=minv)
        assert np.linalg.norm(X - Xg) < 1e-9 * np.linalg.norm(Xg)


# ---- precision policy of the refinement oracle (tests/test_oracle_refine_policy.py) ----
import oracle.refine as orf  # noqa: E402
from tests import test_oracle_refine_policy as pol  # noqa: E402


def _apply32_unrounded(Y32, C64, p):
    # the coefficients multiply the FP32 block without being rounded to FP32
    n, k = Y32.shape
    q = k // p
    if p == 1:
        c = C64[:, 0, 0]
        return (Y32 * (c if c.shape[0] == k else c[0])).astype(np.float32)
    out = np.empty_like(Y32)
    for g in range(q):
        Cg = C64[g] if C64.shape[0] == q else C64[0]
        out[:, g * p:(g + 1) * p] = Y32[:, g * p:(g + 1) * p] @ Cg
    return out


def _product_fp32_accumulated(X32, Y32, variant, p):
    # the block product summed in FP32, widened only at the end
    return ob.block_product(X32, Y32, variant, p).astype(np.float64)


def _policy_pins_fail():
    fails = []
    if pol.gram_pin_mismatches():
        fails.append("gram")
    if pol.apply_pin_mismatches():
        fails.append("apply")
    if pol.iteration_pin_mismatches():
        fails.append("iterations")
    return fails


def test_refine_policy_unmutated_passes():
    assert _policy_pins_fail() == []


@pytest.mark.parametrize("mutation", ["coefficients_not_rounded", "gram_fp32_accumulated"])
def test_refine_policy_mutation_is_caught(monkeypatch, mutation):
    if mutation == "coefficients_not_rounded":
        monkeypatch.setattr(orf, "_apply32", _apply32_unrounded)
    else:
        monkeypatch.setattr(orf, "_block_product64", _product_fp32_accumulated)
    fails = _policy_pins_fail()
    assert fails, mutation
    # the whole-iteration pin catches both on its own
    assert "iterations" in fails


# ---- residual replacement of the reliable refinement oracle (tests/test_oracle_reliable.py) ----
from tests import test_oracle_reliable as rel_pins  # noqa: E402


def _rescale_rho_linear(P, rho_old, f, policy32):
    # the line-6 product scaled like one operand only
    P = (P * np.float32(f)).astype(np.float32) if policy32 else P * f
    return P, rho_old * f


def _rescale_direction_kept(P, rho_old, f, policy32):
    # the search direction left in the old units
    return P, rho_old * (f * f)


def _rescale_restart(P, rho_old, f, policy32):
    # a restart in place of the continued direction: with P = 0 the next
    # line 13 gives P = R
    return np.zeros_like(P), rho_old * (f * f)


def _reliable_pin_fails(variant, p):
    try:
        err, ir, its64 = rel_pins.reliable_fp64_mismatch(variant, p, maxit=1000)
    except Exception:  # a breakdown is a failure of the pin too
        return True
    return not (ir["status"] == 0 and abs(ir["iterations"] - its64) <= 2 and err <= 1e-8)


def test_reliable_unmutated_passes():
    assert not _reliable_pin_fails("block", 0)
    assert not _reliable_pin_fails("parallel", 1)


@pytest.mark.parametrize("mutation", [_rescale_rho_linear, _rescale_direction_kept, _rescale_restart])
@pytest.mark.parametrize("variant,p", [("block", 0), ("parallel", 1), ("hybrid", 2)])
def test_reliable_mutation_is_caught(monkeypatch, mutation, variant, p):
    monkeypatch.setattr(orf, "_rescale_direction", mutation)
    assert _reliable_pin_fails(variant, p)
