"""Pins of the refinement oracle's precision policy (CPU only).

The mixed-precision inner solve is not in the paper; its reading fixes four
rules on top of the block CG iteration (Algorithm 1, Section 3):

1. the block products are accumulated in FP64 from the FP32 operands;
2. the Cholesky and LU solves for lambda and beta run in FP64;
3. lambda and beta are rounded to FP32 before they multiply FP32 blocks;
4. the sparse product and the block updates are FP32 operations on FP32 data.

Each pin below picks inputs for which one rule changes the result and derives
the expected value with exact rational arithmetic (``fractions.Fraction``) and
explicit round-to-nearest-even to 24 or 53 significant bits, so the expected
values share no arithmetic with the oracle:

* block products: FP32 entries whose pairwise products need 47 bits, so an
  FP32 accumulation loses bits that an FP64 one keeps;
* coefficient rounding: coefficients a fraction of an FP32 ulp away from an
  FP32 number, so an update with the unrounded coefficient rounds the other
  way;
* whole iterations: the parallel (p = 1) inner iteration simulated step by step
  on a tiny system with exact arithmetic and the policy's roundings, compared
  bit for bit;
* a band: after m inner iterations the FP32 iterates must differ from the FP64
  iteration on the same FP32-rounded system at FP32 level, not at FP64 level
  and not by O(1).

``tests/test_oracle_mutations.py`` plants the two plausible policy mistakes
(no FP32 rounding of the coefficients; block products accumulated in FP32)
and requires these pins to catch them.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import refine
from oracle.bcg import solve as solve64
from oracle.stencil import stencil_csr
from workload import cell_coefficients, rhs


def round_bits(x: Fraction, bits: int) -> Fraction:
    """Round a rational to the nearest number with `bits` significant bits
    (ties to even); the exponent range of the test values is normal."""
    if x == 0:
        return Fraction(0)
    sign = -1 if x < 0 else 1
    a = abs(x)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    while Fraction(2) ** e > a:
        e -= 1
    while Fraction(2) ** (e + 1) <= a:
        e += 1
    scale = Fraction(2) ** (bits - 1 - e)
    m = a * scale
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return sign * Fraction(fl) / scale


def r32(x: Fraction) -> Fraction:
    return round_bits(x, 24)


def r64(x: Fraction) -> Fraction:
    return round_bits(x, 53)


def F(v) -> Fraction:
    return Fraction(float(v))


def f32_array(vals) -> np.ndarray:
    """FP32 array of exact rationals that must be FP32 numbers."""
    out = np.array([float(v) for v in vals], dtype=np.float32)
    assert all(F(o) == v for o, v in zip(out, vals)), "test value not an FP32 number"
    return out


# ---------------------------------------------------------------- rule 1 --
def _gram_operands():
    """X, Y (4 x 4, FP32): entries 1 + m 2^-23 (and two other binades), so
    every product carries up to 47 significant bits."""
    u = Fraction(1, 2 ** 23)
    mx = [[1, 3, 5, 7], [2 ** 22 + 1, 9, 4095, 77], [11, 2 ** 23 - 1, 13, 1], [8191, 3, 2 ** 21 + 5, 17]]
    my = [[5, 2 ** 23 - 3, 7, 1], [3, 1, 99, 2 ** 20 + 7], [2 ** 22 - 1, 5, 3, 11], [1, 255, 1, 3]]
    X = [[(1 + mx[i][j] * u) * (2 if j == 1 else 1) for j in range(4)] for i in range(4)]
    Y = [[(1 + my[i][j] * u) * (Fraction(1, 2) if j == 2 else 1) for j in range(4)] for i in range(4)]
    return X, Y


def gram_pin_mismatches() -> list:
    """Names of the block products whose value is not the exact FP64 one."""
    X, Y = _gram_operands()
    X32 = np.array([f32_array(r) for r in X])
    Y32 = np.array([f32_array(r) for r in Y])
    n, k = 4, 4
    bad = []
    exact = [[sum(X[i][a] * Y[i][b] for i in range(n)) for b in range(k)] for a in range(k)]
    # the exact sums fit 53 bits, so FP64 accumulation in any order is exact
    assert all(r64(exact[a][b]) == exact[a][b] for a in range(k) for b in range(k))
    cases = {
        ("block", 4): [[[exact[a][b] for b in range(4)] for a in range(4)]],
        ("hybrid", 2): [[[exact[g * 2 + a][g * 2 + b] for b in range(2)] for a in range(2)] for g in range(2)],
        ("global", 2): [[[exact[a][b] + exact[2 + a][2 + b] for b in range(2)] for a in range(2)]],
        ("parallel", 1): [[[exact[j][j]]] for j in range(4)],
        ("global", 1): [[[sum(exact[j][j] for j in range(4))]]],
    }
    for (variant, p), want in cases.items():
        got = refine._block_product64(X32, Y32, variant, p)
        if got.dtype != np.float64 or got.shape != (len(want), p, p):
            bad.append((variant, p, "dtype/shape"))
            continue
        ok = all(F(got[g, a, b]) == want[g][a][b] for g in range(len(want)) for a in range(p) for b in range(p))
        if not ok:
            bad.append((variant, p))
    return bad


def test_block_products_accumulate_in_fp64_from_fp32():
    assert gram_pin_mismatches() == []


def test_gram_operands_separate_fp32_accumulation():
    # the pin is sensitive: an FP32 sum of the same products differs
    X, Y = _gram_operands()
    X32 = np.array([f32_array(r) for r in X])
    Y32 = np.array([f32_array(r) for r in Y])
    g32 = X32.T @ Y32
    exact = [[sum(X[i][a] * Y[i][b] for i in range(4)) for b in range(4)] for a in range(4)]
    assert g32.dtype == np.float32
    assert sum(F(g32[a, b]) != exact[a][b] for a in range(4) for b in range(4)) >= 8


# ---------------------------------------------------------------- rule 3 --
def _apply_cases():
    """(Y rows, packed coefficients, p, variant-shaped packing) with exact
    expected values of the policy: coefficients rounded to FP32, products and
    sums of the update rounded once to FP32 (the sums below are exact in FP32
    summation order too, so the FP32 accumulation of the update is covered)."""
    u = Fraction(1, 2 ** 23)
    cases = []
    # p = 1: lambda a fraction 0.453 of an FP32 ulp above 1 rounds to 1; the
    # unrounded product 1.25 * lambda lies 0.566 ulp above 1.25
    lam = [1 + 29 * u / 64, Fraction(3, 4) - 61 * u / 256, 2 + 13 * u / 32, 1 - 3 * u / 16]
    Y = [[Fraction(5, 4), Fraction(7, 4), Fraction(3, 2), Fraction(13, 8)],
         [Fraction(9, 8), 1, Fraction(15, 8), Fraction(5, 4)]]
    cases.append((Y, [[[c]] for c in lam], 1))
    # p = 2: the coefficient column (1 + 2^-25, 2^-25 + 2^-50) rounds to
    # (1, 2^-25); the policy's update of the row (1, 1) is fl32(1 + 2^-25) = 1,
    # the unrounded one fl32(1 + 2^-24 + 2^-50) = 1 + 2^-23
    t = Fraction(1, 2 ** 25)
    C = [[1 + t, Fraction(1, 2)], [t + Fraction(1, 2 ** 50), 1 + 3 * t]]
    Y2 = [[1, 1], [Fraction(1, 2), 2]]
    cases.append((Y2, [C], 2))
    return cases


def apply_pin_mismatches() -> list:
    bad = []
    for ci, (Y, C, p) in enumerate(_apply_cases()):
        n, k = len(Y), len(Y[0])
        Y32 = np.array([f32_array(r) for r in Y])
        C64 = np.array([[[float(c) for c in row] for row in blk] for blk in C])
        assert all(F(C64[g, a, b]) == C[g][a][b] for g in range(len(C)) for a in range(p) for b in range(p))
        got = refine._apply32(Y32, C64, p)
        if got.dtype != np.float32:
            bad.append((ci, "dtype"))
            continue
        q = k // p
        for i in range(n):
            for g in range(q):
                blk = C[g] if len(C) == q else C[0]
                for b in range(p):
                    want = r32(sum(Y[i][g * p + a] * r32(blk[a][b]) for a in range(p)))
                    if F(got[i, g * p + b]) != want:
                        bad.append((ci, i, g * p + b))
    return bad


def test_coefficients_rounded_to_fp32_before_update():
    assert apply_pin_mismatches() == []


def test_apply_cases_separate_unrounded_coefficients():
    # the pin is sensitive: with the FP64 coefficients every case differs
    for Y, C, p in _apply_cases():
        k = len(Y[0])
        q = k // p
        diff = 0
        for i in range(len(Y)):
            for g in range(q):
                blk = C[g] if len(C) == q else C[0]
                for b in range(p):
                    pol = r32(sum(Y[i][g * p + a] * r32(blk[a][b]) for a in range(p)))
                    unr = r32(sum(Y[i][g * p + a] * blk[a][b] for a in range(p)))
                    diff += pol != unr
        assert diff >= 1


# ---------------------------------------------------- rules 1-4 together --
def _tiny_system():
    """1D Dirichlet Laplacian (2 on the diagonal, -1 off it), n = 7, and two
    right-hand sides of small dyadic numbers (exact in FP32)."""
    n = 7
    A = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")
    A.sort_indices()
    R = [[Fraction(v, 16) for v in row] for row in
         [[3, -5], [7, 1], [-2, 9], [11, -4], [5, 6], [-9, 2], [1, -13]]]
    return A, R


def simulate_parallel(A: sp.csr_matrix, R0, m: int, global_: bool):
    """m inner iterations of the policy for p = 1 (parallel, or global with
    one p x p = 1 x 1 block), every value an exact rational with explicit
    roundings: FP32 sparse product accumulated in CSR order, products exact
    and rounded to FP64, lambda and beta exact quotients rounded to FP32 (the
    FP64 solve then rounding to FP32 gives the same FP32 number unless the
    quotient sits within about 2^-29 of an FP32 rounding boundary, which these
    inputs avoid), updates rounded to FP32."""
    n, k = len(R0), len(R0[0])
    indptr, indices, data = A.indptr, A.indices, A.data
    R = [row[:] for row in R0]
    P = [row[:] for row in R0]
    X = [[Fraction(0)] * k for _ in range(n)]

    def spmv(V):
        out = [[Fraction(0)] * k for _ in range(n)]
        for i in range(n):
            for j in range(k):
                acc = Fraction(0)
                for e in range(indptr[i], indptr[i + 1]):
                    acc = r32(acc + F(data[e]) * V[indices[e]][j])
                out[i][j] = acc
        return out

    def dots(U, V):
        return [r64(sum(U[i][j] * V[i][j] for i in range(n))) for j in range(k)]

    for _ in range(m):
        Q = spmv(P)
        al, rho = dots(P, Q), dots(P, R)
        if global_:
            al, rho = [r64(sum(al))] * k, [r64(sum(rho))] * k
        lam = [r32(rho[j] / al[j]) for j in range(k)]
        X = [[r32(X[i][j] + r32(P[i][j] * lam[j])) for j in range(k)] for i in range(n)]
        R = [[r32(R[i][j] - r32(Q[i][j] * lam[j])) for j in range(k)] for i in range(n)]
        rn = dots(R, R)
        if global_:
            rn = [r64(sum(rn))] * k
        beta = [r32(rn[j] / rho[j]) for j in range(k)]
        P = [[r32(R[i][j] + r32(P[i][j] * beta[j])) for j in range(k)] for i in range(n)]
    return X


def iteration_pin_mismatches(m: int = 4) -> list:
    A, R0 = _tiny_system()
    A32 = A.astype(np.float32)
    R32 = np.array([f32_array(r) for r in R0])
    bad = []
    for variant, global_ in (("parallel", False), ("global", True)):
        want = simulate_parallel(A, R0, m, global_)
        D, its, st = refine.inner_solve32(A32, R32, variant, 1, 0.0, m)
        if its != m or D.dtype != np.float32:
            bad.append((variant, "iterations/dtype", its, D.dtype))
            continue
        for i in range(len(R0)):
            for j in range(len(R0[0])):
                if F(D[i, j]) != want[i][j]:
                    bad.append((variant, i, j))
    return bad


def test_inner_iterations_match_exact_policy_simulation():
    assert iteration_pin_mismatches() == []


# ------------------------------------------------------------------ band --
BAND_CASES = [("block", 0), ("hybrid", 2), ("parallel", 1), ("global", 1)]


def band_ratios(variant, p, m=8):
    """Per-column relative difference of m FP32 inner iterations from m FP64
    iterations (oracle) on the same FP32-rounded matrix and right-hand sides."""
    A = stencil_csr(2, 16, cell_coefficients(2, 16, 0.5))
    A32 = A.astype(np.float32)
    A64 = A32.astype(np.float64)
    B32 = rhs(A.shape[0], 4, "normal", seed=11).astype(np.float32)
    p_eff = refine.normalize_p(variant, p, 4)
    D, its, st = refine.inner_solve32(A32, B32, variant, p_eff, 0.0, m)
    X, info = solve64(A64, B32.astype(np.float64), variant, p, tol=0.0, maxit=m)
    assert its == info["iterations"] == m
    return np.linalg.norm(D.astype(np.float64) - X, axis=0) / np.linalg.norm(X, axis=0)


@pytest.mark.parametrize("variant,p", BAND_CASES)
def test_fp32_iterates_differ_from_fp64_at_fp32_level(variant, p):
    r = band_ratios(variant, p)
    # FP32 unit roundoff is 6e-8; eight iterations on this system amplify it
    # by at most a few hundred; FP64 arithmetic would give ~1e-15, a wrong
    # rule O(1)
    assert np.all(r >= 1e-8), r
    assert np.all(r <= 1e-5), r
