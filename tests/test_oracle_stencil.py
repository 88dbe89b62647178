"""Pins of the oracle's stencil matrices (CPU only).

Pins: closed-form nnz, closed-form Poisson spectrum and eigenvectors, a
hand-derived 2x2 diffusion matrix, bitwise symmetry, and agreement of two
independently written builders.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle.stencil import (poisson_eigenvalues, poisson_eigenvector, stencil_csr,
                            stencil_csr_loops, stencil_nnz)
from workload import WORKLOADS, cell_coefficients

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("dim,N", [(2, 1), (2, 2), (2, 5), (2, 32), (3, 1), (3, 2), (3, 7)])
def test_nnz_closed_form(dim, N):
    A = stencil_csr(dim, N)
    assert A.nnz == stencil_nnz(dim, N)
    if dim == 2:
        assert A.nnz == 5 * N * N - 4 * N
    else:
        assert A.nnz == 7 * N ** 3 - 6 * N ** 2


def test_workload_nnz_matches_closed_form():
    expect = {"poisson2d_32_k8": 4992, "poisson3d_128_k16": 14581760,
              "diffusion3d_192_k64": 49324032, "diffusion2d_512_k32": 1308672,
              "poisson3d_256_k128": 117047296}
    for name, z in expect.items():
        assert WORKLOADS[name].nnz == z


@pytest.mark.parametrize("dim,N", [(2, 4), (2, 6), (3, 3), (3, 4)])
def test_poisson_spectrum_closed_form(dim, N):
    A = stencil_csr(dim, N).toarray()
    ev = np.linalg.eigvalsh(A)
    np.testing.assert_allclose(ev, poisson_eigenvalues(dim, N), rtol=0, atol=1e-12)


@pytest.mark.parametrize("dim,N,modes", [(2, 6, (1, 3)), (3, 4, (2, 1, 4))])
def test_poisson_eigenvector_closed_form(dim, N, modes):
    A = stencil_csr(dim, N)
    v = poisson_eigenvector(dim, N, modes)
    lam = sum(2 - 2 * np.cos(m * np.pi / (N + 1)) for m in modes)
    np.testing.assert_allclose(A @ v, lam * v, atol=1e-12)


def test_poisson_integer_entries_and_sorted_columns():
    for dim, N in [(2, 9), (3, 5)]:
        A = stencil_csr(dim, N)
        rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
        on = rows == A.indices
        assert np.all(A.data[on] == 2.0 * dim)
        assert np.all(A.data[~on] == -1.0)
        for i in range(A.shape[0]):
            c = A.indices[A.indptr[i]:A.indptr[i + 1]]
            assert np.all(np.diff(c) > 0)
        assert A.indices.dtype == np.int32 and A.indptr.dtype == np.int32


def _golden_matrix():
    entries, kappa = {}, None
    with open(os.path.join(GOLDEN, "diffusion2d_N2.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == "kappa":
                kappa = np.array([float(x) for x in parts[1:]])
                continue
            entries[(int(parts[0]), int(parts[1]))] = Fraction(parts[2])
    return kappa, entries


def test_hand_derived_diffusion_2x2():
    kappa, entries = _golden_matrix()
    A = stencil_csr(2, 2, kappa).toarray()
    for i in range(4):
        for j in range(4):
            exact = entries.get((i, j), Fraction(0))
            # a few roundings per entry: within 4 ulp of the exact rational
            assert abs(Fraction(A[i, j]) - exact) <= 4 * abs(exact) * Fraction(2) ** -52


@pytest.mark.parametrize("dim,N,sigma", [(2, 5, 0.0), (2, 6, 1.0), (3, 3, 0.5), (3, 4, 1.0)])
def test_builders_agree_bitwise(dim, N, sigma):
    kappa = None if sigma == 0 else cell_coefficients(dim, N, sigma)
    A = stencil_csr(dim, N, kappa)
    rp, ci, va = stencil_csr_loops(dim, N, kappa)
    assert np.array_equal(A.indptr, np.array(rp))
    assert np.array_equal(A.indices, np.array(ci))
    assert np.array_equal(A.data.view(np.uint64), np.array(va, dtype=np.float64).view(np.uint64))


@pytest.mark.parametrize("dim,N,sigma", [(2, 12, 1.0), (3, 6, 0.5)])
def test_diffusion_bitwise_symmetric_and_spd(dim, N, sigma):
    kappa = cell_coefficients(dim, N, sigma)
    A = stencil_csr(dim, N, kappa)
    At = A.T.tocsr()
    At.sort_indices()
    assert np.array_equal(A.indptr, At.indptr) and np.array_equal(A.indices, At.indices)
    assert np.array_equal(A.data.view(np.uint64), At.data.view(np.uint64))
    assert np.linalg.eigvalsh(A.toarray()).min() > 0


def test_unit_kappa_is_poisson_bitwise():
    for dim, N in [(2, 7), (3, 4)]:
        A = stencil_csr(dim, N)
        B = stencil_csr(dim, N, np.ones(N ** dim))
        assert np.array_equal(A.data.view(np.uint64), B.data.view(np.uint64))


def test_diffusion_row_sums_are_boundary_faces():
    # Interior faces cancel in a row sum; what is left is the sum of the
    # cell's boundary-face coefficients (kappa_c per boundary face).
    dim, N = 2, 8
    kappa = cell_coefficients(dim, N, 1.0)
    A = stencil_csr(dim, N, kappa)
    rs = np.asarray(A.sum(axis=1)).ravel()
    idx = np.arange(N * N)
    x, y = idx % N, idx // N
    nb = (x == 0).astype(int) + (x == N - 1) + (y == 0) + (y == N - 1)
    np.testing.assert_allclose(rs, nb * kappa, rtol=1e-13, atol=1e-13)
