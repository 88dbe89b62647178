"""Adjoint-solve gradients of X = A^{-1} B -- oracle, test infrastructure only.

For a scalar loss L(X) with G = dL/dX and A symmetric positive definite:

* dL/dB = A^{-T} G = A^{-1} G =: Y (one more solve with the same A);
* dL/dA = -Y X^T, so the derivative with respect to the stored value of
  CSR entry e = (i, j) is -sum_c Y[i, c] X[j, c] (the dense outer product
  sampled on the sparsity pattern);
* the cell coefficients enter through the stencil assembly (harmonic faces,
  see ``oracle.stencil``), so dL/dkappa is the assembly's transpose Jacobian
  applied to dL/dvalues.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .stencil import face_coefficients


def sampled_outer(A: sp.csr_matrix, Y: np.ndarray, X: np.ndarray, alpha: float = -1.0) -> np.ndarray:
    """out[e] = alpha * <Y[row(e), :], X[col(e), :]> for every stored entry e."""
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    cols = A.indices
    return alpha * np.einsum("ec,ec->e", Y[rows], X[cols])


def _harmonic_partials(ka: np.ndarray, kb: np.ndarray):
    """d/dka and d/dkb of h = 2 ka kb / (ka + kb)."""
    s2 = (ka + kb) ** 2
    return 2.0 * kb * kb / s2, 2.0 * ka * ka / s2


def kappa_vjp(dim: int, N: int, kappa: np.ndarray, A: sp.csr_matrix, dvalues: np.ndarray) -> np.ndarray:
    """dL/dkappa from dL/dvalues (values in the CSR order of ``A``).

    Every interior face f between cells a and b appears in the values as
    +c_f in diag(a) and diag(b) and as -c_f at (a, b) and (b, a); a boundary
    face of cell c appears as +kappa_c in diag(c).
    """
    n = N ** dim
    kap = np.asarray(kappa, dtype=np.float64)
    D = sp.csr_matrix((np.asarray(dvalues, dtype=np.float64), A.indices, A.indptr), shape=A.shape)
    ddiag = D.diagonal()
    out = np.zeros(n)
    idx = np.arange(n)
    coords = [(idx // N ** d) % N for d in range(dim)]
    for d in range(dim):
        s = N ** d
        has_plus = coords[d] < N - 1
        a = idx[has_plus]
        b = a + s
        da, db = _harmonic_partials(kap[a], kap[b])
        off = np.asarray(D[a, b]).ravel() + np.asarray(D[b, a]).ravel()
        w = ddiag[a] + ddiag[b] - off          # dL/dc_f
        np.add.at(out, a, w * da)
        np.add.at(out, b, w * db)
        # boundary faces: minus side at coord 0, plus side at coord N-1
        for bnd in (coords[d] == 0, coords[d] == N - 1):
            c = idx[bnd]
            np.add.at(out, c, ddiag[c])
    return out


def assemble_values(dim: int, N: int, kappa: np.ndarray, A: sp.csr_matrix) -> np.ndarray:
    """CSR values of the diffusion stencil for coefficients kappa on A's pattern."""
    from .stencil import stencil_csr
    M = stencil_csr(dim, N, kappa)
    assert np.array_equal(M.indptr, A.indptr) and np.array_equal(M.indices, A.indices)
    return M.data


__all__ = ["sampled_outer", "kappa_vjp", "assemble_values", "face_coefficients"]
