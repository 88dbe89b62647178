"""Finite-difference stencil matrices in CSR form (oracle, test infrastructure).

The paper's solver experiment (Section 4) discretises a 2D heterogeneous
Poisson problem with the 5-point stencil; the exact coefficient field is not
given. This module fixes the reading used throughout:

* unknowns are the N**dim interior grid points, Dirichlet neighbours are
  eliminated, lexicographic order with x fastest: c = x + N*y + N*N*z;
* each row lists its columns in ascending order, i.e. the neighbours
  z-, y-, x-, centre, x+, y+, z+ (absent ones skipped);
* constant coefficients give the integer Poisson stencil: 2*dim on the
  diagonal and -1 off the diagonal (exact in FP32 and FP64);
* variable coefficients kappa (one per cell): an interior face between cells
  a and b carries c_f = ((2*kappa_a)*kappa_b)/(kappa_a+kappa_b) (harmonic
  mean, IEEE FP64, evaluated exactly in this operation order), a boundary face
  of cell c carries kappa_c; the off-diagonal entry is -c_f and the diagonal is
  the sum of the cell's face values taken left to right in the fixed order
  x-, x+, y-, y+, z-, z+.

Two builders: ``stencil_csr`` (vectorised NumPy) and ``stencil_csr_loops``
(pure Python, for tiny grids) -- written independently so that one pins the
other.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def stencil_nnz(dim: int, N: int) -> int:
    """Closed form: (2*dim+1)*N^dim minus 2*dim*N^(dim-1) missing neighbours."""
    return (2 * dim + 1) * N ** dim - 2 * dim * N ** (dim - 1)


def _harmonic(ka: np.ndarray, kb: np.ndarray) -> np.ndarray:
    # ((2*ka)*kb)/(ka+kb): each operation rounded once, no fused multiply-add.
    num = np.multiply(np.multiply(2.0, ka), kb)
    den = np.add(ka, kb)
    return np.divide(num, den)


def face_coefficients(dim: int, N: int, kappa: np.ndarray | None):
    """Face values per cell and direction.

    Returns a list over directions d = 0..dim-1 of pairs (minus, plus), each an
    array over cells (lexicographic) holding the coefficient of that cell's
    face in direction -e_d / +e_d (boundary faces carry the cell's own kappa).
    """
    shape = (N,) * dim  # axis order (z, y, x) for dim 3, (y, x) for dim 2
    if kappa is None:
        kap = np.ones(shape)
    else:
        kap = np.asarray(kappa, dtype=np.float64).reshape(shape)
    faces = []
    for d in range(dim):
        ax = dim - 1 - d  # d=0 is x, the last numpy axis
        minus = kap.copy()
        plus = kap.copy()
        lo = [slice(None)] * dim
        hi = [slice(None)] * dim
        lo[ax] = slice(0, N - 1)
        hi[ax] = slice(1, N)
        inner = _harmonic(kap[tuple(lo)], kap[tuple(hi)])  # face between cell i and i+1
        plus[tuple(lo)] = inner
        minus[tuple(hi)] = inner
        faces.append((minus.reshape(-1), plus.reshape(-1)))
    return faces


def stencil_csr(dim: int, N: int, kappa: np.ndarray | None = None) -> sp.csr_matrix:
    """Vectorised CSR build; int32 indices, float64 values."""
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    n = N ** dim
    faces = face_coefficients(dim, N, kappa)
    # diagonal: left-to-right sum in the order x-, x+, y-, y+, z-, z+
    diag = None
    for d in range(dim):
        for f in faces[d]:
            diag = f.copy() if diag is None else diag + f
    idx = np.arange(n, dtype=np.int64)
    coords = [(idx // N ** d) % N for d in range(dim)]  # coords[0] = x
    strides = [N ** d for d in range(dim)]
    # candidate entries in ascending column order: z-, y-, x-, centre, x+, y+, z+
    cols, vals, valid = [], [], []
    for d in reversed(range(dim)):
        cols.append(idx - strides[d])
        vals.append(-faces[d][0])
        valid.append(coords[d] > 0)
    cols.append(idx)
    vals.append(diag)
    valid.append(np.ones(n, dtype=bool))
    for d in range(dim):
        cols.append(idx + strides[d])
        vals.append(-faces[d][1])
        valid.append(coords[d] < N - 1)
    C = np.stack(cols, axis=1)
    V = np.stack(vals, axis=1)
    M = np.stack(valid, axis=1)
    counts = M.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    colind = C[M].astype(np.int32)
    values = V[M].astype(np.float64)
    A = sp.csr_matrix((values, colind, rowptr.astype(np.int32)), shape=(n, n))
    A.has_sorted_indices = True
    return A


def stencil_csr_loops(dim: int, N: int, kappa=None):
    """Pure-Python builder for tiny grids; returns (rowptr, colind, values) lists."""
    n = N ** dim

    def kap(c):
        return 1.0 if kappa is None else float(kappa[c])

    def harm(a, b):
        ka, kb = kap(a), kap(b)
        return ((2.0 * ka) * kb) / (ka + kb)

    rowptr, colind, values = [0], [], []
    for c in range(n):
        xyz = [(c // N ** d) % N for d in range(dim)]
        entries = {}
        face_vals = []  # in the order x-, x+, y-, y+, z-, z+
        for d in range(dim):
            for sgn in (-1, 1):
                nb = xyz[d] + sgn
                if 0 <= nb < N:
                    other = c + sgn * N ** d
                    f = harm(c, other)
                    entries[other] = -f
                else:
                    f = kap(c)
                face_vals.append(f)
        s = face_vals[0]
        for f in face_vals[1:]:
            s = s + f
        entries[c] = s
        for col in sorted(entries):
            colind.append(col)
            values.append(entries[col])
        rowptr.append(len(colind))
    return rowptr, colind, values


def poisson_eigenvalues(dim: int, N: int) -> np.ndarray:
    """Closed-form spectrum of the constant-coefficient stencil, sorted."""
    one = 2.0 - 2.0 * np.cos(np.arange(1, N + 1) * np.pi / (N + 1))
    lam = one
    for _ in range(dim - 1):
        lam = np.add.outer(lam, one).reshape(-1)
    return np.sort(lam)


def poisson_eigenvector(dim: int, N: int, modes) -> np.ndarray:
    """Closed-form eigenvector prod_d sin(i_d*pi*x_d/(N+1)), lexicographic order."""
    x = np.arange(1, N + 1)
    vec = np.ones(1)
    # build with x fastest: outer over (z, y, x) -> ravel C order
    for d in reversed(range(dim)):
        v = np.sin(modes[d] * np.pi * x / (N + 1))
        vec = np.multiply.outer(vec, v).reshape(-1)
    return vec
