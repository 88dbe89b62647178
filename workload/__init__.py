"""Seeded synthetic inputs for the block CG workloads.

This module is shared by the GPU library's tests and benchmark and by the CPU
oracle. It holds the workload table (grid sizes, right-hand-side counts,
variants, tolerances) and the random draws, and nothing of the method's
arithmetic: no matrix assembly, no solver step, no reduction.

Draw conventions (fixed so that every consumer sees the same bits):

* generator: ``numpy.random.default_rng(seed)`` (PCG64);
* cell coefficients: ``rng.lognormal(0, sigma, N**dim)``, one value per grid
  cell in lexicographic order (x fastest), seed 0;
* right-hand sides: ``(n, k)`` in C order, seed 1; ``uniform`` is
  ``rng.uniform(-1, 1, (n, k))``, ``normal`` is ``rng.standard_normal((n, k))``;
* loss weights W for the differentiable solve: standard normal ``(n, k)``,
  seed 2;
* finite-difference probe indices: ``rng.choice(N**dim, count, replace=False)``,
  seed 3;
* long-range index pairs (test matrices with entries far from the diagonal
  and rows longer than the stencils'): ``rng.integers(0, n, (n * per_row, 2))``,
  pairs with equal entries dropped, seed 4.

The paper's second experiment (Section 4) uses a 2D heterogeneous Poisson
problem with a 5-point stencil and random right-hand sides; its coefficient
field and grid are not given, so the diffusion workloads below stand in for it.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Tuple

import numpy as np

SEED_COEFF = 0
SEED_RHS = 1
SEED_LOSS_W = 2
SEED_FD_INDEX = 3
SEED_PAIRS = 4


@dataclass(frozen=True)
class Workload:
    """One synthetic system: grid, coefficient field, right-hand sides."""

    name: str
    dim: int                  # 2 (5-point stencil) or 3 (7-point stencil)
    N: int                    # interior grid points per axis; n = N**dim
    k: int                    # number of right-hand sides
    rhs: str                  # "uniform" (U[-1,1]) or "normal" (N(0,1))
    sigma: float = 0.0        # log-normal sigma of cell coefficients; 0 = Poisson
    variants: Tuple[Tuple[str, int], ...] = ()
    tol: float = 1e-8
    precision: Tuple[str, ...] = ("fp64",)
    notes: str = ""
    extra: dict = field(default_factory=dict, compare=False, hash=False)

    @property
    def n(self) -> int:
        return self.N ** self.dim

    @property
    def nnz(self) -> int:
        # (2*dim+1) entries per row minus the missing neighbours on the
        # Dirichlet boundary: 5N^2-4N in 2D, 7N^3-6N^2 in 3D.
        return (2 * self.dim + 1) * self.N ** self.dim - 2 * self.dim * self.N ** (self.dim - 1)


WORKLOADS = {
    w.name: w
    for w in [
        Workload(
            name="poisson2d_32_k8",
            dim=2, N=32, k=8, rhs="uniform",
            variants=(("block", 8), ("global", 1), ("parallel", 1), ("hybrid", 2), ("hybrid", 4)),
            tol=1e-8,
            notes="2D 5-point Poisson 32x32, n=1024, k=8; small parity case",
        ),
        Workload(
            name="poisson3d_128_k16",
            dim=3, N=128, k=16, rhs="uniform",
            variants=(("block", 16), ("global", 1), ("parallel", 1), ("hybrid", 4)),
            tol=1e-8,
            notes="3D 7-point Poisson 128^3, n=2,097,152, k=16; FP64 solve",
        ),
        Workload(
            name="diffusion3d_192_k64",
            dim=3, N=192, k=64, rhs="normal", sigma=1.0,
            variants=(("hybrid", 8), ("block", 64)),
            tol=1e-10, precision=("fp32_refine", "fp64"),
            notes="3D 7-point diffusion 192^3, log-normal sigma=1, k=64",
        ),
        Workload(
            name="diffusion2d_512_k32",
            dim=2, N=512, k=32, rhs="normal", sigma=0.5,
            variants=(("block", 32),),
            tol=1e-8,
            notes="2D 5-point diffusion 512^2, sigma=0.5, k=32; forward + adjoint",
            extra={"fd_count": 64, "fd_step": 1e-6},
        ),
        Workload(
            name="poisson3d_256_k128",
            dim=3, N=256, k=128, rhs="uniform",
            variants=(("hybrid", 8), ("hybrid", 16), ("global", 1)),
            tol=1e-8, precision=("fp32_refine", "fp64"),
            notes="3D 7-point Poisson 256^3, n=16,777,216, k=128",
        ),
    ]
}


def cell_coefficients(dim: int, N: int, sigma: float, seed: int = SEED_COEFF) -> np.ndarray:
    """Per-cell log-normal coefficients, lexicographic (x fastest), float64."""
    rng = np.random.default_rng(seed)
    return rng.lognormal(0.0, sigma, N ** dim)


def rhs(n: int, k: int, dist: str, seed: int = SEED_RHS) -> np.ndarray:
    """(n, k) right-hand sides, C order, float64."""
    rng = np.random.default_rng(seed)
    if dist == "uniform":
        return rng.uniform(-1.0, 1.0, (n, k))
    if dist == "normal":
        return rng.standard_normal((n, k))
    raise ValueError(f"unknown right-hand-side distribution {dist!r}")


def loss_weights(n: int, k: int, seed: int = SEED_LOSS_W) -> np.ndarray:
    """(n, k) standard-normal weights W of the scalar loss sum(W * X)."""
    return np.random.default_rng(seed).standard_normal((n, k))


def fd_indices(ncells: int, count: int, seed: int = SEED_FD_INDEX) -> np.ndarray:
    """Distinct coefficient indices probed by the finite-difference check."""
    return np.random.default_rng(seed).choice(ncells, count, replace=False)


def long_range_pairs(n: int, per_row: int, seed: int = SEED_PAIRS) -> Tuple[np.ndarray, np.ndarray]:
    """Random (row, column) index pairs with row != column, about per_row per row."""
    ij = np.random.default_rng(seed).integers(0, n, (n * per_row, 2))
    keep = ij[:, 0] != ij[:, 1]
    return ij[keep, 0], ij[keep, 1]


def coefficients_for(w: Workload) -> np.ndarray | None:
    """Cell coefficients of a workload, or None for the constant Poisson case."""
    if w.sigma == 0.0:
        return None
    return cell_coefficients(w.dim, w.N, w.sigma)


def rhs_for(w: Workload) -> np.ndarray:
    return rhs(w.n, w.k, w.rhs)
