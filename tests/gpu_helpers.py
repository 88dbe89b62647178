"""Shared helpers of the GPU tests: move oracle inputs to the device and back."""
import numpy as np
import scipy.sparse as sp
import torch

DEV = "cuda"


def csr_to_dev(A: sp.csr_matrix):
    rowptr = torch.from_numpy(A.indptr.astype(np.int32)).to(DEV)
    colind = torch.from_numpy(A.indices.astype(np.int32)).to(DEV)
    values = torch.from_numpy(A.data.astype(np.float64)).to(DEV)
    return rowptr, colind, values


def dev(x: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def rel(a: np.ndarray, b: np.ndarray) -> float:
    """Largest per-column relative error max_j ||a_j - b_j|| / ||b_j|| of two
    n x k blocks (a vector is one column), so that one wrong column or row
    block cannot hide in the norm of the others. A zero column of b is
    measured against the largest column norm of b (1 if b is zero)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.ndim == 1:
        a, b = a[:, None], b[:, None]
    assert a.shape == b.shape, (a.shape, b.shape)
    nb = np.linalg.norm(b, axis=0)
    top = float(nb.max()) if nb.size and nb.max() > 0 else 1.0
    den = np.where(nb > 0, nb, top)
    return float(np.max(np.linalg.norm(a - b, axis=0) / den))


def log(msg: str) -> None:
    print(msg, flush=True)
