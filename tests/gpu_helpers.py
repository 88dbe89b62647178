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
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def log(msg: str) -> None:
    print(msg, flush=True)
