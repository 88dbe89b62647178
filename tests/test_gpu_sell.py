"""SELL-C-sigma storage of the sparse product (Section 4), on the GPU.

With sigma = 1 every row keeps its position and every row of Q = A P is
summed from the same entries in the same order (padding adds exact zeros),
so a solve must be bitwise the same as with CSR: iteration counts and X.
With sorting (sigma > 1) rows change steps and the partial products of the
Gram matrices are summed in another order; those iterates are compared with
the FP64 oracle at the fixed-iteration tolerance of the CSR path (1e-10
relative, Frobenius).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import torch

import oracle
from oracle.bcg import solve as oracle_solve
from oracle.stencil import stencil_csr
from tests.gpu_helpers import csr_to_dev, dev, host, log, rel
from workload import WORKLOADS, cell_coefficients, long_range_pairs, rhs, rhs_for

pytestmark = pytest.mark.gpu

FIXED_TOL = 1e-10


def _P():
    import paper_1912_11930_amd as P
    return P


def _long_range(N=40, per_row=6):
    """2D diffusion plus symmetric far couplings: rows of 8 to ~30 entries,
    diagonally dominant (SPD)."""
    A = stencil_csr(2, N, cell_coefficients(2, N, 0.5))
    n = A.shape[0]
    i, j = long_range_pairs(n, per_row)
    C = sp.coo_matrix((np.full(i.size, -0.05), (i, j)), shape=(n, n)).tocsr()
    C = C + C.T
    d = np.asarray(abs(C).sum(axis=1)).ravel()
    return (A + C + sp.diags(d)).tocsr()


def _matrix(name):
    if name == "diffusion3d_13":      # n = 2197: a ragged last slice, rows of 4 to 7 entries
        return stencil_csr(3, 13, cell_coefficients(3, 13, 0.8))
    if name == "diffusion2d_37":      # n = 1369
        return stencil_csr(2, 37, cell_coefficients(2, 37, 0.5))
    if name == "long_range":
        return _long_range()
    raise KeyError(name)


KP = [(16, "block", 0), (16, "hybrid", 4), (32, "block", 0), (64, "hybrid", 8), (48, "hybrid", 16)]


def _pair(A, k, variant, p, sigma=1, precision="fp64"):
    P = _P()
    a = P.BCG(*csr_to_dev(A), k=k, subalgebra=variant, p=p)
    b = P.BCG(*csr_to_dev(A), k=k, subalgebra=variant, p=p)
    if precision != "fp64":
        a.set_precision(precision)
        b.set_precision(precision)
    b.set_sell(True, sigma)
    return a, b


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
@pytest.mark.parametrize("name", ["diffusion3d_13", "diffusion2d_37", "long_range"])
@pytest.mark.parametrize("k,variant,p", KP)
def test_sell_sigma1_bitwise_equals_csr(precision, name, k, variant, p):
    log(f"sell sigma=1 {precision} {name} k={k} {variant} p={p}")
    A = _matrix(name)
    B = dev(rhs(A.shape[0], k, "normal", seed=500 + k))
    csr, sell = _pair(A, k, variant, p, 1, precision)
    if precision == "fp64":
        Xc, ic = csr.solve(B, tol=0.0, maxit=8)
        Xs, is_ = sell.solve(B, tol=0.0, maxit=8)
        assert ic["iterations"] == is_["iterations"] == 8
    else:
        Xc, ic = csr.solve(B, tol=1e-9)
        Xs, is_ = sell.solve(B, tol=1e-9)
        assert ic["status"] == is_["status"] == oracle.OK
        assert ic["iterations"] == is_["iterations"]
        assert ic["outer_iterations"] == is_["outer_iterations"]
    assert torch.equal(Xc, Xs)


# every width and group instantiation of the two products: K = 64..128, groups
# of 16, 32 and 64 columns, the global and parallel subalgebras
KP_WIDE = [(64, "block", 0), (80, "hybrid", 8), (96, "parallel", 1), (112, "hybrid", 16), (128, "hybrid", 16),
           (128, "global", 1)]


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
@pytest.mark.parametrize("k,variant,p", KP_WIDE)
def test_sell_sigma1_bitwise_wide_blocks(precision, k, variant, p):
    log(f"sell sigma=1 wide {precision} k={k} {variant} p={p}")
    A = _matrix("long_range")
    B = dev(rhs(A.shape[0], k, "normal", seed=700 + k))
    csr, sell = _pair(A, k, variant, p, 1, precision)
    if precision == "fp64":
        Xc, ic = csr.solve(B, tol=0.0, maxit=6)
        Xs, is_ = sell.solve(B, tol=0.0, maxit=6)
    else:
        Xc, ic = csr.solve(B, tol=1e-8)
        Xs, is_ = sell.solve(B, tol=1e-8)
        assert ic["status"] == is_["status"] == oracle.OK
    assert ic["iterations"] == is_["iterations"]
    assert torch.equal(Xc, Xs)
    if precision == "fp64":
        Xo, _ = oracle_solve(A, host(B), variant, p, tol=0.0, maxit=6)
        assert rel(host(Xs), Xo) <= FIXED_TOL


@pytest.mark.parametrize("sigma", [16, 64, 4096])
@pytest.mark.parametrize("name", ["diffusion3d_13", "long_range"])
@pytest.mark.parametrize("k,variant,p", [(16, "block", 0), (32, "hybrid", 8), (64, "hybrid", 8), (48, "global", 16)])
def test_sell_sorted_fixed_iterations(sigma, name, k, variant, p):
    log(f"sell sigma={sigma} {name} k={k} {variant} p={p}")
    A = _matrix(name)
    B = rhs(A.shape[0], k, "normal", seed=600 + k)
    Xo, io = oracle_solve(A, B, variant, p, tol=0.0, maxit=8)
    s = _P().BCG(*csr_to_dev(A), k=k, subalgebra=variant, p=p)
    s.set_sell(True, sigma)
    Xg, ig = s.solve(dev(B), tol=0.0, maxit=8)
    assert ig["iterations"] == io["iterations"] == 8
    assert rel(host(Xg), Xo) <= FIXED_TOL


@pytest.mark.parametrize("variant,p", [("block", 0), ("hybrid", 4)])
def test_sell_sorted_refine_reaches_fp64_accuracy(variant, p):
    log(f"sell refine sigma=64 {variant} p={p}")
    A = _long_range()
    B = rhs(A.shape[0], 16, "normal", seed=7)
    s = _P().BCG(*csr_to_dev(A), k=16, subalgebra=variant, p=p)
    s.set_precision("fp32_refine")
    s.set_sell(True, 64)
    tol = 1e-10
    X, info = s.solve(dev(B), tol=tol)
    Xh = host(X)
    assert info["status"] == oracle.OK, info
    R = B - A @ Xh
    assert float(np.max(np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0))) <= tol
    Xref = np.column_stack([spla.spsolve(A.tocsc(), B[:, j]) for j in range(B.shape[1])])
    assert rel(Xh, Xref) <= 1e-7


def test_sell_follows_values_schedule_and_jacobi():
    """The SELL copy takes the handle's current values at every solve and is
    rebuilt when the row schedule changes."""
    log("sell values / schedule / jacobi")
    P = _P()
    A = _matrix("diffusion3d_13")
    A2 = stencil_csr(3, 13, cell_coefficients(3, 13, 1.2))
    assert np.array_equal(A.indptr, A2.indptr) and np.array_equal(A.indices, A2.indices)
    k = 16
    B = dev(rhs(A.shape[0], k, "normal", seed=11))
    csr, sell = _pair(A, k, "block", 0, 1)
    v2 = dev(A2.data.astype(np.float64))
    for s in (csr, sell):
        s.update_values(v2)
    Xc, _ = csr.solve(B, tol=0.0, maxit=8)
    Xs, _ = sell.solve(B, tol=0.0, maxit=8)
    assert torch.equal(Xc, Xs)
    Xo, _ = oracle_solve(A2, host(B), "block", 0, tol=0.0, maxit=8)
    assert rel(host(Xs), Xo) <= FIXED_TOL
    # a random row schedule: the copy follows it
    order = torch.from_numpy(np.random.default_rng(3).permutation(A.shape[0]).astype(np.int32)).cuda()
    for s in (csr, sell):
        s.set_row_schedule(order)
    Xc, _ = csr.solve(B, tol=0.0, maxit=8)
    Xs, _ = sell.solve(B, tol=0.0, maxit=8)
    assert torch.equal(Xc, Xs)
    # Jacobi scaling: the copy takes the scaled values
    for s in (csr, sell):
        s.set_preconditioner("jacobi")
    Xc, ic = csr.solve(B, tol=1e-8)
    Xs, is_ = sell.solve(B, tol=1e-8)
    assert ic["status"] == is_["status"] == oracle.OK
    assert ic["iterations"] == is_["iterations"]
    assert torch.equal(Xc, Xs)
    # back to the natural order and CSR
    for s in (csr, sell):
        s.set_row_schedule(None)
        s.set_preconditioner("none")
    sell.set_sell(False)
    Xc, _ = csr.solve(B, tol=0.0, maxit=5)
    Xs, _ = sell.solve(B, tol=0.0, maxit=5)
    assert torch.equal(Xc, Xs)


def test_sell_follows_rejected_schedule():
    """A rejected row schedule leaves the natural order, for the SELL copy too."""
    A = _matrix("diffusion2d_37")
    B = dev(rhs(A.shape[0], 16, "normal", seed=12))
    csr, sell = _pair(A, 16, "block", 0, 1)
    order = torch.from_numpy(np.random.default_rng(4).permutation(A.shape[0]).astype(np.int32)).cuda()
    sell.set_row_schedule(order)
    bad = order.clone()
    bad[5] = A.shape[0]
    with pytest.raises(_P().BCGError):
        sell.set_row_schedule(bad)
    Xc, _ = csr.solve(B, tol=0.0, maxit=6)
    Xs, _ = sell.solve(B, tol=0.0, maxit=6)
    assert torch.equal(Xc, Xs)


def test_sell_rejects_bad_sigma():
    P = _P()
    A = _matrix("diffusion2d_37")
    s = P.BCG(*csr_to_dev(A), k=16, subalgebra="block", p=0)
    for bad in (0, -16, 17, 40):
        with pytest.raises(P.BCGError) as e:
            s.set_sell(True, bad)
        assert e.value.status == -1
    B = rhs(A.shape[0], 16, "normal", seed=5)
    Xo, _ = oracle_solve(A, B, "block", 0, tol=0.0, maxit=4)
    Xg, _ = s.solve(dev(B), tol=0.0, maxit=4)     # still the CSR product
    assert rel(host(Xg), Xo) <= FIXED_TOL


@pytest.mark.parametrize("k,variant,p", [(16, "block", 0), (32, "hybrid", 16), (64, "hybrid", 8)])
def test_sell_wide_offsets_bitwise(monkeypatch, k, variant, p):
    """64-bit lane offsets (forced) give the same bits as 32-bit ones."""
    monkeypatch.setenv("BCG_WIDE_OFFSETS", "1")
    log(f"sell wide offsets k={k} {variant} p={p}")
    A = _matrix("long_range")
    B = dev(rhs(A.shape[0], k, "normal", seed=900 + k))
    csr, sell = _pair(A, k, variant, p, 1)
    Xc, _ = csr.solve(B, tol=0.0, maxit=6)
    Xs, _ = sell.solve(B, tol=0.0, maxit=6)
    assert torch.equal(Xc, Xs)


def test_sell_k8_uses_csr_path():
    """k = 8 has no matrix-core product: the SELL copy is kept but unused."""
    A = _matrix("long_range")
    B = dev(rhs(A.shape[0], 8, "normal", seed=8))
    csr, sell = _pair(A, 8, "hybrid", 2, 32)
    Xc, _ = csr.solve(B, tol=0.0, maxit=6)
    Xs, _ = sell.solve(B, tol=0.0, maxit=6)
    assert torch.equal(Xc, Xs)


def test_full_size_poisson3d_128_k16_sell():
    """128^3 Poisson, k = 16, block, tiled row order, FP32 + refinement to
    1e-8: SELL with sigma = 1 is bitwise the CSR solve; sorted (sigma = 64)
    it converges with the same true-residual bound."""
    P = _P()
    w = WORKLOADS["poisson3d_128_k16"]
    log("full size 128^3 k=16 sell")
    rp, ci, va = P.stencil(w.dim, w.N)
    B = torch.from_numpy(rhs_for(w)).cuda()
    order = P.stencil_schedule(w.dim, w.N, 32)
    X = {}
    for mode in ("csr", "sell1", "sell64"):
        s = P.BCG(rp, ci, va, k=w.k, subalgebra="block", p=0)
        s.set_row_schedule(order)
        s.set_precision("fp32_refine")
        if mode != "csr":
            s.set_sell(True, 1 if mode == "sell1" else 64)
        X[mode], info = s.solve(B, tol=1e-8)
        log(f"{mode}: {info['iterations']} iterations, true {info['true_rel_res']:.3e}")
        assert info["status"] == oracle.OK
        assert info["true_rel_res"] <= 1e-8
        del s
    assert torch.equal(X["csr"], X["sell1"])
    assert rel(host(X["sell64"]), host(X["csr"])) <= 1e-6
