"""GPU (HIP) path vs the FP64 oracle, column by column, through the C ABI.

Tolerances (FP64): the two sides run the same recurrences with different
summation orders, so they differ by rounding amplified along the iteration.
Errors are the largest per-column relative error (``rel``), so that one bad
column cannot hide in the norm of the others.
Fixed-iteration iterates must agree to 1e-10 in every column; converged
solves (tol 1e-8) must stop at the same iteration (a tie at the stop boundary
may shift it by one) and agree to 1e-8 relative, the accuracy the method
itself delivers. Integer and CSR work is compared bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle.bcg import solve as oracle_solve
from oracle.grad import kappa_vjp as oracle_kappa_vjp, sampled_outer as oracle_sampled_outer
from oracle.stencil import stencil_csr
from tests.gpu_helpers import csr_to_dev, dev, host, log, rel
from workload import WORKLOADS, cell_coefficients, long_range_pairs, rhs, rhs_for

pytestmark = pytest.mark.gpu

FIXED_TOL = 1e-10
CONVERGED_TOL = 1e-8


def _lib():
    import paper_1912_11930_amd as P
    return P


def _solver(A, k, variant, p):
    P = _lib()
    return P.BCG(*csr_to_dev(A), k=k, subalgebra=variant, p=p)


# ----------------------------------------------------------------- CSR (a0)
@pytest.mark.parametrize("dim,N,sigma", [
    (2, 1, 0.0), (2, 2, 1.0), (2, 3, 0.5), (3, 1, 0.0), (3, 2, 1.0), (3, 5, 1.0),
    (2, 32, 0.0), (2, 512, 0.5), (3, 128, 0.0), (3, 192, 1.0),
])
def test_stencil_bitexact(dim, N, sigma):
    log(f"stencil dim={dim} N={N} sigma={sigma}")
    P = _lib()
    kappa = None if sigma == 0 else cell_coefficients(dim, N, sigma)
    A = stencil_csr(dim, N, kappa)
    rp, ci, va = P.stencil(dim, N, None if kappa is None else dev(kappa))
    assert np.array_equal(host(rp), A.indptr)
    assert np.array_equal(host(ci), A.indices)
    assert np.array_equal(host(va).view(np.uint64), A.data.view(np.uint64))


# ------------------------------------------------ fixed-iteration iterates
CASES_SMALL = [("block", 0), ("global", 1), ("global", 2), ("parallel", 1), ("hybrid", 2), ("hybrid", 4)]


@pytest.mark.parametrize("variant,p", CASES_SMALL)
@pytest.mark.parametrize("m", [1, 10, 50])
def test_fixed_iterations_poisson2d_32(variant, p, m):
    w = WORKLOADS["poisson2d_32_k8"]
    log(f"fixed {variant} p={p} m={m}")
    A = stencil_csr(w.dim, w.N)
    B = rhs_for(w)
    Xo, io = oracle_solve(A, B, variant, p, tol=0.0, maxit=m)
    s = _solver(A, w.k, variant, p)
    Xg, ig = s.solve(dev(B), tol=0.0, maxit=m)
    assert ig["iterations"] == io["iterations"] == m
    assert ig["status"] == io["status"] == oracle.NOT_CONVERGED
    assert rel(host(Xg), Xo) <= FIXED_TOL
    np.testing.assert_allclose(ig["ratios"], io["ratios"], rtol=1e-8, atol=0)


# ragged tails and tile geometry: n not a multiple of the rows per tile, odd p
# (no register blocking), products too large for the fused path
KP_CASES = [
    (1, "block", 0), (3, "hybrid", 3), (5, "parallel", 1), (6, "global", 3), (12, "hybrid", 3),
    (12, "global", 4), (24, "hybrid", 8), (32, "block", 0), (40, "hybrid", 5), (64, "hybrid", 8),
    (64, "global", 16), (96, "hybrid", 48), (128, "block", 0), (128, "hybrid", 16), (128, "global", 1),
    (256, "hybrid", 16),
]


@pytest.mark.parametrize("k,variant,p", KP_CASES)
def test_fixed_iterations_k_p_grid(k, variant, p):
    log(f"k={k} {variant} p={p}")
    N = 37 if k <= 64 else 23
    A = stencil_csr(2, N, cell_coefficients(2, N, 0.7))
    B = rhs(A.shape[0], k, "normal", seed=k)
    m = 6
    Xo, io = oracle_solve(A, B, variant, p, tol=0.0, maxit=m)
    s = _solver(A, k, variant, p)
    Xg, ig = s.solve(dev(B), tol=0.0, maxit=m)
    assert ig["iterations"] == io["iterations"]
    assert ig["status"] == io["status"]
    assert rel(host(Xg), Xo) <= FIXED_TOL


@pytest.mark.parametrize("gw", ["1", "2", "vec", "mfma"])
@pytest.mark.parametrize("k,variant,p", [(32, "hybrid", 16), (64, "hybrid", 4), (128, "hybrid", 16),
                                         (128, "global", 1), (32, "parallel", 1)])
def test_update_groups_per_wave(monkeypatch, k, variant, p, gw):
    # the matrix-core update passes with one or two column groups per wave
    # (two: both groups' rows move as whole lines), or the k-specialised vector
    # update passes beside the matrix-core sparse product; FP64 iterates
    # against the oracle, ragged row count
    if gw == "vec":
        monkeypatch.setenv("BCG_UPDATE_VEC64", "3")
    elif gw == "mfma":
        monkeypatch.setenv("BCG_UPDATE_VEC64", "0")
    else:
        monkeypatch.setenv("BCG_UPDATE_GW", gw)
    log(f"groups per wave {gw}: k={k} {variant} p={p}")
    N = 29
    A = stencil_csr(2, N, cell_coefficients(2, N, 0.7))
    B = rhs(A.shape[0], k, "normal", seed=70 + k)
    Xo, io = oracle_solve(A, B, variant, p, tol=0.0, maxit=5)
    s = _solver(A, k, variant, p)
    Xg, ig = s.solve(dev(B), tol=0.0, maxit=5)
    assert ig["iterations"] == io["iterations"] == 5
    assert rel(host(Xg), Xo) <= FIXED_TOL


# ---------------------------------------------------- converged solutions
def _converged_case(A, B, variant, p, tol=1e-8, maxit=5000):
    Xo, io = oracle_solve(A, B, variant, p, tol=tol, maxit=maxit)
    s = _solver(A, B.shape[1], variant, p)
    Xg, ig = s.solve(dev(B), tol=tol, maxit=maxit)
    assert io["status"] == oracle.OK
    assert ig["status"] == oracle.OK, ig
    if ig["iterations"] != io["iterations"]:
        # a tie at the stop boundary: both sides must agree at the oracle's count
        assert abs(ig["iterations"] - io["iterations"]) == 1
        assert min(max(ig["ratios"]), max(io["ratios"])) <= tol * (1 + 1e-6)
        Xg2, _ = s.solve(dev(B), tol=0.0, maxit=io["iterations"])
        Xg = Xg2
    assert rel(host(Xg), Xo) <= CONVERGED_TOL
    assert ig["true_rel_res"] <= 100 * tol
    return ig, io


@pytest.mark.parametrize("variant,p", [("block", 0), ("global", 1), ("parallel", 1), ("hybrid", 2), ("hybrid", 4)])
def test_converged_poisson2d_32(variant, p):
    w = WORKLOADS["poisson2d_32_k8"]
    log(f"converged {variant} p={p}")
    _converged_case(stencil_csr(w.dim, w.N), rhs_for(w), variant, p, tol=w.tol)


@pytest.mark.parametrize("variant,p", [("block", 0), ("global", 4), ("parallel", 1), ("hybrid", 4)])
def test_converged_diffusion_ragged(variant, p):
    log(f"converged diffusion {variant} p={p}")
    A = stencil_csr(3, 13, cell_coefficients(3, 13, 1.0))
    B = rhs(A.shape[0], 16, "normal")
    _converged_case(A, B, variant, p)


# ----------------------------------------------------------- status codes
def test_status_codes_match_oracle():
    P = _lib()
    A = stencil_csr(2, 12)
    B = rhs(A.shape[0], 4, "uniform")
    s = _solver(A, 4, "block", 0)
    # NaN in B
    Bn = B.copy(); Bn[5, 2] = np.nan
    with pytest.raises(P.BCGError) as e:
        s.solve(dev(Bn))
    assert e.value.status == oracle.EINVAL
    # zero column in a non-diagonal subalgebra
    Bz = B.copy(); Bz[:, 1] = 0.0
    with pytest.raises(P.BCGError):
        s.solve(dev(Bz))
    # ... but fine for parallel, the zero lane stays zero
    sp_ = _solver(A, 4, "parallel", 1)
    Xz, iz = sp_.solve(dev(Bz), tol=1e-10, maxit=500)
    Xo, io = oracle_solve(A, Bz, "parallel", 1, tol=1e-10, maxit=500)
    assert iz["status"] == io["status"] == oracle.OK
    assert np.all(host(Xz)[:, 1] == 0.0)
    assert rel(host(Xz), Xo) <= CONVERGED_TOL
    # all-zero B: immediate success
    X0, i0 = s.solve(dev(np.zeros_like(B)))
    assert i0["status"] == oracle.OK and i0["iterations"] == 0
    # not converged
    _, inc = s.solve(dev(B), tol=1e-14, maxit=3)
    assert inc["status"] == oracle.NOT_CONVERGED and inc["iterations"] == 3
    # breakdown: negative definite operator, X stays at X0
    An = A.copy(); An.setdiag(-A.diagonal())
    sn = _solver(An, 4, "block", 0)
    Xb, ib = sn.solve(dev(B))
    _, ob = oracle_solve(An, B, "block", 0)
    assert ib["status"] == ob["status"] == oracle.EBREAKDOWN
    assert ib["iterations"] == ob["iterations"] == 0
    assert np.all(host(Xb) == 0.0)
    # breakdown: rank-deficient block [b, b]
    Bd = np.stack([B[:, 0], B[:, 0]], axis=1)
    sd = _solver(A, 2, "block", 0)
    _, idd = sd.solve(dev(Bd))
    assert idd["status"] == oracle.EBREAKDOWN == oracle_solve(A, Bd, "block", 0)[1]["status"]
    # invalid arguments
    with pytest.raises(P.BCGError):
        _solver(A, 4, "hybrid", 3)
    with pytest.raises(P.BCGError):
        s.solve(dev(B), tol=-1.0)


def test_repeated_solves_bitwise_identical():
    A = stencil_csr(3, 17, cell_coefficients(3, 17, 1.0))
    B = rhs(A.shape[0], 16, "normal")
    s = _solver(A, 16, "hybrid", 4)
    X1, i1 = s.solve(dev(B), tol=1e-8)
    X2, i2 = s.solve(dev(B), tol=1e-8)
    assert i1["iterations"] == i2["iterations"]
    assert np.array_equal(host(X1).view(np.uint64), host(X2).view(np.uint64))


def test_warm_start_and_x0():
    A = stencil_csr(2, 20, cell_coefficients(2, 20, 0.5))
    B = rhs(A.shape[0], 8, "uniform")
    X0 = 0.3 * rhs(A.shape[0], 8, "normal", seed=9)
    Xo, io = oracle_solve(A, B, "hybrid", 4, tol=0.0, maxit=7, X0=X0)
    s = _solver(A, 8, "hybrid", 4)
    Xg, ig = s.solve(dev(B), X=dev(X0), tol=0.0, maxit=7)
    assert rel(host(Xg), Xo) <= FIXED_TOL


# --------------------------------------------------- gradient kernels (a10)
def test_sampled_outer_matches_oracle():
    A = stencil_csr(3, 9, cell_coefficients(3, 9, 1.0))
    k = 12
    Y = rhs(A.shape[0], k, "normal", seed=4)
    X = rhs(A.shape[0], k, "normal", seed=5)
    s = _solver(A, k, "block", 0)
    out = host(s.csr_outer(dev(Y), dev(X), -1.0))
    np.testing.assert_allclose(out, oracle_sampled_outer(A, Y, X, -1.0), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("dim,N", [(2, 9), (3, 6), (2, 512)])
def test_kappa_vjp_matches_oracle(dim, N):
    P = _lib()
    kappa = cell_coefficients(dim, N, 0.5)
    A = stencil_csr(dim, N, kappa)
    dv = np.random.default_rng(1).standard_normal(A.nnz)
    g = host(P.stencil_kappa_vjp(dim, N, dev(kappa), dev(dv)))
    np.testing.assert_allclose(g, oracle_kappa_vjp(dim, N, kappa, A, dv), rtol=1e-12, atol=1e-12)


# --------------------------------------------- k-specialised row kernels
FAST_CASES = [(k, v, p) for k in (8, 16, 32, 64, 128) for (v, p) in
              [("parallel", 1), ("hybrid", 2), ("hybrid", 4), ("hybrid", 8), ("hybrid", 16), ("global", 4)]
              if p <= k] + [(8, "block", 0), (16, "block", 0), (16, "global", 1), (128, "global", 8)]


@pytest.mark.parametrize("path", ["default", "no_mfma"])
@pytest.mark.parametrize("k,variant,p", FAST_CASES)
def test_fast_path_fixed_iterations(monkeypatch, k, variant, p, path):
    # default: matrix-core kernels where k is a multiple of 16; no_mfma: the
    # k-specialised vector kernels for the same shapes
    if path == "no_mfma":
        monkeypatch.setenv("BCG_NO_MFMA", "1")
    log(f"fast k={k} {variant} p={p} {path}")
    N = 41 if k <= 32 else 19                      # ragged: n not a multiple of the rows per step
    A = stencil_csr(2, N, cell_coefficients(2, N, 0.8))
    B = rhs(A.shape[0], k, "normal", seed=100 + k)
    m = 8
    Xo, io = oracle_solve(A, B, variant, p, tol=0.0, maxit=m)
    s = _solver(A, k, variant, p)
    Xg, ig = s.solve(dev(B), tol=0.0, maxit=m)
    assert ig["iterations"] == io["iterations"] == m
    assert rel(host(Xg), Xo) <= FIXED_TOL


@pytest.mark.parametrize("k,variant,p", [(16, "block", 0), (32, "block", 0), (32, "hybrid", 16), (64, "hybrid", 8),
                                         (128, "global", 4)])
def test_wide_offsets_fixed_iterations(monkeypatch, k, variant, p):
    # the sparse products' 64-bit offset form, which systems whose operands
    # exceed 4 GiB take (forced here on a small one)
    monkeypatch.setenv("BCG_WIDE_OFFSETS", "1")
    log(f"wide offsets k={k} {variant} p={p}")
    N = 41 if k <= 32 else 19
    A = stencil_csr(2, N, cell_coefficients(2, N, 0.8))
    B = rhs(A.shape[0], k, "normal", seed=300 + k)
    m = 8
    Xo, io = oracle_solve(A, B, variant, p, tol=0.0, maxit=m)
    s = _solver(A, k, variant, p)
    Xg, ig = s.solve(dev(B), tol=0.0, maxit=m)
    assert ig["iterations"] == io["iterations"] == m
    assert rel(host(Xg), Xo) <= FIXED_TOL


@pytest.mark.parametrize("k,variant,p", [(8, "block", 0), (16, "hybrid", 4), (64, "hybrid", 8), (128, "global", 1)])
def test_generic_path_forced(monkeypatch, k, variant, p):
    # the generic LDS-tiled kernels stay correct for shapes the fast path also covers
    monkeypatch.setenv("BCG_GENERIC_ONLY", "1")
    log(f"generic k={k} {variant} p={p}")
    A = stencil_csr(2, 29, cell_coefficients(2, 29, 0.8))
    B = rhs(A.shape[0], k, "normal", seed=7)
    Xo, io = oracle_solve(A, B, variant, p, tol=0.0, maxit=8)
    s = _solver(A, k, variant, p)
    Xg, ig = s.solve(dev(B), tol=0.0, maxit=8)
    assert rel(host(Xg), Xo) <= FIXED_TOL


# ------------------------------------------------ matrix-core row kernels
# group widths 16/32/64, column-group counts 1..8 (3, 5, 7: waves per XCD not
# a multiple of the group count), ragged row tails, grids below 8 workgroups
MFMA_CASES = [
    (32, "block", 0, 2, 41), (64, "block", 0, 2, 23), (64, "hybrid", 32, 2, 23), (64, "global", 32, 2, 23),
    (96, "hybrid", 32, 2, 19), (128, "hybrid", 32, 2, 17), (128, "global", 32, 2, 17), (64, "global", 64, 2, 19),
    (48, "hybrid", 16, 2, 29), (48, "parallel", 1, 3, 7), (80, "hybrid", 8, 2, 21), (112, "global", 16, 2, 13),
    (112, "hybrid", 16, 2, 3), (128, "parallel", 1, 2, 10), (128, "hybrid", 2, 3, 5), (16, "block", 0, 2, 1),
    (16, "hybrid", 4, 2, 3), (32, "global", 2, 3, 4),
]


@pytest.mark.parametrize("k,variant,p,dim,N", MFMA_CASES)
def test_mfma_path_fixed_iterations(k, variant, p, dim, N):
    log(f"mfma k={k} {variant} p={p} dim={dim} N={N}")
    A = stencil_csr(dim, N, cell_coefficients(dim, N, 0.8))
    B = rhs(A.shape[0], k, "normal", seed=300 + k)
    m = 6 if A.shape[0] > 1 else 1
    Xo, io = oracle_solve(A, B, variant, p, tol=0.0, maxit=m)
    s = _solver(A, k, variant, p)
    Xg, ig = s.solve(dev(B), tol=0.0, maxit=m)
    assert ig["iterations"] == io["iterations"]
    assert ig["status"] == io["status"]
    assert rel(host(Xg), Xo) <= FIXED_TOL


@pytest.mark.parametrize("variant,p", [("block", 0), ("hybrid", 32)])
def test_mfma_path_converged_k64(variant, p):
    log(f"mfma converged k=64 {variant} p={p}")
    A = stencil_csr(3, 11, cell_coefficients(3, 11, 1.0))
    B = rhs(A.shape[0], 64, "normal", seed=9)
    _converged_case(A, B, variant, p)


def test_misaligned_x_uses_generic_path():
    # a solution view that is not 16-byte aligned is still solved correctly
    A = stencil_csr(2, 17)
    k = 8
    B = rhs(A.shape[0], k, "uniform")
    Xo, _ = oracle_solve(A, B, "hybrid", 4, tol=0.0, maxit=6)
    buf = torch.zeros(A.shape[0] * k + 1, dtype=torch.float64, device="cuda")
    Xv = buf[1:].view(A.shape[0], k)
    s = _solver(A, k, "hybrid", 4)
    s.solve(dev(B), X=Xv, tol=0.0, maxit=6)
    assert rel(host(Xv), Xo) <= FIXED_TOL


def test_misaligned_x_k16():
    # k a multiple of 16 (matrix-core shapes) with an X view that is only 8-byte aligned
    A = stencil_csr(2, 17)
    k = 16
    B = rhs(A.shape[0], k, "uniform")
    Xo, _ = oracle_solve(A, B, "hybrid", 8, tol=0.0, maxit=6)
    buf = torch.zeros(A.shape[0] * k + 1, dtype=torch.float64, device="cuda")
    Xv = buf[1:].view(A.shape[0], k)
    s = _solver(A, k, "hybrid", 8)
    s.solve(dev(B), X=Xv, tol=0.0, maxit=6)
    assert rel(host(Xv), Xo) <= FIXED_TOL


# ------------------------------------------------ sparse-product row order
def _tiled_order(N, T):
    parts = []
    for ty in range(0, N, T):
        for tx in range(0, N, T):
            z, y, x = np.meshgrid(np.arange(N), np.arange(ty, min(N, ty + T)), np.arange(tx, min(N, tx + T)),
                                  indexing="ij")
            parts.append((x + N * y + N * N * z).ravel())
    return np.concatenate(parts).astype(np.int32)


def _brick_order(N, tile, brick):
    """Definition of the brick schedule: key (tile column (ty, tx), tile z,
    brick z, y, x inside the tile, cell z, y, x inside the brick)."""
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    x, y, z = x.ravel(), y.ravel(), z.ravel()
    tx, ty, tz = tile
    bx, by, bz = brick
    tile_id = ((y // ty) * (N // tx) + x // tx) * (N // tz) + z // tz
    lx, ly, lz = x % tx, y % ty, z % tz
    brick_id = ((lz // bz) * (ty // by) + ly // by) * (tx // bx) + lx // bx
    cell = ((lz % bz) * by + ly % by) * bx + lx % bx
    key = (tile_id * (tx * ty * tz) + brick_id * (bx * by * bz) + cell).astype(np.int64)
    return np.argsort(key, kind="stable").astype(np.int32)


@pytest.mark.parametrize("N,tile,brick", [(8, (4, 4, 2), (2, 2, 2)), (12, (6, 4, 3), (3, 2, 1)),
                                          (32, (16, 32, 2), (4, 2, 2)), (16, (16, 16, 16), (16, 1, 1))])
def test_brick_schedule_matches_definition(N, tile, brick):
    P = _lib()
    got = host(P.stencil_brick_schedule(N, tile, brick))
    assert np.array_equal(got, _brick_order(N, tile, brick))
    assert np.array_equal(np.sort(got), np.arange(N ** 3))


@pytest.mark.parametrize("N,T", [(5, 2), (13, 4), (128, 32)])
def test_stencil_schedule_matches_definition(N, T):
    P = _lib()
    got = host(P.stencil_schedule(3, N, T))
    assert np.array_equal(got, _tiled_order(N, T))
    assert np.array_equal(host(P.stencil_schedule(2, N, T)), np.arange(N * N))


@pytest.mark.parametrize("k,variant,p", [(16, "block", 0), (8, "hybrid", 4), (64, "hybrid", 8), (128, "global", 1),
                                         (12, "hybrid", 3)])
def test_row_schedule_random_and_tiled(k, variant, p):
    # any row order of the sparse product gives the same iterates (up to the
    # rounding order of the partial products)
    P = _lib()
    N = 11 if k <= 64 else 7
    A = stencil_csr(3, N, cell_coefficients(3, N, 0.6))
    B = rhs(A.shape[0], k, "normal", seed=21)
    Xo, _ = oracle_solve(A, B, variant, p, tol=0.0, maxit=7)
    bricks = _brick_order(N, (N, 1, 1), (1, 1, 1)) if N % 2 else _brick_order(N, (4, 2, 2), (2, 2, 1))
    for order in (np.random.default_rng(5).permutation(A.shape[0]).astype(np.int32), _tiled_order(N, 4), bricks):
        s = _solver(A, k, variant, p)
        s.set_row_schedule(dev(order))
        Xg, ig = s.solve(dev(B), tol=0.0, maxit=7)
        assert rel(host(Xg), Xo) <= FIXED_TOL
        s.set_row_schedule(None)
        Xn, _ = s.solve(dev(B), tol=0.0, maxit=7)
        assert rel(host(Xn), Xo) <= FIXED_TOL


@pytest.mark.parametrize("fault", ["out_of_range", "negative", "duplicate"])
def test_row_schedule_rejects_non_permutation(fault):
    P = _lib()
    A = stencil_csr(2, 9)
    s = _solver(A, 8, "block", 0)
    bad = np.arange(A.shape[0], dtype=np.int32)[::-1].copy()
    if fault == "out_of_range":
        bad[3] = A.shape[0]
    elif fault == "negative":
        bad[3] = -1
    else:
        bad[7] = bad[40]      # row bad[7] is never computed, bad[40] twice
    with pytest.raises(P.BCGError) as e:
        s.set_row_schedule(dev(bad))
    assert e.value.status == oracle.EINVAL
    B = rhs(A.shape[0], 8, "uniform")
    Xo, _ = oracle_solve(A, B, "block", 0, tol=0.0, maxit=5)
    Xg, _ = s.solve(dev(B), tol=0.0, maxit=5)      # still the natural order
    assert rel(host(Xg), Xo) <= FIXED_TOL


@pytest.mark.parametrize("fault", ["rowptr0", "decreasing", "rowptr_n", "col_high", "col_negative"])
def test_create_rejects_malformed_csr(fault):
    # the device check at create returns EINVAL before any kernel follows a
    # row range; the arrays stay within their allocations in every case
    P = _lib()
    A = stencil_csr(2, 9)
    rp, ci, va = A.indptr.astype(np.int32).copy(), A.indices.astype(np.int32).copy(), A.data.copy()
    if fault == "rowptr0":
        rp[0] = 1
    elif fault == "decreasing":
        rp[10] = rp[9] - 1
    elif fault == "rowptr_n":
        rp[-1] = rp[-1] - 1
    elif fault == "col_high":
        ci[17] = A.shape[0]
    else:
        ci[17] = -3
    with pytest.raises(P.BCGError) as e:
        P.BCG(dev(rp), dev(ci), dev(va), k=8, subalgebra="block")
    assert e.value.status == oracle.EINVAL
    # the well-formed matrix still builds and solves
    s = _solver(A, 8, "block", 0)
    B = rhs(A.shape[0], 8, "uniform")
    Xg, _ = s.solve(dev(B), tol=0.0, maxit=3)
    Xo, _ = oracle_solve(A, B, "block", 0, tol=0.0, maxit=3)
    assert rel(host(Xg), Xo) <= FIXED_TOL


# ------------------------------------------- rows longer than 8 entries
def _long_range_csr(N=40, per_row=6):
    """2D N^2 diffusion plus symmetric couplings at random far positions
    (about 2 per_row per row, so rows hold 8 to ~30 entries, most of them far
    from the diagonal), the diagonal raised by the couplings' row sums
    (diagonally dominant, SPD)."""
    import scipy.sparse as sp
    A = stencil_csr(2, N, cell_coefficients(2, N, 0.5))
    n = A.shape[0]
    i, j = long_range_pairs(n, per_row)
    C = sp.coo_matrix((np.full(i.size, -0.05), (i, j)), shape=(n, n)).tocsr()
    C = C + C.T
    d = np.asarray(abs(C).sum(axis=1)).ravel()
    return (A + C + sp.diags(d)).tocsr()


@pytest.mark.parametrize("path", ["default", "no_mfma", "generic"])
@pytest.mark.parametrize("k,variant,p", [(16, "block", 0), (16, "hybrid", 4), (8, "hybrid", 2), (32, "hybrid", 32)])
def test_long_rows_fixed_iterations(monkeypatch, path, k, variant, p):
    """General CSR: rows of 8 to ~30 entries at scattered columns, so the
    sparse products take more than one 8-entry batch per row. FP64 iterates
    against the oracle after 8 iterations, on every row-kernel path."""
    if path == "no_mfma":
        monkeypatch.setenv("BCG_NO_MFMA", "1")
    elif path == "generic":
        monkeypatch.setenv("BCG_GENERIC_ONLY", "1")
    log(f"long rows k={k} {variant} p={p} {path}")
    A = _long_range_csr()
    nnz = np.diff(A.indptr)
    assert nnz.max() > 16 and (nnz > 8).mean() > 0.9
    B = rhs(A.shape[0], k, "normal", seed=300 + k)
    Xo, io = oracle_solve(A, B, variant, p, tol=0.0, maxit=8)
    s = _solver(A, k, variant, p)
    Xg, ig = s.solve(dev(B), tol=0.0, maxit=8)
    assert ig["iterations"] == io["iterations"] == 8
    assert rel(host(Xg), Xo) <= FIXED_TOL


# ---------------------------------------- stop rule at the iteration cap
@pytest.mark.parametrize("poll", [None, "1"])
@pytest.mark.parametrize("k,variant,p", [(8, "block", 0), (8, "hybrid", 2), (8, "parallel", 1), (6, "hybrid", 3),
                                         (12, "hybrid", 12)])
def test_stop_on_last_allowed_iteration(monkeypatch, poll, k, variant, p):
    """The stop rule is tested before the iteration cap (line 12 reading): a
    solve that converges on exactly its last allowed iteration succeeds with
    that count, one allowed iteration fewer is NOT_CONVERGED. With a status
    poll after every iteration (BCG_POLL_EVERY=1) the host sees the final
    iteration before any later launch runs. Register (p = 2, 8), Gauss-Jordan
    (p = 3, 12) and parallel (p = 1) small steps; results against the oracle."""
    if poll:
        monkeypatch.setenv("BCG_POLL_EVERY", poll)
    log(f"stop at cap k={k} {variant} p={p} poll={poll}")
    A = stencil_csr(2, 23, cell_coefficients(2, 23, 0.5))
    B = rhs(A.shape[0], k, "normal", seed=700 + k)
    tol = 1e-8
    s = _solver(A, k, variant, p)
    _, free = s.solve(dev(B), tol=tol, maxit=5000)
    assert free["status"] == oracle.OK
    n = free["iterations"]
    Xg, ig = s.solve(dev(B), tol=tol, maxit=n)
    assert ig["status"] == oracle.OK and ig["iterations"] == n
    Xo, io = oracle_solve(A, B, variant, p, tol=0.0, maxit=n)
    assert rel(host(Xg), Xo) <= CONVERGED_TOL
    Xc, ic = s.solve(dev(B), tol=tol, maxit=n - 1)
    assert ic["status"] == oracle.NOT_CONVERGED and ic["iterations"] == n - 1
    Xo1, _ = oracle_solve(A, B, variant, p, tol=0.0, maxit=n - 1)
    assert rel(host(Xc), Xo1) <= CONVERGED_TOL


# ------------------------------------------ full-size launch configuration
@pytest.mark.parametrize("variant,p,order", [("block", 0, "natural"), ("block", 0, "tiled"), ("hybrid", 4, "tiled")])
def test_full_size_poisson3d_128_fixed_iterations(variant, p, order):
    """128^3 Poisson, k = 16: the chunked sparse-product grid and the two-stage
    reduction of its partial products at the benchmark's size, 6 iterations."""
    P = _lib()
    w = WORKLOADS["poisson3d_128_k16"]
    log(f"full size {variant} p={p} {order}")
    A = stencil_csr(w.dim, w.N)
    B = rhs_for(w)
    m = 6
    Xo, io = oracle_solve(A, B, variant, p, tol=0.0, maxit=m)
    s = P.BCG(*P.stencil(w.dim, w.N), k=w.k, subalgebra=variant, p=p)
    if order == "tiled":
        s.set_row_schedule(P.stencil_schedule(w.dim, w.N, 32))
    Xg, ig = s.solve(dev(B), tol=0.0, maxit=m)
    assert ig["iterations"] == io["iterations"] == m
    assert rel(host(Xg), Xo) <= FIXED_TOL
    np.testing.assert_allclose(ig["ratios"], io["ratios"], rtol=1e-8, atol=0)


# -------- p x p steps on workgroups (p = 3, 12, 24, 64) and in registers (p = 32)
@pytest.mark.parametrize("k,variant,p", [(6, "hybrid", 3), (12, "hybrid", 12), (48, "hybrid", 24), (32, "block", 0),
                                         (64, "block", 0), (64, "global", 32)])
def test_workgroup_small_steps(k, variant, p):
    """Gauss-Jordan small steps for sizes outside {1, 2, 4, 8, 16, 32}, and the
    register steps at p = 32 (two 16-lane pivot rows): iterates,
    Cholesky breakdown (a group with two equal columns) and breakdown on a
    negative definite operator, each against the oracle."""
    log(f"workgroup small steps k={k} {variant} p={p}")
    A = stencil_csr(2, 23, cell_coefficients(2, 23, 0.5))
    B = rhs(A.shape[0], k, "normal", seed=500 + k)
    Xo, io = oracle_solve(A, B, variant, p, tol=0.0, maxit=6)
    s = _solver(A, k, variant, p)
    Xg, ig = s.solve(dev(B), tol=0.0, maxit=6)
    assert ig["iterations"] == io["iterations"] == 6
    assert rel(host(Xg), Xo) <= FIXED_TOL
    Bd = B.copy()
    pe = k if variant == "block" else p
    for g0 in range(0, k, pe):  # two equal columns in every group (global sums the groups)
        Bd[:, g0 + 1] = Bd[:, g0]
    _, od = oracle_solve(A, Bd, variant, p, tol=1e-8, maxit=50)
    _, gd = s.solve(dev(Bd), tol=1e-8, maxit=50)
    assert od["status"] == gd["status"] == oracle.EBREAKDOWN
    assert od["iterations"] == gd["iterations"]
    An = A.copy()
    An.setdiag(-A.diagonal())
    sn = _solver(An, k, variant, p)
    Xn, gn = sn.solve(dev(B), tol=1e-8, maxit=50)
    _, on = oracle_solve(An, B, variant, p, tol=1e-8, maxit=50)
    assert gn["status"] == on["status"] == oracle.EBREAKDOWN
    assert gn["iterations"] == on["iterations"]
