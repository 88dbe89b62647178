"""The C-ABI library loads and exports every function of include/bcg.h (CPU only).

No compute call is made here: only host-side argument validation, which
returns before any device work.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bcg.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bcg_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1912_11930_amd import _capi
    if not os.path.exists(_capi.LIB_PATH):
        pytest.fail("libbcg.so is not built (run python -m paper_1912_11930_amd.build)")
    return _capi.lib()


def test_every_declared_symbol_is_exported(lib):
    from paper_1912_11930_amd import _capi
    names = _declared()
    assert len(names) >= 13
    bound = {n for n, _, _ in _capi.SIGNATURES}
    assert set(names) == bound, (set(names) ^ bound)
    for name in names:
        assert hasattr(lib, name), name


def test_stencil_nnz_host_only(lib):
    assert lib.bcg_stencil_nnz(2, 32) == 4992
    assert lib.bcg_stencil_nnz(3, 128) == 14581760
    assert lib.bcg_stencil_nnz(3, 256) == 117047296
    assert lib.bcg_stencil_nnz(4, 8) == -1
    assert lib.bcg_stencil_nnz(2, 0) == -1
    assert lib.bcg_stencil_nnz(3, 1300) == -1      # n beyond int32


def test_argument_validation_without_device(lib):
    from paper_1912_11930_amd import _capi
    h = ctypes.c_void_p()
    assert lib.bcg_create(None, 8, 0, 0, ctypes.byref(h)) == _capi.BCG_EINVAL
    assert b"CSR" in lib.bcg_last_error()
    csr = _capi.Csr(16, 64, 1, 2, 3)               # non-NULL dummies: rejected before use
    for k, sub, p in [(0, 0, 0), (257, 0, 0), (8, 0, 4), (8, 2, 2), (8, 3, 3), (8, 1, 16), (8, 9, 1)]:
        assert lib.bcg_create(ctypes.byref(csr), k, sub, p, ctypes.byref(h)) == _capi.BCG_EINVAL
    bad = _capi.Csr(-1, 64, 1, 2, 3)
    assert lib.bcg_create(ctypes.byref(bad), 8, 0, 0, ctypes.byref(h)) == _capi.BCG_EINVAL
    assert lib.bcg_set_precision(None, 1, 1e-4, 10, 10) == _capi.BCG_EINVAL
    assert lib.bcg_solve(None, None, None, 1e-8, 10) == _capi.BCG_EINVAL
    assert lib.bcg_set_sell(None, 1, 1) == _capi.BCG_EINVAL
    assert lib.bcg_stencil_build(4, 8, None, None, None, None, None) == _capi.BCG_EINVAL
    lib.bcg_destroy(None)


def test_brick_schedule_rejects_sizes_without_device(lib):
    from paper_1912_11930_amd import _capi
    three = ctypes.c_int * 3
    f = lib.bcg_stencil_brick_schedule
    assert f(32, three(16, 32, 2), three(4, 2, 2), None, None) == _capi.BCG_EINVAL      # order NULL
    assert f(32, three(12, 32, 2), three(4, 2, 2), 1, None) == _capi.BCG_EINVAL         # tile does not divide N
    assert f(32, three(16, 32, 2), three(3, 2, 2), 1, None) == _capi.BCG_EINVAL         # brick does not divide tile
    assert f(0, three(1, 1, 1), three(1, 1, 1), 1, None) == _capi.BCG_EINVAL
    assert f(1300, three(1, 1, 1), three(1, 1, 1), 1, None) == _capi.BCG_EINVAL         # N^3 beyond int32


def test_noalloc_argument_validation_without_device(lib):
    # every rejection below happens on the host, before the fixed array is touched
    from paper_1912_11930_amd import _capi
    EINVAL = _capi.BCG_EINVAL
    f = lib.bcg_solve_noalloc
    assert f(None, 8, 0, 0, 4, 5, 1e-8, 10, None, None) == EINVAL
    csr = _capi.Csr(16, 64, 1, 2, 3)
    assert f(ctypes.byref(csr), 8, 0, 0, None, 5, 1e-8, 10, None, None) == EINVAL      # B NULL
    assert f(ctypes.byref(csr), 8, 0, 0, 4, 4, 1e-8, 10, None, None) == EINVAL        # B aliases X
    assert f(ctypes.byref(csr), 8, 0, 0, 4, 5, -1.0, 10, None, None) == EINVAL        # tol < 0
    assert f(ctypes.byref(csr), 8, 3, 3, 4, 5, 1e-8, 10, None, None) == EINVAL        # p does not divide k
    big = _capi.Csr(10_000_000, 70_000_000, 1, 2, 3)                                  # 3 n k doubles > 128 MiB
    assert f(ctypes.byref(big), 8, 0, 0, 4, 5, 1e-8, 10, None, None) == EINVAL
    assert b"workspace" in lib.bcg_last_error()
