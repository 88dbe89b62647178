"""SELL-16-sigma layout of the library (host code, CPU only) against its
definition: slices of 16 positions, two 8-position halves stored slot by
slot, width = longest row of the slice (at least 1), rows sorted by
decreasing length (stable) within windows of sigma positions, padding =
the row's own column with entry index -1. The GPU tests check that the
sparse product on this layout is bitwise the CSR one."""
import ctypes

import numpy as np
import pytest


@pytest.fixture(scope="module")
def lib():
    from paper_1912_11930_amd import _capi
    return _capi.lib()


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _layout(lib, rp, ci, order, sigma):
    n = rp.size - 1
    slots = lib.bcg_sell_layout(n, _ptr(rp), _ptr(ci), _ptr(order), sigma, None, None, None, None)
    assert slots > 0, lib.bcg_last_error()
    ns = (n + 15) // 16
    sp = np.empty(ns + 1, np.int32)
    perm = np.empty(16 * ns, np.int32)
    col = np.empty(slots, np.int32)
    mp = np.empty(slots, np.int32)
    assert lib.bcg_sell_layout(n, _ptr(rp), _ptr(ci), _ptr(order), sigma, _ptr(sp), _ptr(perm), _ptr(col),
                               _ptr(mp)) == slots
    return sp, perm, col, mp


def _pattern(n, seed):
    """Random CSR pattern with row lengths 0..min(12, n) (empty rows included)."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, min(13, n + 1), n)
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    ci = np.concatenate([np.sort(rng.choice(n, size=l, replace=False)) for l in lens]).astype(np.int32)
    return rp, ci


def _expected_order(lens, order, sigma):
    pos = order.copy()
    if sigma > 1:
        for w0 in range(0, pos.size, sigma):
            win = pos[w0:w0 + sigma]
            pos[w0:w0 + sigma] = win[np.argsort(-lens[win], kind="stable")]
    return pos


@pytest.mark.parametrize("n", [1, 16, 37, 200])
@pytest.mark.parametrize("sigma", [1, 16, 32])
@pytest.mark.parametrize("ordered", [False, True])
def test_layout_matches_definition(lib, n, sigma, ordered):
    rp, ci = _pattern(n, seed=n + sigma)
    lens = np.diff(rp)
    order = np.random.default_rng(7).permutation(n).astype(np.int32) if ordered else None
    sp, perm, col, mp = _layout(lib, rp, ci, order, sigma)
    pos = _expected_order(lens, order if ordered else np.arange(n, dtype=np.int32), sigma)
    ns = (n + 15) // 16
    assert np.array_equal(perm[:n], pos)
    assert np.all(perm[n:] == pos[-1])
    assert sp[0] == 0
    seen = np.zeros(rp[-1], np.int64)
    for S in range(ns):
        real = [p for p in range(16 * S, 16 * S + 16) if p < n]
        w = max(1, max(lens[perm[p]] for p in real))
        assert sp[S + 1] - sp[S] == 16 * w
        for r in range(16):
            row = perm[16 * S + r]
            length = lens[row] if 16 * S + r < n else 0
            for t in range(w):
                e = sp[S] + 8 * w * (r >> 3) + 8 * t + (r & 7)
                if t < length:
                    assert mp[e] == rp[row] + t and col[e] == ci[rp[row] + t]
                    seen[mp[e]] += 1
                else:
                    assert mp[e] == -1 and col[e] == row
    assert np.all(seen == 1)          # every CSR entry exactly once


def test_layout_rejects_bad_arguments(lib):
    from paper_1912_11930_amd import _capi
    rp, ci = _pattern(20, seed=1)
    for sigma in (0, 17, -16):
        assert lib.bcg_sell_layout(20, _ptr(rp), _ptr(ci), None, sigma, None, None, None, None) == _capi.BCG_EINVAL
    bad = np.arange(20, dtype=np.int32)
    bad[3] = 20
    assert lib.bcg_sell_layout(20, _ptr(rp), _ptr(ci), _ptr(bad), 1, None, None, None, None) == _capi.BCG_EINVAL
    dec = rp.copy()
    dec[5] = dec[6] + 1
    assert lib.bcg_sell_layout(20, _ptr(dec), _ptr(ci), None, 1, None, None, None, None) == _capi.BCG_EINVAL
    assert lib.bcg_sell_layout(0, _ptr(rp), _ptr(ci), None, 1, None, None, None, None) == _capi.BCG_EINVAL
