"""CPU pins of the brick row order's definition (the reference the GPU
schedule is compared with in test_gpu_parity.py): checked against the
geometric properties the order is meant to have, not against its own formula."""
import numpy as np
import pytest

from tests.test_gpu_parity import _brick_order


def _cells(order, N):
    """(z, y, x) of every position of the order (rows are x-fastest)."""
    r = order.astype(np.int64)
    return r // (N * N), (r // N) % N, r % N


@pytest.mark.parametrize("N,tile,brick", [(8, (4, 4, 2), (2, 2, 2)), (12, (6, 4, 3), (3, 2, 1)),
                                          (32, (16, 32, 2), (4, 2, 2)), (16, (8, 8, 16), (4, 2, 2))])
def test_brick_order_geometry(N, tile, brick):
    tx, ty, tz = tile
    bx, by, bz = brick
    order = _brick_order(N, tile, brick)
    assert np.array_equal(np.sort(order), np.arange(N ** 3))  # a permutation
    z, y, x = _cells(order, N)
    nb, nt = bx * by * bz, tx * ty * tz
    # every run of nb positions is one axis-aligned brick, x fastest, then y, then z
    for s in range(0, N ** 3, nb):
        zz, yy, xx = z[s:s + nb], y[s:s + nb], x[s:s + nb]
        assert xx.min() % bx == 0 and yy.min() % by == 0 and zz.min() % bz == 0
        assert np.array_equal(xx - xx.min(), np.tile(np.arange(bx), by * bz))
        assert np.array_equal(yy - yy.min(), np.tile(np.repeat(np.arange(by), bx), bz))
        assert np.array_equal(zz - zz.min(), np.repeat(np.arange(bz), bx * by))
    # every run of nt positions is one tile; the tiles of a tile column follow
    # each other through z, and the bricks of a tile go x, then y, then z
    col0 = None
    for t, s in enumerate(range(0, N ** 3, nt)):
        zz, yy, xx = z[s:s + nt], y[s:s + nt], x[s:s + nt]
        assert xx.max() - xx.min() == tx - 1 and yy.max() - yy.min() == ty - 1 and zz.max() - zz.min() == tz - 1
        assert len(set(zip(zz.tolist(), yy.tolist(), xx.tolist()))) == nt
        col = (yy.min() // ty, xx.min() // tx)
        if t % (N // tz) == 0:
            col0 = col
            assert zz.min() == 0
        else:
            assert col == col0 and zz.min() == (t % (N // tz)) * tz
        firsts = [(zz[b], yy[b], xx[b]) for b in range(0, nt, nb)]
        keys = [((fz - zz.min()) // bz, (fy - yy.min()) // by, (fx - xx.min()) // bx) for fz, fy, fx in firsts]
        assert keys == sorted(keys)
    # tile columns in row-major order over (y, x)
    cols = [(y[s] // ty, x[s] // tx) for s in range(0, N ** 3, nt * (N // tz))]
    assert cols == sorted(cols) and len(set(cols)) == (N // tx) * (N // ty)
