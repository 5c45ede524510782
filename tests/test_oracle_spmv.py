"""Oracle pins for y = A x and its row-sum order.

The mathematics fixes the value of every row sum when the arithmetic is exact, and the
definition y_i = sum_j a_ij x_j, taken in ascending column order from 0.0, fixes the rounding
otherwise:

* integer matrices and vectors of small magnitude make every partial sum exact, so y must
  equal the integer product for rows of any length (1 .. 300 entries here), whatever the
  order;
* a row of any length is the sequential sum in ascending column order from 0.0;
* products 2^-53 (positions 0..63) and 1.0 (position 64) tell the sequential order from any
  blocked one: added in order, the small products sum exactly to 2^-47 before the 1.0 arrives
  (1 + 2^-47); a split into interleaved partial sums would meet the 1.0 with each small
  product separately and round them all away (1.0).
"""
import numpy as np

from oracle import oracle as orc


def _csr(rows):
    rp = np.zeros(len(rows) + 1, dtype=np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([c for r in rows for c, _ in r], dtype=np.int32)
    val = np.array([v for r in rows for _, v in r], dtype=np.float64)
    return rp, col, val


def test_integer_products_are_exact():
    rng = np.random.Generator(np.random.PCG64(7))
    ncols = 400
    lengths = [0, 1, 2, 63, 64, 65, 66, 127, 128, 129, 200, 300]
    rows = []
    for L in lengths:
        cols = np.sort(rng.choice(ncols, size=L, replace=False))
        rows.append([(int(c), float(rng.integers(-9, 10))) for c in cols])
    rp, col, val = _csr(rows)
    x = rng.integers(-9, 10, size=ncols).astype(np.float64)
    y = orc.spmv(rp, col, val, x)
    dense = np.zeros((len(rows), ncols), dtype=np.int64)
    for i, r in enumerate(rows):
        for c, v in r:
            dense[i, c] = int(v)
    assert np.array_equal(y, (dense @ x.astype(np.int64)).astype(np.float64))


def test_rows_sum_in_column_order():
    rng = np.random.Generator(np.random.PCG64(8))
    rows = []
    for L in (1, 5, 17, 63, 64, 65, 130, 1000):
        cols = np.sort(rng.choice(2000, size=L, replace=False))
        rows.append([(int(c), float(v)) for c, v in zip(cols, rng.standard_normal(L))])
    rp, col, val = _csr(rows)
    x = rng.standard_normal(2000)
    y = orc.spmv(rp, col, val, x)
    for i, r in enumerate(rows):
        s = 0.0
        for c, v in r:
            s += v * x[c]
        assert y[i] == s


def test_long_rows_are_not_blocked():
    tiny = 2.0 ** -53
    # row 0: 65 entries, products tiny at positions 0..63 and 1.0 at position 64;
    # row 1: 2000 entries, tiny at 0..1998 and 1.0 last
    r0 = [(c, tiny) for c in range(64)] + [(64, 1.0)]
    r1 = [(c, tiny) for c in range(1999)] + [(1999, 1.0)]
    rp, col, val = _csr([r0, r1])
    y = orc.spmv(rp, col, val, np.ones(2000))
    assert y[0] == 1.0 + 2.0 ** -47          # 64 * 2^-53 is exact, then 1.0 is added
    assert y[1] == 1.0 + 1999 * tiny         # 1999 * 2^-53 is exact below 2^-42
    assert 1999 * tiny + 1.0 != 1.0
