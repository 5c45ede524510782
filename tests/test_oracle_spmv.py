"""Oracle pins for y = A x and its row-sum order.

The mathematics fixes the value of every row sum when the arithmetic is exact, and the
reading fixes the rounding order otherwise:

* integer matrices and vectors of small magnitude make every partial sum exact, so y must
  equal the integer product for rows of any length (1 .. 300 entries here: both sides of the
  64-entry split), whatever the order;
* a row of at most 64 entries is the sequential sum in ascending column order from 0.0;
* a row of more than 64 entries is 64 interleaved partial sums (positions l, l+64, ...),
  each in order from 0.0, added in order from 0.0.  Products 2^-53 (positions 0..63) and 1.0
  (position 64) separate the two orders: in plain order the small products add exactly to
  2^-47 before the 1.0 arrives (1 + 2^-47), in the split order each meets the 1.0 (or a sum
  of at least 1.0) and rounds away (1.0).
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


def test_short_rows_sum_in_column_order():
    rng = np.random.Generator(np.random.PCG64(8))
    rows = []
    for L in (1, 5, 17, 63, 64):
        cols = np.sort(rng.choice(200, size=L, replace=False))
        rows.append([(int(c), float(v)) for c, v in zip(cols, rng.standard_normal(L))])
    rp, col, val = _csr(rows)
    x = rng.standard_normal(200)
    y = orc.spmv(rp, col, val, x)
    for i, r in enumerate(rows):
        s = 0.0
        for c, v in r:
            s += v * x[c]
        assert y[i] == s


def test_long_rows_use_the_interleaved_split():
    tiny = 2.0 ** -53
    # row 0: 65 entries, products tiny at positions 0..63 and 1.0 at position 64
    # row 1: the same 64 tiny products and the 1.0 at position 63 of a 64-entry row
    r0 = [(c, tiny) for c in range(64)] + [(64, 1.0)]
    r1 = [(c, tiny) for c in range(63)] + [(63, 1.0)]
    rp, col, val = _csr([r0, r1])
    y = orc.spmv(rp, col, val, np.ones(65))
    assert y[0] == 1.0                       # split order: every tiny product rounds away
    assert 64 * tiny + 1.0 == 1.0 + 2.0 ** -47  # the plain order would give this instead
    plain = 0.0
    for _, v in r1:
        plain += v
    assert y[1] == plain and plain > 1.0     # 64 entries: still the plain order


def test_long_row_partials_follow_positions_not_columns():
    # a 130-entry row over scattered columns: positions 0, 64, 128 form p_0; the order within
    # the row is by position (ascending column), whatever the column numbers
    rng = np.random.Generator(np.random.PCG64(9))
    cols = np.sort(rng.choice(5000, size=130, replace=False))
    v = rng.standard_normal(130)
    rp, col, val = _csr([[(int(c), float(a)) for c, a in zip(cols, v)]])
    x = rng.standard_normal(5000)
    prods = v * x[cols]
    parts = []
    for l in range(64):
        p = 0.0
        for k in range(l, 130, 64):
            p += prods[k]
        parts.append(p)
    s = 0.0
    for p in parts:
        s += p
    assert orc.spmv(rp, col, val, x)[0] == s
