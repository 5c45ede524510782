"""Pins of the oracle's strength test and filtered matrix (plain and OffLmp lumping).

Sources: Sec. 1.1 (strength criterion, filtered matrix), Sec. 1.2 (27-point stencil example
and its negative filtered diagonal), Sec. 2.3 (Algorithm 2, alternative lumping).
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_2103_10476_amd import problems as pb

HZ_S7 = math.sqrt(7.0) / 2.0


def rows_of(rp):
    return np.repeat(np.arange(len(rp) - 1), np.diff(rp))


def center(nint):
    c = nint // 2
    return c + nint * (c + nint * c)


def row_dict(rp, col, val, i):
    return {int(col[e]): float(val[e]) for e in range(rp[i], rp[i + 1])}


# ---- strength ---------------------------------------------------------------------------

def test_strength_brute_force_random(orc):
    """Dense brute force of |A_ij| >= theta sqrt(A_ii A_jj) (away from exact ties)."""
    rng = np.random.default_rng(0)
    for trial in range(20):
        n = 12
        d = rng.uniform(-1, 1, (n, n)) * (rng.uniform(size=(n, n)) < 0.5)
        d = d + d.T
        d[np.arange(n), np.arange(n)] = rng.uniform(0.5, 4.0, n)
        if trial % 3 == 0:
            d[3, 3] = -1.0  # a negative diagonal: its connections are weak
        p = pb.from_dense(d)
        theta = rng.uniform(0.0, 0.6)
        m = orc.strength(p.n, p.rp, p.col, p.val, theta)
        r = rows_of(p.rp)
        for e in range(p.nnz):
            i, j = r[e], p.col[e]
            if i == j:
                assert m[e] == 3
                continue
            di, dj = d[i, i], d[j, j]
            if di * dj <= 0:
                assert m[e] == 0
                continue
            lhs, rhs = abs(d[i, j]), theta * math.sqrt(di * dj)
            if abs(lhs - rhs) > 1e-12 * rhs:
                assert m[e] == (1 if lhs >= rhs else 0)


def test_strength_all_strong_filtered_equals_A(orc):
    """Sec. 1.1: when every connection is strong, the filtered matrix is A itself."""
    p = pb.fd7_stretched(6, 1.0)
    m = orc.strength(p.n, p.rp, p.col, p.val, 0.0)
    assert np.all(m[p.col != rows_of(p.rp)] == 1)
    rp, col, val = orc.lump(p.n, p.rp, p.col, p.val, m)
    assert np.array_equal(rp, p.rp) and np.array_equal(col, p.col)
    assert np.array_equal(val, p.val)


def test_explicit_zeros_are_weak(orc):
    p = pb.q1_hex(6)  # axis-neighbour entries are stored exact zeros
    m = orc.strength(p.n, p.rp, p.col, p.val, 0.02)
    zero_off = (p.val == 0) & (p.col != rows_of(p.rp))
    assert zero_off.sum() > 0 and np.all(m[zero_off] == 0)


# ---- plain lumping ----------------------------------------------------------------------

@pytest.mark.parametrize("name", ["fd5_16x16_a100", "fd7_8_a1000"])
@pytest.mark.parametrize("theta", [0.02, 0.25])
def test_plain_lumping_keeps_row_sums(orc, name, theta):
    """Sec. 1.1: the filtered matrix has the same row sums as A."""
    p = pb.workload(name)
    m = orc.strength(p.n, p.rp, p.col, p.val, theta)
    rp, col, val = orc.lump(p.n, p.rp, p.col, p.val, m)
    rs_a = np.bincount(rows_of(p.rp), weights=p.val, minlength=p.n)
    rs_b = np.bincount(rows_of(rp), weights=val, minlength=p.n)
    scale = np.bincount(rows_of(p.rp), weights=np.abs(p.val), minlength=p.n)
    assert np.all(np.abs(rs_a - rs_b) <= 1e-14 * 16 * scale)
    # the pattern is the diagonal plus the strong entries
    keep = (m == 1) | (m == 3)
    r = rows_of(p.rp)
    assert np.array_equal(col, p.col[keep]) and np.array_equal(rows_of(rp), r[keep])


def test_plain_negative_diagonal_printed_example(orc):
    """Sec. 1.2: for h_z > sqrt(7)/2 a threshold keeping only the positive z-edge entries
    gives a negative filtered diagonal.  h_z = 2: interior row x 72 is 288; -9 (8); -12 (8);
    +48 (2); -30 (4); -24 (4); theta = 0.15 keeps only the +48 -> 288 - 384 = -96."""
    p = pb.q1_stretched_box(5, Fraction(2))
    i = center(5)
    r = row_dict(p.rp, p.col, p.val, i)
    assert sorted(round(v * 72, 9) for v in r.values()) == sorted(
        [288.0] + [-9.0] * 8 + [-12.0] * 8 + [48.0] * 2 + [-30.0] * 4 + [-24.0] * 4)
    m = orc.strength(p.n, p.rp, p.col, p.val, 0.15)
    rp, col, val = orc.lump(p.n, p.rp, p.col, p.val, m)
    rb = row_dict(rp, col, val, i)
    assert len(rb) == 3
    assert rb[i] * 72 == pytest.approx(-96.0, abs=1e-9)


# ---- OffLmp (Algorithm 2) ---------------------------------------------------------------

def test_offlmp_printed_stencil_kminus_nonempty(orc):
    """Sec. 1.2 stencil at h_z = sqrt(7)/2 with theta in (7.5/144, 12/144]: kept +12 (2) and
    -12 (4); r = -120, kappa+ = 24, rhat = -96, ddom(A_i) = 4/3; the growth bound allows
    r* = 96, so the diagonal becomes 48, the -12 entries stay, the +12 entries become 0.
    Plain lumping gives diagonal 24 instead (ddom 3 = 72/24 > 1.1*4/3)."""
    p = pb.q1_hex(6, hx=1.0, hy=1.0, hz=HZ_S7)
    i = center(5)
    s = 36.0 * HZ_S7
    m = orc.strength(p.n, p.rp, p.col, p.val, 0.07)
    rp, col, val = orc.lump(p.n, p.rp, p.col, p.val, m, offlmp=True, tau=1.1)
    rb = {k: v * s for k, v in row_dict(rp, col, val, i).items()}
    assert rb.pop(i) == pytest.approx(48.0, abs=1e-10)
    vals = sorted(rb.values())
    assert len(vals) == 6
    np.testing.assert_allclose(vals[:4], -12.0, atol=1e-10)
    assert vals[4:] == [0.0, 0.0]
    rp2, col2, val2 = orc.lump(p.n, p.rp, p.col, p.val, m, offlmp=False)
    rb2 = {k: v * s for k, v in row_dict(rp2, col2, val2, i).items()}
    assert rb2[i] == pytest.approx(24.0, abs=1e-10)


def test_offlmp_kminus_empty_reading(orc):
    """h_z = 2, theta = 0.15: only the +48 z-edges are kept, K- is empty.  Reading: the whole
    r = -384 goes to K+ when that keeps ddom within tau*ddom(A_i): entries 48*(1-4) = -144,
    diagonal 288, ddom 1 <= 1.1*480/288; the row sum stays 0."""
    p = pb.q1_stretched_box(5, Fraction(2))
    i = center(5)
    m = orc.strength(p.n, p.rp, p.col, p.val, 0.15)
    rp, col, val = orc.lump(p.n, p.rp, p.col, p.val, m, offlmp=True, tau=1.1)
    rb = {k: v * 72 for k, v in row_dict(rp, col, val, i).items()}
    assert rb.pop(i) == pytest.approx(288.0, abs=1e-9)
    np.testing.assert_allclose(sorted(rb.values()), [-144.0, -144.0], atol=1e-9)


def _random_rows(rng, count):
    out = []
    for _ in range(count):
        m = int(rng.integers(2, 9))
        off = rng.normal(size=m) * rng.uniform(0.1, 3.0)
        kept = rng.uniform(size=m) < 0.5
        aii = abs(off).sum() * rng.uniform(0.5, 1.5)
        out.append((aii, off, kept))
    return out


def _row_problem(aii, off, kept):
    """One tested row 0 embedded in a matrix whose other rows are diagonal."""
    m = len(off)
    n = m + 1
    d = np.eye(n)
    d[0, 0] = aii
    d[0, 1:] = off
    p = pb.from_dense(d, keep_zero_pattern=np.ones((n, n), bool) & (np.arange(n)[:, None] == 0))
    mask = np.zeros(p.nnz, dtype=np.uint8)
    r = rows_of(p.rp)
    for e in range(p.nnz):
        if p.col[e] == r[e]:
            mask[e] = 3
        elif r[e] == 0 and kept[p.col[e] - 1]:
            mask[e] = 1
    return p, mask


def test_offlmp_invariants_random_rows(orc):
    """Algorithm 2 invariants: removed entries are gone; the row sum of A is kept (except the
    K- empty rows where no admissible lumping exists); ddom(Abar_i) <= tau*ddom(A_i) whenever
    an admissible r* exists; r* < A_ii when K- is nonempty, so the diagonal stays positive;
    for rows with only negative off-diagonals and zero row sum it equals plain lumping."""
    rng = np.random.default_rng(1)
    tau = 1.1
    checked = 0
    for aii, off, kept in _random_rows(rng, 400):
        p, mask = _row_problem(aii, off, kept)
        rp, col, val = orc.lump(p.n, p.rp, p.col, p.val, mask, offlmp=True, tau=tau)
        row = row_dict(rp, col, val, 0)
        assert set(row) == {0} | {j + 1 for j in range(len(off)) if kept[j]}
        r = off[~kept].sum()
        kp = off[kept & (off > 0)].sum()
        has_km = np.any(kept & (off < 0))
        ddom_a = np.abs(off).sum() / aii
        rowsum_kept = abs(sum(row.values()) - (aii + off.sum())) <= 1e-12 * (aii + np.abs(off).sum())
        if r >= 0 or -r <= kp:
            assert rowsum_kept
        elif has_km:
            assert rowsum_kept
            assert row[0] > 0
            ddom_b = sum(abs(v) for k, v in row.items() if k != 0) / row[0]
            # admissible iff some r in [0, U] meets the bound; check the bound when met
            U = min(abs(r + kp), aii)
            rstar = aii - row[0]
            if ddom_b <= tau * ddom_a * (1 + 1e-12) and rstar < U * (1 - 1e-9):
                # the largest admissible r*: the growth bound is active
                assert ddom_b == pytest.approx(tau * ddom_a, rel=1e-9)
            if ddom_b > tau * ddom_a * (1 + 1e-12):
                # then no admissible r* exists: ddom is at its minimum over [0, U]
                c, a, U = -off[kept & (off < 0)].sum() - (r + kp), aii, min(abs(r + kp), aii)
                grid = np.linspace(0, U, 101)
                assert ddom_b <= np.min((c - grid) / (a - grid)) * (1 + 1e-9)
            checked += 1
        else:
            lumped = abs(r + kp) / aii <= tau * ddom_a
            assert rowsum_kept == lumped or not np.any(kept)
    assert checked > 20


def test_offlmp_equals_plain_on_mmatrix_rows(orc):
    """Sec. 2.3: all off-diagonals negative and zero row sum -> ddom stays 1, any reasonable
    lumping agrees; OffLmp equals plain lumping there (C2-like interior rows)."""
    p = pb.fd7_stretched(10, 1000.0)
    m = orc.strength(p.n, p.rp, p.col, p.val, 0.3)
    a = orc.lump(p.n, p.rp, p.col, p.val, m, offlmp=False)
    b = orc.lump(p.n, p.rp, p.col, p.val, m, offlmp=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    rows = rows_of(a[0])
    has_kept = np.diff(a[0]) > 1
    same = a[2] == b[2]
    assert np.all(same[has_kept[rows]])
    # rows with no kept off-diagonal: Sec. 2.3 skips the lumping (diagonal stays A_ii)
    lone = np.nonzero(~has_kept)[0]
    assert lone.size > 0
    d = {i: v for i, v in zip(rows, b[2]) if not has_kept[i]}
    for i in lone:
        aii = [p.val[e] for e in range(p.rp[i], p.rp[i + 1]) if p.col[e] == i][0]
        assert d[i] == aii
