"""Pins of the oracle's smoothing diagonal, eigenvalue estimate, prolongator and Cnstrnt.

Sources: Sec. 1.1 (prolongator smoothing, damping 4/(3 lambda)), Sec. 1.2 (Gershgorin bound
for strictly diagonally dominant matrices), Sec. 2.1 (1-norm diagonal; circulant example),
Sec. 2.2 (safeguard; diagonal example; root-row value), Sec. 2.4 (Algorithm 3).
"""
import numpy as np
import pytest

from paper_2103_10476_amd import problems as pb


def rows_of(rp):
    return np.repeat(np.arange(len(rp) - 1), np.diff(rp))


def dense(rp, col, val, n, m=None):
    d = np.zeros((n, n if m is None else m))
    d[rows_of(rp), col] = val
    return d


def five_point_periodic(side=12):
    return pb.periodic_stencil_2d(side, side, {(0, 0): 4.0, (1, 0): -1.0, (-1, 0): -1.0,
                                               (0, 1): -1.0, (0, -1): -1.0})


def test_circulant_printed_diagonals_and_eigenvalues(orc):
    """Sec. 2.1: periodic 5-point Poisson: Dbar = 4, Dtilde = 8, lambda_bar = 2,
    lambda_tilde = 1 (power estimates approach them from below)."""
    p = five_point_periodic()
    m = orc.strength(p.n, p.rp, p.col, p.val, 0.0)
    Ab = orc.lump(p.n, p.rp, p.col, p.val, m)
    dbar = orc.diag(p.n, *Ab, one_norm=False)
    dtil = orc.diag(p.n, *Ab, one_norm=True)
    assert np.all(dbar == 0.25) and np.all(dtil == 0.125)
    lbar = orc.power(p.n, *Ab, dbar, iters=10)
    ltil = orc.power(p.n, *Ab, dtil, iters=10)
    assert 1.8 < lbar <= 2.0 + 1e-14
    assert ltil == lbar / 2  # exact power-of-two scaling of every iterate
    lbar200 = orc.power(p.n, *Ab, dbar, iters=200)
    assert 1.99 < lbar200 <= 2.0 + 1e-14


def test_circulant_1norm_prolongator_equals_plain(orc):
    """Sec. 2.1: on a circulant the 1-norm step reproduces plain SA exactly
    (power-method mode: bitwise identical P)."""
    p = five_point_periodic()
    kw = dict(theta=0.0, max_levels=2, max_coarse=10)
    h0 = orc.OracleHierarchy(p.n, p.rp, p.col, p.val + 0.0, **kw)
    h1 = orc.OracleHierarchy(p.n, p.rp, p.col, p.val + 0.0, variants=["1norm"],
                             one_norm_power=1, **kw)
    for a, b in zip(h0.levels[0].P, h1.levels[0].P):
        assert np.array_equal(a, b)
    assert h1.levels[0].lam == h0.levels[0].lam / 2


@pytest.mark.parametrize("sigma,expect", [(1.0 / 3.0, 1.0 / 3.0), (-1.0 / 3.0, -1.0 / 3.0)])
def test_diagonal_abar_example(orc, sigma, expect):
    """Sec. 2.2: for a diagonal Abar, Dtilde^{-1} Abar = I and lambda = 1 give
    P = -Ptent/3; with the safeguard (sigma = 1/3, D := 2 s_i) it becomes +Ptent/3.
    sigma = -1/3 makes the safeguard inactive (4/(3(1-sigma)) = 1)."""
    n = 6
    d = np.diag([1.0, 2.0, 3.0, 0.5, 4.0, 7.0])
    p = pb.from_dense(d)
    invD = orc.diag(p.n, p.rp, p.col, p.val, one_norm=True, sigma=sigma)
    agg = np.array([0, 0, 1, 1, 2, 2], dtype=np.int32)
    rp, col, val = orc.prolongator(p.n, p.rp, p.col, p.val, invD, agg, 4.0 / 3.0)
    P = dense(rp, col, val, n, 3)
    Pt = np.zeros((n, 3))
    Pt[np.arange(n), agg] = 1
    np.testing.assert_allclose(P, expect * Pt, atol=1e-15)


def test_prolongator_dense_brute_force(orc):
    """Sec. 1.1: P = (I - omega D^{-1} Abar) Ptent, checked densely on a small problem,
    plain and 1Norm, and the closed-form row sums 1 - omega s_i / D_i on aggregated rows."""
    p = pb.workload("fd5_12x12_a100")
    for one_norm in (False, True):
        h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, theta=0.02, max_levels=2,
                                max_coarse=10, variants=["1norm"] if one_norm else [])
        L = h.levels[0]
        Ab = dense(*L.Abar, p.n)
        Pt = np.zeros((p.n, L.nc))
        ok = L.agg >= 0
        Pt[np.nonzero(ok)[0], L.agg[ok]] = 1.0
        Pd = (np.eye(p.n) - L.omega * np.diag(L.invD) @ Ab) @ Pt
        P = dense(*L.P, p.n, L.nc)
        np.testing.assert_allclose(P, Pd, atol=1e-14 * np.abs(Pd).max())
        s = Ab.sum(axis=1)
        np.testing.assert_allclose(P.sum(axis=1)[ok], (1 - L.omega * L.invD * s)[ok],
                                   atol=1e-13)
        # pattern: the aggregates reached by the filtered row
        for i in range(p.n):
            cols = set(L.P[1][L.P[0][i]:L.P[0][i + 1]])
            reach = {int(L.agg[k]) for k in L.Abar[1][L.Abar[0][i]:L.Abar[0][i + 1]]
                     if L.agg[k] >= 0}
            assert cols == reach


def test_constant_in_range_of_P_when_abar_annihilates_constants(orc):
    """Sec. 1.1: if Abar 1 = 0 then the constant lies in range(P): P 1 = 1."""
    p = five_point_periodic(9)  # singular (periodic): built step by step, no coarse solve
    m = orc.strength(p.n, p.rp, p.col, p.val, 0.0)
    agg, root, nc = orc.aggregate(p.n, p.rp, p.col, m)
    Ab = orc.lump(p.n, p.rp, p.col, p.val, m)
    invD = orc.diag(p.n, *Ab)
    lam = orc.power(p.n, *Ab, invD)
    rp, col, val = orc.prolongator(p.n, *Ab, invD, agg, 4.0 / (3.0 * lam))
    P = dense(rp, col, val, p.n, nc)
    np.testing.assert_allclose(P @ np.ones(nc), 1.0, atol=1e-14)


def test_root_row_safeguard_bound(orc):
    """Sec. 2.2: a root whose filtered row lies inside its aggregate gets
    P_ij = 1 - (4/3) s_i/Dtilde_ii >= sigma = 1/3 (lambda_tilde = 1, safeguard on)."""
    p = pb.workload("fd7_12_a1000")
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, theta=0.02, variants=["1norm"],
                            max_levels=2, max_coarse=10)
    L = h.levels[0]
    found = 0
    for i in np.nonzero(L.is_root)[0]:
        ks = L.Abar[1][L.Abar[0][i]:L.Abar[0][i + 1]]
        if np.all(L.agg[ks] == L.agg[i]):
            vals = L.Abar[2][L.Abar[0][i]:L.Abar[0][i + 1]]
            s = vals.sum()
            e = [x for x in range(L.P[0][i], L.P[0][i + 1]) if L.P[1][x] == L.agg[i]][0]
            assert L.P[2][e] == pytest.approx(1 - (4 / 3) * s * L.invD[i], abs=1e-14)
            assert L.P[2][e] >= 1 / 3 - 1e-14
            found += 1
    assert found > 10


def test_gershgorin_bounds(orc):
    """Sec. 2.1: lambda of Dtilde^{-1} Abar is at most 1; Sec. 1.2: lambda of Dbar^{-1} Abar
    is below 2 when Abar is strictly diagonally dominant."""
    for name in ("fd7_10_a1000", "fd5_16x16_a100", "q1_box24_hz2"):
        p = pb.workload(name) if name != "q1_box24_hz2" else pb.q1_stretched_box(8)
        m = orc.strength(p.n, p.rp, p.col, p.val, 0.02)
        Ab = orc.lump(p.n, p.rp, p.col, p.val, m)
        dt = orc.diag(p.n, *Ab, one_norm=True)
        assert orc.power(p.n, *Ab, dt) <= 1.0 + 1e-13
    # strictly dominant: add a reaction term
    p = pb.fd7_stretched(8, 10.0)
    rows = rows_of(p.rp)
    val = p.val + np.where(p.col == rows, 1e-3, 0.0)
    m = orc.strength(p.n, p.rp, p.col, val, 0.0)
    Ab = orc.lump(p.n, p.rp, p.col, val, m)
    db = orc.diag(p.n, *Ab, one_norm=False)
    lam = orc.power(p.n, *Ab, db)
    assert 0 < lam < 2.0


def test_small_diagonal_failure_mode_and_fixes(orc):
    """Sec. 1.2: on 1x1x2 hexahedra a threshold keeping only the positive z-edge entries
    makes plain filtered diagonals negative (Dbar^{-1} Abar indefinite); the 1-norm diagonal
    is positive on every row and OffLmp keeps every filtered diagonal positive (Sec. 2.1-2.3).
    All variants still give a convergent solver on this input."""
    from fractions import Fraction
    p = pb.q1_stretched_box(24, Fraction(2))
    m = orc.strength(p.n, p.rp, p.col, p.val, 0.15)
    plain = orc.lump(p.n, p.rp, p.col, p.val, m)
    rows = rows_of(plain[0])
    dplain = plain[2][plain[1] == rows]
    assert np.sum(dplain < 0) > 1000
    assert np.all(orc.diag(p.n, *plain, one_norm=True) > 0)
    off = orc.lump(p.n, p.rp, p.col, p.val, m, offlmp=True)
    assert np.all(off[2][off[1] == rows_of(off[0])] > 0)
    b = pb.random_rhs(p.n, 7)
    for var in ([], ["1norm"], ["offlmp"], ["1norm", "offlmp"]):
        h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, theta=0.15, variants=var)
        r = h.solve(b)
        assert r["converged"] and r["iterations"] < 40


def test_no_strong_connection_level_becomes_coarsest(orc):
    """Reading: a level with no strong connection cannot be aggregated; it is solved
    directly instead of reporting a stall."""
    from fractions import Fraction
    p = pb.q1_stretched_box(8, Fraction(2))
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, theta=0.15, max_coarse=20)
    assert h.levels[-1].n > 20
    r = h.solve(pb.random_rhs(p.n, 7))
    assert r["converged"]


# ---- Cnstrnt (Algorithm 3) --------------------------------------------------------------

def test_cnstrnt_worked_example(orc):
    """Algorithm 3 on (0.65, 1.16, -0.46): pin -0.46 to 0 and 1.16 to 1, spread -0.30 over
    the rest -> (0.35, 1, 0); row sum 1.35 kept."""
    rp = np.array([0, 3], dtype=np.int32)
    col = np.array([0, 1, 2], dtype=np.int32)
    v = orc.cnstrnt(1, rp, col, np.array([0.65, 1.16, -0.46]), np.array([1], np.int32))
    np.testing.assert_allclose(v, [0.35, 1.0, 0.0], atol=1e-15)


def _projection(p):
    """Exact Euclidean projection onto {0<=x<=1, sum x = sum p} over the nonzero pattern
    (bisection on the shift mu of clip(p - mu, 0, 1))."""
    s = p.sum()
    lo, hi = p.min() - 1, p.max() + 1
    for _ in range(200):
        mu = 0.5 * (lo + hi)
        if np.clip(p - mu, 0, 1).sum() > s:
            lo = mu
        else:
            hi = mu
    return np.clip(p - 0.5 * (lo + hi), 0, 1)


def test_cnstrnt_random_rows_invariants(orc):
    """Sec. 2.4: feasible rows end in [0,1] with the same sum and pattern; infeasible rows
    (sum < 0 or sum > nnz) become the tentative row; the result is never closer to P than the
    exact projection (Algorithm 3 is a heuristic for it)."""
    rng = np.random.default_rng(3)
    n_feas = 0
    for _ in range(500):
        m = int(rng.integers(1, 8))
        v = rng.normal(0.4, 0.6, m)
        v[rng.uniform(size=m) < 0.15] = 0.0
        cols = np.sort(rng.choice(20, m, replace=False)).astype(np.int32)
        aggi = int(cols[rng.integers(0, m)])
        out = orc.cnstrnt(1, np.array([0, m], np.int32), cols, v, np.array([aggi], np.int32))
        if np.all((v >= 0) & (v <= 1)):
            assert np.array_equal(out, v)
            continue
        nz = v != 0
        s = v[nz].sum()
        if s < 0 or s > nz.sum():
            assert np.array_equal(out, (cols == aggi).astype(float))
            continue
        tent = (cols == aggi).astype(float)
        if np.array_equal(out, tent) and not np.isclose(out.sum(), v.sum()):
            # Algorithm 3 pinned every entry while a residual remained (e.g. (1.2, -0.1)):
            # the degenerate guard takes the tentative row
            n_degenerate = locals().get("n_degenerate", 0) + 1
            continue
        n_feas += 1
        assert np.all(out[~nz] == 0)
        assert np.all((out >= -1e-15) & (out <= 1 + 1e-15))
        assert out.sum() == pytest.approx(v.sum(), abs=1e-13)
        proj = np.zeros(m)
        proj[nz] = _projection(v[nz])
        assert np.linalg.norm(out - v) >= np.linalg.norm(proj - v) - 1e-9
    assert n_feas > 50
