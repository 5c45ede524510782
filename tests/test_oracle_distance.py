"""Oracle pins for the distance-Laplacian strength (Sec. 3.1) and the coarse coordinates.

L^(d) has A's pattern, off-diagonals -1/|x_i - x_j|^p (p = 1, the paper's text, or p = 2) and a
zero row sum; (i,j) is strong iff |L_ij| >= theta sqrt(L_ii L_jj).  On integer grids every
quantity is an exact small integer (or a power-of-two fraction), so the labels have closed forms
in the neighbour counts:

* uniform unit grid: w = 1, L_ii = n_i (the number of stored neighbours), so (i,j) is strong
  iff n_i n_j <= 1/theta^2, for either power;
* unit spacing in x and y, spacing 1/4 in z: w = 1 in-plane, 4^p across planes,
  L_ii = p_i + 4^p q_i (p_i in-plane and q_i vertical neighbours);
* the labels depend on the coordinates only: any matrix values on the pattern, any power-of-two
  scaling, integer translation or axis permutation of the coordinates give the same labels;
* when A itself is the weighted graph Laplacian of the coordinates, the classical test on A
  and the distance test take the same decisions (both compare the same numbers).

Coarse coordinates are the aggregates' centroids; a full setup on coordinates builds a
hierarchy whose every coarse level carries them, and solves the stretched problems.
"""
import math

import numpy as np
import pytest

from paper_2103_10476_amd import problems as pb


def _counts(p):
    return np.diff(p.rp) - 1  # stored neighbours (the diagonal is always stored)


def _offdiag(p):
    rows = np.repeat(np.arange(p.n), np.diff(p.rp))
    return rows, p.col, rows != p.col


@pytest.mark.parametrize("power", [1, 2])
@pytest.mark.parametrize("theta", [0.1, 0.19, 0.25, 0.3])
def test_uniform_grid_closed_form(orc, theta, power):
    p = pb.fd7_stretched(6, 1.0)  # pattern of a 6^3 7-point grid (values unused)
    X = pb.grid_coords(np.arange(6.0), np.arange(6.0), np.arange(6.0))
    m = orc.distance_strength(p.n, p.rp, p.col, X, theta, power)
    rows, cols, off = _offdiag(p)
    n = _counts(p)
    want = np.where(off, np.where(n[rows] * n[cols] <= 1.0 / theta ** 2, 1, 0), 3)
    assert np.array_equal(m, want.astype(np.uint8))
    # a smaller theta than 1/6 makes every connection strong
    m0 = orc.distance_strength(p.n, p.rp, p.col, X, 0.16, power)
    assert np.all(m0[off] == 1)


@pytest.mark.parametrize("power", [1, 2])
@pytest.mark.parametrize("theta", [0.02, 0.05, 0.2, 0.45])
def test_anisotropic_grid_closed_form(orc, theta, power):
    nx, nz = 5, 7
    p = pb.fd7_stretched(nz, 1.0, nx=nx, ny=nx)
    X = pb.grid_coords(np.arange(nx, dtype=float), np.arange(nx, dtype=float),
                       0.25 * np.arange(nz))
    m = orc.distance_strength(p.n, p.rp, p.col, X, theta, power)
    rows, cols, off = _offdiag(p)
    vertical = np.abs(cols - rows) == nx * nx
    q = np.zeros(p.n, dtype=np.int64)
    np.add.at(q, rows[vertical], 1)
    pcount = _counts(p) - q
    wz = 4.0 ** power
    Ld = pcount + wz * q
    w = np.where(vertical, wz, 1.0)
    strong = w * w >= theta * theta * Ld[rows] * Ld[cols]
    want = np.where(off, strong.astype(np.uint8), 3)
    assert np.array_equal(m, want.astype(np.uint8))
    if theta == 0.05 and power == 2:  # vertical strong, in-plane weak inside
        inner = (pcount[rows] == 4) & (q[rows] == 2) & (pcount[cols] == 4) & (q[cols] == 2)
        assert np.all(m[off & vertical & inner] == 1)
        assert np.all(m[off & ~vertical & inner] == 0)


@pytest.mark.parametrize("power", [1, 2])
def test_labels_depend_on_coordinates_only(orc, power):
    p = pb.q1_hex(7)
    X = pb.q1_coords(7)
    m = orc.distance_strength(p.n, p.rp, p.col, X, 0.05, power)
    # power-of-two scaling, integer translation (on an integer grid), axis permutation
    Xi = X * 7.0  # integer coordinates 1..6
    for Y in (X * 0.125, X * 1024.0, Xi + 3.0, Xi - 100.0):
        assert np.array_equal(orc.distance_strength(p.n, p.rp, p.col, Y, 0.05, power), m)
    # the full setup ignores A's values for the labels: D A D gives the same fine labels
    rng = np.random.Generator(np.random.PCG64(2))
    d = rng.uniform(0.5, 2.0, size=p.n)
    rows = np.repeat(np.arange(p.n), np.diff(p.rp))
    h1 = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, coords=X, theta=0.05, max_coarse=20,
                             dist_power=power)
    h2 = orc.OracleHierarchy(p.n, p.rp, p.col, (d[rows] * p.val) * d[p.col], coords=X,
                             theta=0.05, max_coarse=20, dist_power=power)
    assert np.array_equal(h1.levels[0].mask, m)
    assert np.array_equal(h2.levels[0].mask, m)
    assert np.array_equal(h1.levels[0].agg, h2.levels[0].agg)


def test_axis_permutation_of_a_box(orc):
    # 4 x 5 x 6 grid with spacings (1, 2, 1/2): the labels of the permuted problem are the
    # permuted labels
    sx, sy, sz = 4, 5, 6
    base = pb.fd7_stretched(sz, 1.0, nx=sx, ny=sy)
    X = pb.grid_coords(np.arange(sx) * 1.0, np.arange(sy) * 2.0, np.arange(sz) * 0.5)
    m = orc.distance_strength(base.n, base.rp, base.col, X, 0.1)
    # relabel: new axes (z, x, y) so new x-fastest order is z fastest
    perm = pb.fd7_stretched(sy, 1.0, nx=sz, ny=sx)
    Y = pb.grid_coords(np.arange(sz) * 0.5, np.arange(sx) * 1.0, np.arange(sy) * 2.0)
    mp = orc.distance_strength(perm.n, perm.rp, perm.col, Y, 0.1)
    # node (i,j,k) of the base is node (k,i,j) of the permuted grid
    def new_index(v):
        i, j, k = v % sx, (v // sx) % sy, v // (sx * sy)
        return k + sz * (i + sx * j)
    lab = {}
    rows = np.repeat(np.arange(perm.n), np.diff(perm.rp))
    for r, c, v in zip(rows, perm.col, mp):
        lab[(int(r), int(c))] = int(v)
    rows = np.repeat(np.arange(base.n), np.diff(base.rp))
    for r, c, v in zip(rows, base.col, m):
        assert lab[(new_index(int(r)), new_index(int(c)))] == int(v)


@pytest.mark.parametrize("power", [1, 2])
def test_graph_laplacian_matrix_agrees_with_classical_test(orc, power):
    """A = L^(d) of random coordinates (weights 1/d^p, diagonal summed in ascending column
    order from 0): the classical labels of A are the distance labels."""
    p = pb.q1_hex(6)
    rng = np.random.Generator(np.random.PCG64(11))
    X = pb.q1_coords(6) + rng.uniform(-0.03, 0.03, size=(p.n, 3))
    val = np.empty(p.nnz)
    for i in range(p.n):
        s, dpos = 0.0, -1
        for e in range(p.rp[i], p.rp[i + 1]):
            j = p.col[e]
            if j == i:
                dpos = e
                continue
            t = X[i] - X[j]
            d2 = 0.0
            for k in range(3):
                d2 = d2 + t[k] * t[k]
            w = 1.0 / math.sqrt(d2) if power == 1 else 1.0 / d2
            val[e] = -w
            s = s + w
        val[dpos] = s
    for theta in (0.02, 0.08, 0.15):
        assert np.array_equal(orc.strength(p.n, p.rp, p.col, val, theta),
                              orc.distance_strength(p.n, p.rp, p.col, X, theta, power))


def test_coarse_coordinates_are_centroids(orc):
    p = pb.fd7_stretched(12, 100.0)
    X = pb.fd7_coords(12, 100.0)
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, coords=X, max_coarse=10)
    assert len(h.levels) >= 3
    for l in range(len(h.levels) - 1):
        L, Ln = h.levels[l], h.levels[l + 1]
        assert Ln.coords.shape == (L.nc, 3)
        for J in range(L.nc):
            members = np.flatnonzero(L.agg == J)
            assert members.size > 0
            c = X[members] if l == 0 else L.coords[members]
            ref = np.array([sum(sorted(c[:, k].tolist())) for k in range(3)]) / members.size
            assert np.allclose(Ln.coords[J], ref, rtol=1e-15, atol=0)
            # inside the bounding box of the members (up to the rounding of sum / count:
            # three equal values summed and divided by 3 can land one ulp off)
            slack = 4e-16 * np.abs(c).max(axis=0)
            assert np.all(Ln.coords[J] >= c.min(axis=0) - slack)
            assert np.all(Ln.coords[J] <= c.max(axis=0) + slack)


def test_distance_setup_solves_stretched_problems(orc):
    cases = [(pb.fd7_stretched(14, 1000.0), pb.fd7_coords(14, 1000.0), {}),
             (pb.fd5_stretched(40, 40, 100.0), pb.fd5_coords(40, 40, 100.0), {}),
             (pb.q1_stretched_box(10), pb.q1_coords(11, 1, 1, 2),
              dict(variants=("offlmp",), cheb_boost=1.1))]
    for p, X, kw in cases:
        h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, coords=X, max_coarse=30, rtol=1e-8,
                                **kw)
        r = h.solve(pb.random_rhs(p.n, 4))
        assert r["converged"], p.name
        assert r["rel_residual"] <= 1e-8
        assert len(h.levels) >= 2


def test_distance_setup_errors(orc):
    p = pb.fd7_stretched(5, 10.0)
    X = pb.fd7_coords(5, 10.0)
    Y = X.copy()
    Y[7] = Y[8]  # nodes 7 and 8 are x-neighbours: a zero distance
    with pytest.raises(orc.OracleError) as e:
        orc.OracleHierarchy(p.n, p.rp, p.col, p.val, coords=Y, max_coarse=10)
    assert e.value.code == -1
    Y = X.copy()
    Y[3, 1] = np.nan
    with pytest.raises(orc.OracleError):
        orc.OracleHierarchy(p.n, p.rp, p.col, p.val, coords=Y, max_coarse=10)
    with pytest.raises(orc.OracleError):
        orc.OracleHierarchy(p.n, p.rp, p.col, p.val, max_coarse=10,
                            coords=np.zeros((p.n, 4)) + np.arange(p.n)[:, None])
    with pytest.raises(orc.OracleError):
        orc.OracleHierarchy(p.n, p.rp, p.col, p.val, coords=X, max_coarse=10, dist_power=3)
    # a problem that fits the coarsest level never computes labels: no error
    Y = X.copy()
    Y[7] = Y[8]
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, coords=Y, max_coarse=1000)
    assert len(h.levels) == 1
