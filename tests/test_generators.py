"""Pins of the synthetic problem generators (closed forms and the paper's printed stencil)."""
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_2103_10476_amd import problems as pb

GOLDEN = __file__.replace("test_generators.py", "golden/q1_stencil_hz_sqrt7_over_2.txt")


def _classes():
    """Offset -> neighbour class of the 27-point stencil (z is the stretched axis)."""
    out = {}
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                nz = (dx != 0) + (dy != 0) + (dz != 0)
                if nz == 0:
                    c = "diagonal"
                elif nz == 3:
                    c = "corner"
                elif nz == 2:
                    c = "xy_face" if dz == 0 else "xz_or_yz_face"
                else:
                    c = "z_edge" if dz != 0 else "x_or_y_edge"
                out[(dx, dy, dz)] = c
    return out


def _center_row(p, nint):
    """Map offset -> value for the unknown at the centre of an nint^3 interior grid."""
    c = nint // 2
    i = c + nint * (c + nint * c)
    out = {}
    for e in range(p.rp[i], p.rp[i + 1]):
        j = int(p.col[e])
        jx, jy, jz = j % nint, (j // nint) % nint, j // (nint * nint)
        out[(jx - c, jy - c, jz - c)] = float(p.val[e])
    return out


def test_q1_stencil_printed_values():
    """Sec. 1.2: 27-point stencil x 36 h_z at h_z = sqrt(7)/2 is 144, -4.5, -7.5, 12, -12, -6."""
    hz = math.sqrt(7.0) / 2.0
    p = pb.q1_hex(4, hx=1.0, hy=1.0, hz=hz)
    row = _center_row(p, 3)
    assert len(row) == 27
    printed = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        name, count, value = line.split()
        printed[name] = (int(count), float(value))
    cls = _classes()
    seen = {}
    for off, v in row.items():
        seen.setdefault(cls[off], []).append(v * 36.0 * hz)
    for name, (count, value) in printed.items():
        assert len(seen[name]) == count
        np.testing.assert_allclose(seen[name], value, rtol=1e-12, atol=1e-12)
    assert abs(sum(row.values())) < 1e-13


@pytest.mark.parametrize("hz", [Fraction(1), Fraction(2), Fraction(3, 2)])
def test_q1_stencil_closed_form(hz):
    """Sec. 1.2 closed forms: 32+64h^2, -1-2h^2, -4-2h^2, 16h^2-16, 2-8h^2, 8-8h^2 (x 36 h_z)."""
    p = pb.q1_hex(4, hx=Fraction(1), hy=Fraction(1), hz=hz)
    row = _center_row(p, 3)
    h2 = float(hz * hz)
    expect = {"diagonal": 32 + 64 * h2, "corner": -1 - 2 * h2, "xz_or_yz_face": -4 - 2 * h2,
              "z_edge": 16 * h2 - 16, "xy_face": 2 - 8 * h2, "x_or_y_edge": 8 - 8 * h2}
    cls = _classes()
    for off, v in row.items():
        assert v * 36.0 * float(hz) == pytest.approx(expect[cls[off]], abs=1e-12)


def test_q1_unit_cube_textbook_stencil():
    """h = 1 cube: the Q1 Laplacian stencil is 8/3, -1/6 (12 edge), -1/12 (8), 0 (6 axis)."""
    p = pb.q1_hex(4, hx=Fraction(1), hy=Fraction(1), hz=Fraction(1))
    row = _center_row(p, 3)
    for off, v in row.items():
        nz = sum(o != 0 for o in off)
        expect = {0: 8 / 3, 1: 0.0, 2: -1 / 6, 3: -1 / 12}[nz]
        assert v == pytest.approx(expect, abs=1e-15)
        if nz == 1:
            assert v == 0.0  # exact zero, stored


def _check_sym_rowsums(p, interior_zero=True):
    d = p.to_dense() if p.n <= 5000 else None
    rows = np.repeat(np.arange(p.n), np.diff(p.rp))
    assert np.all(np.diff(p.col)[np.diff(rows) == 0] > 0)  # ascending columns
    assert np.all(p.col[np.searchsorted(rows, np.arange(p.n))] <= np.arange(p.n))
    if d is not None:
        assert np.array_equal(d, d.T)
    rs = np.bincount(rows, weights=p.val, minlength=p.n)
    scale = np.bincount(rows, weights=np.abs(p.val), minlength=p.n)
    assert np.all(rs >= -1e-12 * scale)
    return rs, scale


def test_fd5_c1_shape_and_symmetry():
    p = pb.workload("fd5_64x64_a100")
    assert p.n == 4096 and p.nnz == 4096 + 2 * (63 * 64 + 63 * 64) == 20224
    rs, scale = _check_sym_rowsums(p)
    # interior rows (no boundary neighbour) sum to zero
    g = np.arange(p.n)
    x, y = g % 64, g // 64
    inner = (x > 0) & (x < 63) & (y > 0) & (y < 63)
    assert np.all(np.abs(rs[inner]) <= 1e-12 * scale[inner])
    assert np.all(rs[~inner] > 0)
    # finest y cell aspect 1:100
    hy = pb.graded_spacing(64, 100.0)
    assert hy[0] * 100 == pytest.approx(1 / 65) and hy[-1] == pytest.approx(1 / 65)


@pytest.mark.parametrize("n,nnz", [(16, 16**3 + 6 * 15 * 16**2), (128, 14581760),
                                   (160, 28518400)])
def test_fd7_nnz_closed_form(n, nnz):
    p = pb.fd7_stretched(n, 1000.0)
    assert p.n == n**3 and p.nnz == nnz


def test_fd7_symmetric_small():
    p = pb.fd7_stretched(12, 1000.0)
    _check_sym_rowsums(p)


def test_q1_randkappa_shape():
    p = pb.q1_random_kappa(10, seed=3)
    assert p.n == 9**3 and p.nnz == (3 * 9 - 2) ** 3
    _check_sym_rowsums(p)
    d = p.to_dense()
    # M-matrix sign pattern of Q1 on cubes: off-diagonals <= 0
    off = d - np.diag(np.diag(d))
    assert np.all(off <= 0)


def test_rhs_seeded():
    a = pb.random_rhs(1000, 2)
    b = pb.random_rhs(1000, 2)
    assert np.array_equal(a, b) and a.min() >= -1 and a.max() < 1
    assert not np.array_equal(a, pb.random_rhs(1000, 3))


def test_serving_requests_seeded():
    r1 = pb.serving_requests(32)
    r2 = pb.serving_requests(32)
    assert r1 == r2
    assert all(16 <= r["side"] <= 96 for r in r1)
    assert {r["kind"] for r in r1} == {"fd7", "q1"}


# ---- general hexahedral Q1 meshes (Sec. 3.2-3.3, App. A-B) --------------------------------

def _dense(p):
    d = np.zeros((p.n, p.n))
    d[np.repeat(np.arange(p.n), np.diff(p.rp)), p.col] = p.val
    return d


def _uniform_nodes(ne, lengths=(1.0, 1.0, 1.0)):
    axes = [np.arange(ne + 1) * (L / ne) for L in lengths]
    Z, Y, X = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    return np.stack([X, Y, Z], axis=-1)


def test_q1_mesh_on_uniform_bricks_is_the_exact_stiffness():
    # Gauss quadrature is exact on bricks: the rational-arithmetic Q1 cube, to rounding
    p0 = pb.q1_hex(6)
    p, rhs, X = pb.q1_mesh(_uniform_nodes(6))
    assert np.array_equal(p.rp, p0.rp) and np.array_equal(p.col, p0.col)
    assert np.abs(p.val - p0.val).max() <= 4e-15 * np.abs(p0.val).max()
    assert np.all(rhs == 0.0)
    assert np.allclose(X, pb.q1_coords(6), rtol=0, atol=1e-15)
    # a 2 x 1 x 3 brick mesh against the closed-form element of q1_element_matrix
    p1 = pb.q1_hex(5, hx=Fraction(2, 5), hy=Fraction(1, 5), hz=Fraction(3, 5))
    q, _, _ = pb.q1_mesh(_uniform_nodes(5, (2.0, 1.0, 3.0)))
    assert np.abs(q.val - p1.val).max() <= 4e-15 * np.abs(p1.val).max()


def test_q1_mesh_patch_test_on_perturbed_mesh():
    """Isoparametric Q1 reproduces linear fields on any hexahedral mesh: with linear boundary
    data and no forcing the discrete solution is the linear field at every interior node."""
    nodes = pb.perturbed_cube_nodes(7, seed=3, lengths=(1.0, 2.0, 5.0))
    lin = lambda x, y, z: 1.0 + 2.0 * x - 0.5 * y + 0.25 * z
    p, rhs, X = pb.q1_mesh(nodes, 0.0, lin)
    u = np.linalg.solve(_dense(p), rhs)
    assert np.abs(u - lin(X[:, 0], X[:, 1], X[:, 2])).max() <= 1e-11
    # trilinear data is reproduced only on bricks (the stretched-cube meshes)
    q, rb, Y = pb.q1_mesh(pb.stretched_cube_nodes(1, 5, 10, ne=6), 0.0, pb.u_trilinear)
    v = np.linalg.solve(_dense(q), rb)
    assert np.abs(v - pb.u_trilinear(Y[:, 0], Y[:, 1], Y[:, 2])).max() <= 1e-10


def test_q1_mesh_reaction_row_sums_are_lumped_masses():
    """With u = 1 everywhere the stiffness part vanishes row by row, so each interior row of
    [A_II A_IB] sums to reaction * integral of the node's hat function, which on a tensor mesh of
    bricks is the product of half the neighbouring widths per axis."""
    r = 1.0  # (a tiny reaction would leave the row sums inside the stiffness's rounding)
    nodes = pb.stretched_cube_nodes(5, 5, 10, ne=6)
    p, rhs, X = pb.q1_mesh(nodes, r, lambda x, y, z: np.ones_like(x))
    rows = _dense(p).sum(axis=1) - rhs          # A_II 1 + A_IB 1
    ax = [pb.linear_sizes(6, 0.1, k / 10.0) for k in (5, 5, 10)]
    half = [0.5 * (a[2:] - a[:-2]) for a in ax]  # interior nodes 1..5 of each axis
    want = r * np.einsum("k,j,i->kji", half[2], half[1], half[0]).reshape(-1)
    assert np.allclose(rows, want, rtol=1e-11, atol=0)


def test_q1_mesh_spd_and_symmetric():
    p, _, _ = pb.perturbed_cube(5, seed=1)
    d = _dense(p)
    assert np.array_equal(d, d.T)
    assert np.linalg.eigvalsh(d).min() > 0
    q, _, _ = pb.stretched_cube(1, 1, 10, 1e2, ne=5)
    e = _dense(q)
    assert np.abs(e - e.T).max() <= 1e-15 * np.abs(e).max()
    assert np.linalg.eigvalsh(e).min() > 0


def test_perturbed_and_stretched_node_recipes():
    ne = 12
    nodes = pb.perturbed_cube_nodes(ne, seed=7)
    base = _uniform_nodes(ne)
    dev = (nodes / np.array([1.0, 1.0, 100.0]) - base) * ne
    assert dev.min() >= 0.0 and dev.max() < 0.2 + 1e-12
    assert np.array_equal(nodes, pb.perturbed_cube_nodes(ne, seed=7))
    assert not np.array_equal(nodes, pb.perturbed_cube_nodes(ne, seed=8))
    for k in (1, 5, 10):
        x = pb.linear_sizes(60, 0.1, k / 10.0)
        h = np.diff(x)
        assert abs(h[0] - 0.1) < 1e-15 and abs(h[-1] - k / 10.0) < 1e-15
        assert abs(x[-1] - 3.0 * (k + 1)) < 1e-12   # the App. B domain length
        assert np.allclose(np.diff(h), (k / 10.0 - 0.1) / 59, atol=1e-15)
    assert len(pb.STRETCH_CONFIGS) == 10 and len(pb.STRETCH_SIGMAS) == 5
