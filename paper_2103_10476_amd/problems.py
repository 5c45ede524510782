"""Seeded synthetic problems for the SA-AMG solver: matrices and right-hand sides.

This module builds inputs only.  It holds none of the method's arithmetic and is the one
module that both the GPU path and the CPU oracle receive their inputs from.

All matrices are CSR with int32 row pointers and column indices (columns strictly ascending
within each row, diagonal always stored) and float64 values.  Unknowns are numbered in
natural lexicographic order with x running fastest.  Dirichlet boundary nodes are
eliminated: only interior unknowns are kept, and couplings to boundary nodes contribute to
the diagonal only.

Problem families (the paper's test families are FE cubes with stretched or perturbed
meshes, a heterogeneous reservoir model and wind-turbine pressure systems, Sec. 3; none of
their meshes or data are available, so these are synthetic stand-ins of the same character):

* ``fd5_stretched``  2-D 5-point finite-volume Laplacian, y spacing graded geometrically.
* ``fd7_stretched``  3-D 7-point finite-volume Laplacian, z spacing graded geometrically
  (the character of the stretched cube of Sec. 3.2 and the stretched wind meshes of Sec. 3.4).
* ``q1_hex``         3-D 27-point trilinear (Q1) hexahedral stiffness matrix on a tensor mesh
  with per-element coefficient kappa (the 27-point stencil of Sec. 1.2; random kappa over six
  decades stands in for the heterogeneous permeability of Sec. 3.3).
* ``periodic_*``     small periodic stencils used by the tests (circulant examples of Sec. 2.1).
"""
from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction
import itertools

import numpy as np


@dataclass
class CsrProblem:
    """A square sparse matrix in CSR form plus a description of how it was made."""

    n: int
    rp: np.ndarray   # int32 [n+1]
    col: np.ndarray  # int32 [nnz]
    val: np.ndarray  # float64 [nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.rp[-1])

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.rp))
        d[rows, self.col] = self.val
        return d


def _csr_from_offsets(shape, offsets, coeffs, name):
    """Assemble CSR from a structured stencil.

    ``shape`` = unknowns per axis (x first).  ``offsets`` is a list of integer offset tuples
    and ``coeffs[t]`` an array of the grid's shape holding the coefficient that couples each
    unknown to its neighbour at ``offsets[t]``.  Entries whose neighbour falls outside the
    grid are not stored.  Offsets must be listed so that the linear index offset ascends,
    which makes the columns of every row ascend.
    """
    dims = len(shape)
    n = int(np.prod(shape))
    strides = [1]
    for d in range(dims - 1):
        strides.append(strides[-1] * shape[d])
    lin = [sum(o[d] * strides[d] for d in range(dims)) for o in offsets]
    order = np.argsort(lin, kind="stable")
    offsets = [offsets[t] for t in order]
    coeffs = [coeffs[t] for t in order]
    # grid coordinates of every unknown, C order over reversed axes so x is fastest
    grids = np.meshgrid(*[np.arange(s) for s in reversed(shape)], indexing="ij")
    coords = [g.reshape(-1) for g in reversed(grids)]  # coords[d] for axis d, x fastest
    valid = []
    for o in offsets:
        ok = np.ones(n, dtype=bool)
        for d in range(dims):
            c = coords[d] + o[d]
            ok &= (c >= 0) & (c < shape[d])
        valid.append(ok)
    counts = np.zeros(n, dtype=np.int64)
    for ok in valid:
        counts += ok
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    nnz = int(rp[-1])
    if nnz >= 2**31:
        raise ValueError("nnz too large for int32 indices")
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    pos = rp[:-1].copy()
    idx = np.arange(n, dtype=np.int64)
    for t, o in enumerate(offsets):
        ok = valid[t]
        dst = pos[ok]
        col[dst] = (idx[ok] + lin[order[t]]).astype(np.int32)
        val[dst] = np.asarray(coeffs[t]).reshape(-1)[ok]
        pos[ok] += 1
    return CsrProblem(n, rp.astype(np.int32), col, val, name)


def graded_spacing(nint: int, aspect: float) -> np.ndarray:
    """Cell widths h_k = h * aspect**(k/nint - 1), k = 0..nint, with h = 1/(nint+1).

    The interval below interior node k (1-based) is h_{k-1}, the one above is h_k.  The
    finest cell, at the low boundary, has aspect 1:aspect against the uniform spacing h;
    the last one is 1:1.
    """
    h = 1.0 / (nint + 1)
    k = np.arange(nint + 1, dtype=np.float64)
    return h * aspect ** (k / nint - 1.0)


def fd5_stretched(nx: int = 64, ny: int = 64, aspect: float = 100.0) -> CsrProblem:
    """2-D 5-point finite-volume Laplacian, x uniform (h = 1/(nx+1)), y graded.

    Row (i, j): west/east coupling -dy_j/h, south -h/h_{j-1}, north -h/h_j with
    dy_j = (h_{j-1} + h_j)/2; the diagonal is the sum of the magnitudes of all couplings,
    including those to eliminated boundary nodes.  Symmetric by construction.
    """
    h = 1.0 / (nx + 1)
    hy = graded_spacing(ny, aspect)                 # ny+1 widths
    dy = 0.5 * (hy[:-1] + hy[1:])                   # ny interior control-volume heights
    cx = dy / h                                     # per row j
    cs = h / hy[:-1]                                # coupling to j-1 (below)
    cn = h / hy[1:]                                 # coupling to j+1 (above)
    shape = (nx, ny)
    J = np.broadcast_to(np.arange(ny)[:, None], (ny, nx))  # [y, x] layout
    cxg = cx[J]
    csg = cs[J]
    cng = cn[J]
    diag = ((cxg + cxg) + csg) + cng
    offs = [(0, -1), (-1, 0), (0, 0), (1, 0), (0, 1)]
    coeffs = [-csg, -cxg, diag, -cxg, -cng]
    return _csr_from_offsets(shape, offs, coeffs, f"fd5_stretched_{nx}x{ny}_a{aspect:g}")


def fd7_stretched(n: int = 128, aspect: float = 1000.0, nx: int | None = None,
                  ny: int | None = None) -> CsrProblem:
    """3-D 7-point finite-volume Laplacian on n^3 unknowns, x/y uniform, z graded.

    x/y couplings in layer k: -dz_k (face area h*dz_k over distance h); z couplings:
    -h^2/h_{k-1} (below), -h^2/h_k (above); diagonal = sum of coupling magnitudes including
    those to the eliminated boundary.  Symmetric by construction.
    """
    nx = n if nx is None else nx
    ny = n if ny is None else ny
    nz = n
    h = 1.0 / (nx + 1)
    hz = graded_spacing(nz, aspect)
    dz = 0.5 * (hz[:-1] + hz[1:])
    cxy = dz                                        # (h*dz)/h, kept exact as dz
    cdn = (h * h) / hz[:-1]
    cup = (h * h) / hz[1:]
    K = np.broadcast_to(np.arange(nz)[:, None, None], (nz, ny, nx))
    cxyg = cxy[K]
    cdng = cdn[K]
    cupg = cup[K]
    diag = ((((cxyg + cxyg) + cxyg) + cxyg) + cdng) + cupg
    offs = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    coeffs = [-cdng, -cxyg, -cxyg, diag, -cxyg, -cxyg, -cupg]
    return _csr_from_offsets((nx, ny, nz), offs, coeffs,
                             f"fd7_stretched_{nx}x{ny}x{nz}_a{aspect:g}")


def cd7_upwind(n: int = 64, aspect: float = 1.0, beta=(1.0, 0.5, 0.25),
               nx: int | None = None, ny: int | None = None) -> CsrProblem:
    """3-D convection-diffusion -lap(u) + beta . grad(u), finite volumes on the grid of
    ``fd7_stretched(n, aspect)`` with first-order upwinding of the constant velocity ``beta``.

    The diffusive couplings are those of ``fd7_stretched``.  A face with flux q = beta . n * area
    adds q to the diagonal when q > 0 (outflow) and -|q| to the coupling with the neighbour
    across it when q < 0 (inflow); inflow from an eliminated boundary node is dropped.  The
    matrix is nonsymmetric with a symmetric pattern, an M-matrix, diagonally dominant.
    (A synthetic nonsymmetric family standing in for the wind-turbine pressure systems of
    Sec. 3.4, which are not available.)"""
    nx = n if nx is None else nx
    ny = n if ny is None else ny
    nz = n
    bx, by, bz = (float(v) for v in beta)
    h = 1.0 / (nx + 1)
    hz = graded_spacing(nz, aspect)
    dz = 0.5 * (hz[:-1] + hz[1:])
    cxy = dz
    cdn = (h * h) / hz[:-1]
    cup = (h * h) / hz[1:]
    K = np.broadcast_to(np.arange(nz)[:, None, None], (nz, ny, nx))
    axy = (h * dz)[K]              # area of an x or y face in layer k
    az = h * h                     # area of a z face
    qx, qy, qz = bx * axy, by * axy, bz * az
    # per direction: inflow couplings (to the upstream neighbour) and outflow on the diagonal
    west = -cxy[K] - np.maximum(qx, 0.0)    # neighbour i-1 is upstream when bx > 0
    east = -cxy[K] - np.maximum(-qx, 0.0)
    south = -cxy[K] - np.maximum(qy, 0.0)
    north = -cxy[K] - np.maximum(-qy, 0.0)
    down = -cdn[K] - max(qz, 0.0)
    up = -cup[K] - max(-qz, 0.0)
    diff = ((((cxy[K] + cxy[K]) + cxy[K]) + cxy[K]) + cdn[K]) + cup[K]
    conv = (np.abs(qx) + np.abs(qy)) + abs(qz)   # outflow through the downstream faces
    diag = diff + conv
    offs = [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    coeffs = [down, south, west, diag, east, north, up]
    return _csr_from_offsets((nx, ny, nz), offs, coeffs,
                             f"cd7_upwind_{nx}x{ny}x{nz}_a{aspect:g}_b{bx:g},{by:g},{bz:g}")


def q1_element_matrix(hx, hy, hz):
    """Trilinear hex element stiffness for -div(grad u) on an hx*hy*hz brick (kappa = 1).

    K = (hy*hz/hx) k(x)m(x)m + (hx*hz/hy) m(x)k(x)m + (hx*hy/hz) m(x)m(x)k with the 1-D
    stiffness k = [[1,-1],[-1,1]] and mass m = [[1/3,1/6],[1/6,1/3]].  Local node index
    a = ax + 2*ay + 4*az.  Arguments may be Fractions (exact) or floats.
    """
    one = Fraction(1) if isinstance(hx, Fraction) else 1.0
    k1 = [[one, -one], [-one, one]]
    m1 = [[one / 3, one / 6], [one / 6, one / 3]]
    K = [[None] * 8 for _ in range(8)]
    for a in range(8):
        ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
        for b in range(8):
            bx, by, bz = b & 1, (b >> 1) & 1, (b >> 2) & 1
            K[a][b] = ((hy * hz / hx) * k1[ax][bx] * m1[ay][by] * m1[az][bz]
                       + (hx * hz / hy) * m1[ax][bx] * k1[ay][by] * m1[az][bz]
                       + (hx * hy / hz) * m1[ax][bx] * m1[ay][by] * k1[az][bz])
    return K


def q1_hex(ne: int = 100, kappa: np.ndarray | None = None, hx=None, hy=None, hz=None,
           nex: int | None = None, ney: int | None = None) -> CsrProblem:
    """27-point Q1 stiffness on an ne^3 element tensor mesh, Dirichlet boundary eliminated.

    ``kappa`` holds one coefficient per element (element index x fastest); default 1.
    Element sizes default to 1/ne (the unit cube).  The element matrix is formed exactly in
    rational arithmetic when the sizes are Fractions, so entries that vanish exactly (the
    axis neighbours of the isotropic cube) are stored as exact zeros.  The unknowns are the
    (ne-1)^3 interior nodes, so the matrix has (3(ne-1)-2)^3 stored entries.
    """
    nex = ne if nex is None else nex
    ney = ne if ney is None else ney
    nez = ne
    if hx is None:
        hx = hy = hz = Fraction(1, ne)
    K = q1_element_matrix(hx, hy, hz)
    Kf = np.array([[float(K[a][b]) for b in range(8)] for a in range(8)])
    if kappa is None:
        kappa = np.ones(nex * ney * nez)
    kap = np.asarray(kappa, dtype=np.float64).reshape(nez, ney, nex)   # [z, y, x]
    nix, niy, niz = nex - 1, ney - 1, nez - 1
    # interior node (i,j,k) 1-based; element (ex,ey,ez) 0-based spans nodes ex..ex+1
    offs = list(itertools.product((-1, 0, 1), repeat=3))             # (dx,dy,dz)
    coeffs = []
    ii = np.arange(1, nix + 1)
    jj = np.arange(1, niy + 1)
    kk = np.arange(1, niz + 1)
    for (dx, dy, dz) in offs:
        c = np.zeros((niz, niy, nix))
        for (a, b, cc) in itertools.product((0, 1), repeat=3):
            # element with lower corner (i-1+a, j-1+b, k-1+cc); node local coords (1-a,..)
            lx, ly, lz = 1 - a, 1 - b, 1 - cc
            mx, my, mz = lx + dx, ly + dy, lz + dz
            if not (0 <= mx <= 1 and 0 <= my <= 1 and 0 <= mz <= 1):
                continue
            la = lx + 2 * ly + 4 * lz
            lb = mx + 2 * my + 4 * mz
            kv = kap[np.ix_(kk - 1 + cc, jj - 1 + b, ii - 1 + a)]
            c = c + kv * Kf[la, lb]
        coeffs.append(c)
    # coeffs arrays are [z,y,x]; _csr_from_offsets wants arrays in its own x-fastest layout
    offs_xyz = [(dx, dy, dz) for (dx, dy, dz) in offs]
    return _csr_from_offsets((nix, niy, niz), offs_xyz, coeffs,
                             f"q1_hex_{nex}x{ney}x{nez}")


def q1_random_kappa(ne: int = 100, seed: int = 3, lo: float = -3.0, hi: float = 3.0):
    """Q1 cube with kappa_e = 10**u_e, u_e ~ U[lo, hi] i.i.d. from numpy PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.uniform(lo, hi, size=ne ** 3)
    p = q1_hex(ne, kappa=10.0 ** u)
    p.name = f"q1_randkappa_{ne}_s{seed}"
    return p


def q1_stretched_box(nint: int = 24, hz=Fraction(2)) -> CsrProblem:
    """Q1 Poisson on 1 x 1 x hz elements (kappa = 1), nint^3 interior unknowns."""
    ne = nint + 1
    p = q1_hex(ne, hx=Fraction(1), hy=Fraction(1), hz=hz)
    p.name = f"q1_box_{nint}_hz{hz}"
    return p


# ---------------------------------------------------------------------------------------
# Q1 on general hexahedral meshes (the test families of Sec. 3.2-3.3 and App. A-B)
# ---------------------------------------------------------------------------------------

def _q1_reference():
    """Trilinear shape functions at the 2x2x2 Gauss points of [-1,1]^3 (weights 1).

    Returns (N [8 gp, 8 nodes], dN [8 gp, 8 nodes, 3]); local node a = ax + 2 ay + 4 az sits
    at reference corner (2ax-1, 2ay-1, 2az-1)."""
    g = 1.0 / np.sqrt(3.0)
    corners = np.array([[2 * (a & 1) - 1, 2 * ((a >> 1) & 1) - 1, 2 * ((a >> 2) & 1) - 1]
                        for a in range(8)], dtype=np.float64)
    pts = np.array([[sx * g, sy * g, sz * g] for sz in (-1, 1) for sy in (-1, 1)
                    for sx in (-1, 1)])
    N = np.empty((8, 8))
    dN = np.empty((8, 8, 3))
    for q, (x, y, z) in enumerate(pts):
        fx = 1.0 + corners[:, 0] * x
        fy = 1.0 + corners[:, 1] * y
        fz = 1.0 + corners[:, 2] * z
        N[q] = fx * fy * fz / 8.0
        dN[q, :, 0] = corners[:, 0] * fy * fz / 8.0
        dN[q, :, 1] = fx * corners[:, 1] * fz / 8.0
        dN[q, :, 2] = fx * fy * corners[:, 2] / 8.0
    return N, dN


def q1_mesh(nodes: np.ndarray, reaction: float = 0.0, u_dirichlet=None, name: str = "q1_mesh"):
    """Q1 (trilinear) finite elements for reaction*u - div(grad u) = 0 on a structured
    hexahedral mesh, Dirichlet data on the whole boundary eliminated.

    ``nodes`` has shape (nz+1, ny+1, nx+1, 3): the position of every mesh node (x index
    fastest); elements are the cells of this logical grid and may be any non-degenerate
    hexahedra.  Element matrices use 2x2x2 Gauss quadrature of the stiffness and of
    ``reaction`` times the mass (exact on axis-aligned bricks).  Element contributions are added
    element by element in element order (x fastest), local pairs in (a, b) order.  The unknowns
    are the interior nodes in x-fastest order; the pattern is the 27-point stencil, every
    entry stored.  ``u_dirichlet(x, y, z)`` gives the boundary values; the right-hand side is
    then -A_IB u_D (zero forcing), otherwise the returned rhs is zero.

    Returns (CsrProblem, rhs, coords) with coords the interior nodes' positions (n x 3)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    nz1, ny1, nx1, _ = nodes.shape
    nx, ny, nz = nx1 - 1, ny1 - 1, nz1 - 1
    if min(nx, ny, nz) < 2:
        raise ValueError("need at least 2 elements per direction")
    flat = nodes.reshape(-1, 3)
    gid = np.arange(nx1 * ny1 * nz1).reshape(nz1, ny1, nx1)
    interior = np.full(gid.size, -1, dtype=np.int64)
    inner = gid[1:-1, 1:-1, 1:-1].reshape(-1)
    interior[inner] = np.arange(inner.size)
    # element -> 8 global nodes, local a = ax + 2 ay + 4 az
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ex, ey, ez = ex.reshape(-1), ey.reshape(-1), ez.reshape(-1)
    conn = np.stack([gid[ez + ((a >> 2) & 1), ey + ((a >> 1) & 1), ex + (a & 1)]
                     for a in range(8)], axis=1)                        # (E, 8)
    X = flat[conn]                                                      # (E, 8, 3)
    Nq, dNq = _q1_reference()
    E = conn.shape[0]
    XT = np.ascontiguousarray(X.transpose(0, 2, 1))                     # (E, 3, 8)
    K = np.zeros((E, 8, 8))
    for q in range(8):
        J = XT @ dNq[q]                                                 # dx_i / dxi_j
        det = np.linalg.det(J)
        if not np.all(det > 0.0):
            raise ValueError("inverted or degenerate element")
        G = dNq[q] @ np.linalg.inv(J)                                   # grad N_a (E, 8, 3)
        K += det[:, None, None] * (G @ G.transpose(0, 2, 1))
        if reaction != 0.0:
            K += (reaction * det)[:, None, None] * np.outer(Nq[q], Nq[q])[None]
    # the interior pattern and, per row, the position of each of the 27 offsets
    nix, niy, niz = nx - 1, ny - 1, nz - 1
    offs = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    dummy = [np.zeros((niz, niy, nix)) for _ in offs]
    pat = _csr_from_offsets((nix, niy, niz), offs, dummy, name)
    n = pat.n
    ii = np.arange(n)
    cx, cy, cz = ii % nix, (ii // nix) % niy, ii // (nix * niy)
    slot = np.full((n, 27), -1, dtype=np.int64)
    cnt = np.zeros(n, dtype=np.int64)
    for t, (dx, dy, dz) in enumerate(offs):   # offsets in ascending linear order
        ok = ((cx + dx >= 0) & (cx + dx < nix) & (cy + dy >= 0) & (cy + dy < niy)
              & (cz + dz >= 0) & (cz + dz < niz))
        slot[ok, t] = pat.rp[:-1][ok] + cnt[ok]
        cnt += ok
    gpos = flat  # node positions by global id
    gi = np.repeat(conn[:, :, None], 8, axis=2).reshape(-1)             # row node of (e,a,b)
    gj = np.repeat(conn[:, None, :], 8, axis=1).reshape(-1)             # column node
    kv = K.reshape(-1)
    ri, cj = interior[gi], interior[gj]
    both = (ri >= 0) & (cj >= 0)
    # offset of the column node from the row node, in grid steps
    def grid_xyz(g):
        return g % nx1, (g // nx1) % ny1, g // (nx1 * ny1)
    ax_, ay_, az_ = grid_xyz(gi[both])
    bx_, by_, bz_ = grid_xyz(gj[both])
    t = (bx_ - ax_ + 1) + 3 * (by_ - ay_ + 1) + 9 * (bz_ - az_ + 1)
    pos = slot[ri[both], t]
    val = np.bincount(pos, weights=kv[both], minlength=pat.nnz)
    rhs = np.zeros(n)
    if u_dirichlet is not None:
        bnd = (ri >= 0) & (cj < 0)
        xb = gpos[gj[bnd]]
        ub = u_dirichlet(xb[:, 0], xb[:, 1], xb[:, 2])
        rhs = -np.bincount(ri[bnd], weights=kv[bnd] * ub, minlength=n)
    prob = CsrProblem(n, pat.rp, pat.col, val, name)
    return prob, rhs, flat[inner].copy()


def q1_elasticity(nodes: np.ndarray, young: float = 1.0, poisson: float = 0.3,
                  fixed: np.ndarray | None = None, name: str = "q1_elasticity"):
    """3-D linear elasticity with trilinear (Q1) hexahedra on a structured mesh: 3 unknowns
    per node (displacements x, y, z), numbered node-major (dof = 3 node + component) over the
    free nodes in x-fastest node order.

    Element matrices K_e = sum over the 2x2x2 Gauss points of det(J) B^T C B, C the isotropic
    elasticity matrix of (young, poisson) in Voigt order (xx, yy, zz, yz, xz, xy) with
    engineering shear strains.  ``fixed`` (a boolean per mesh node, shape of nodes[..., 0])
    marks clamped nodes, eliminated with zero displacement; by default the face x = 0.  The
    pattern holds every 3x3 block between nodes of a common element, all entries stored.

    Returns (CsrProblem, coords of the free nodes (m x 3), rigid-body modes (n x 6): the
    translations x, y, z and the rotations about z, x, y (-y, x, 0), (0, -z, y), (z, 0, -x))."""
    nodes = np.asarray(nodes, dtype=np.float64)
    nz1, ny1, nx1, _ = nodes.shape
    nx, ny, nz = nx1 - 1, ny1 - 1, nz1 - 1
    if fixed is None:
        fixed = np.zeros((nz1, ny1, nx1), dtype=bool)
        fixed[:, :, 0] = True
    fixed = np.asarray(fixed, dtype=bool).reshape(-1)
    flat = nodes.reshape(-1, 3)
    nn = flat.shape[0]
    free = np.flatnonzero(~fixed)
    nid = np.full(nn, -1, dtype=np.int64)
    nid[free] = np.arange(free.size)
    gid = np.arange(nn).reshape(nz1, ny1, nx1)
    ez, ey, ex = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ex, ey, ez = ex.reshape(-1), ey.reshape(-1), ez.reshape(-1)
    conn = np.stack([gid[ez + ((a >> 2) & 1), ey + ((a >> 1) & 1), ex + (a & 1)]
                     for a in range(8)], axis=1)
    X = flat[conn]
    XT = np.ascontiguousarray(X.transpose(0, 2, 1))
    lam = young * poisson / ((1.0 + poisson) * (1.0 - 2.0 * poisson))
    mu = young / (2.0 * (1.0 + poisson))
    Cm = np.zeros((6, 6))
    Cm[:3, :3] = lam
    Cm[[0, 1, 2], [0, 1, 2]] += 2.0 * mu
    Cm[[3, 4, 5], [3, 4, 5]] = mu
    _, dNq = _q1_reference()
    E = conn.shape[0]
    K = np.zeros((E, 24, 24))
    for q in range(8):
        J = XT @ dNq[q]
        det = np.linalg.det(J)
        if not np.all(det > 0.0):
            raise ValueError("inverted or degenerate element")
        G = dNq[q] @ np.linalg.inv(J)                       # (E, 8, 3) shape gradients
        B = np.zeros((E, 6, 24))
        for a in range(8):
            gx, gy, gz = G[:, a, 0], G[:, a, 1], G[:, a, 2]
            B[:, 0, 3 * a] = gx
            B[:, 1, 3 * a + 1] = gy
            B[:, 2, 3 * a + 2] = gz
            B[:, 3, 3 * a + 1] = gz
            B[:, 3, 3 * a + 2] = gy
            B[:, 4, 3 * a] = gz
            B[:, 4, 3 * a + 2] = gx
            B[:, 5, 3 * a] = gy
            B[:, 5, 3 * a + 1] = gx
        K += det[:, None, None] * (B.transpose(0, 2, 1) @ (Cm @ B))
    # node graph: nodes sharing an element; dof pattern = 3x3 blocks
    gi = np.repeat(conn[:, :, None], 8, axis=2).reshape(-1)
    gj = np.repeat(conn[:, None, :], 8, axis=1).reshape(-1)
    keep = (nid[gi] >= 0) & (nid[gj] >= 0)
    pairs = np.unique(nid[gi[keep]] * free.size + nid[gj[keep]])
    prow, pcol = pairs // free.size, pairs % free.size
    m = free.size
    ncnt = np.bincount(prow, minlength=m)
    nrp = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(ncnt, out=nrp[1:])
    n = 3 * m
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = np.repeat(3 * ncnt, 3).cumsum()
    nnz = int(rp[-1])
    col = np.empty(nnz, dtype=np.int32)
    for c in range(3):           # row (node I, component c): blocks J ascending, components
        r = 3 * np.arange(m) + c
        base = rp[r]
        for b in range(3):
            idx = base[prow] + 3 * (np.arange(pairs.size) - nrp[prow]) + b
            col[idx] = (3 * pcol + b).astype(np.int32)
    # scatter element entries: position of (node I comp a, node J comp b)
    slot_of_pair = np.searchsorted(pairs, nid[gi[keep]] * free.size + nid[gj[keep]])
    ks = K.reshape(E, 8, 3, 8, 3).transpose(0, 1, 3, 2, 4).reshape(-1, 3, 3)[keep]
    I = nid[gi[keep]]
    val = np.zeros(nnz)
    for a in range(3):
        for b in range(3):
            pos = rp[3 * I + a] + 3 * (slot_of_pair - nrp[I]) + b
            val += np.bincount(pos, weights=ks[:, a, b], minlength=nnz)
    prob = CsrProblem(n, rp.astype(np.int32), col, val, name)
    xyz = flat[free]
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    one, zero = np.ones(m), np.zeros(m)
    modes = [(one, zero, zero), (zero, one, zero), (zero, zero, one),
             (-y, x, zero), (zero, -z, y), (z, zero, -x)]
    rbm = np.stack([np.stack(md, axis=1).reshape(-1) for md in modes], axis=1)
    return prob, xyz.copy(), rbm


def elastic_beam(nx: int = 40, ny: int = 8, nz: int = 8, length: float = 5.0,
                 stretch: float = 1.0, young: float = 1.0, poisson: float = 0.3):
    """A cantilever: nx x ny x nz Q1 elements on [0, length] x [0, 1] x [0, 1] (the z
    spacing graded by ``stretch`` like ``graded_spacing``), clamped at x = 0."""
    ax = np.linspace(0.0, length, nx + 1)
    ay = np.linspace(0.0, 1.0, ny + 1)
    if stretch == 1.0:
        az = np.linspace(0.0, 1.0, nz + 1)
    else:
        h = stretch ** (np.arange(nz, dtype=np.float64) / max(nz - 1, 1))
        az = np.concatenate([[0.0], np.cumsum(h / h.sum())])
    Z, Y, Xg = np.meshgrid(az, ay, ax, indexing="ij")
    nodes = np.stack([Xg, Y, Z], axis=-1)
    return q1_elasticity(nodes, young, poisson,
                         name=f"elastic_beam_{nx}x{ny}x{nz}_s{stretch:g}")


def u_trilinear(x, y, z):
    """Boundary data of Sec. 3.2-3.3: 1 + x + y + z + xy + xz + yz + xyz."""
    return 1.0 + x + y + z + x * y + x * z + y * z + x * y * z


def perturbed_cube_nodes(ne: int = 60, seed: int = 0, amp: float = 0.2,
                         lengths=(1.0, 1.0, 100.0)) -> np.ndarray:
    """Mesh nodes of the randomly perturbed cube (Sec. 3.2, App. A).

    A uniform grid of ne elements per direction on [0,1]^3; every node coordinate is moved by
    amp * u / ne with u ~ U[0,1) (three draws per node, in node order x fastest, x then y
    then z, from numpy PCG64(seed)); then each axis is scaled by ``lengths`` (z by 100, the
    100:1 stretching).  The paper's meshes come from a mesh generator's random stream that is
    not available; this reproduces the recipe, not those meshes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = np.arange(ne + 1, dtype=np.float64) / ne
    Z, Y, Xg = np.meshgrid(g, g, g, indexing="ij")
    base = np.stack([Xg, Y, Z], axis=-1)                               # (z, y, x, 3)
    u = rng.uniform(0.0, 1.0, size=base.shape)
    pts = (base + amp * u / ne) * np.asarray(lengths, dtype=np.float64)
    return pts


def linear_sizes(ne: int, first: float, last: float) -> np.ndarray:
    """Node positions along an axis of ne elements whose sizes vary linearly from ``first``
    to ``last`` (summed from 0.0 in element order)."""
    h = first + (last - first) * np.arange(ne, dtype=np.float64) / (ne - 1)
    x = np.empty(ne + 1)
    acc = 0.0
    x[0] = 0.0
    for e in range(ne):
        acc = acc + h[e]
        x[e + 1] = acc
    return x


def stretched_cube_nodes(kx: int, ky: int, kz: int, ne: int = 60) -> np.ndarray:
    """Mesh nodes of the triaxially stretched cube (Sec. 3.3, App. B): along axis d the ne
    element sizes vary linearly from 0.1 to k_d/10, so the axis spans 3(k_d + 1)."""
    ax = [linear_sizes(ne, 0.1, k / 10.0) for k in (kx, ky, kz)]
    Z, Y, Xg = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return np.stack([Xg, Y, Z], axis=-1)


def perturbed_cube(ne: int = 60, seed: int = 0):
    """The randomly perturbed cube problem: (CsrProblem, rhs, coords)."""
    return q1_mesh(perturbed_cube_nodes(ne, seed), 0.0, u_trilinear,
                   f"q1_perturbed_{ne}_s{seed}")


def stretched_cube(kx: int, ky: int, kz: int, sigma: float, ne: int = 60):
    """The triaxially stretched reaction-diffusion cube (reaction 1/sigma): (CsrProblem, rhs,
    coords)."""
    return q1_mesh(stretched_cube_nodes(kx, ky, kz, ne), 1.0 / sigma, u_trilinear,
                   f"q1_stretch_{kx}_{ky}_{kz}_sig{sigma:g}_{ne}")


STRETCH_CONFIGS = [(kx, ky, kz) for kx in (1, 5, 10) for ky in (1, 5, 10) for kz in (1, 5, 10)
                   if kx <= ky <= kz]
STRETCH_SIGMAS = (1e1, 1e2, 1e3, 1e4, 1e5)


def periodic_stencil_2d(nx: int, ny: int, stencil: dict) -> CsrProblem:
    """Periodic 2-D stencil (circulant); ``stencil`` maps (dx, dy) -> value."""
    n = nx * ny
    rows = []
    for j in range(ny):
        for i in range(nx):
            ent = {}
            for (dx, dy), v in stencil.items():
                c = ((j + dy) % ny) * nx + (i + dx) % nx
                ent[c] = ent.get(c, 0.0) + v
            rows.append(sorted(ent.items()))
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([c for r in rows for c, _ in r], dtype=np.int32)
    val = np.array([v for r in rows for _, v in r], dtype=np.float64)
    return CsrProblem(n, rp, col, val, f"periodic_{nx}x{ny}")


def from_dense(d: np.ndarray, keep_zero_pattern: np.ndarray | None = None) -> CsrProblem:
    """CSR of a dense matrix; stores nonzeros, the diagonal, and any pattern entries given."""
    d = np.asarray(d, dtype=np.float64)
    n = d.shape[0]
    pat = d != 0
    pat[np.arange(n), np.arange(n)] = True
    if keep_zero_pattern is not None:
        pat |= keep_zero_pattern
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum(pat.sum(axis=1))
    rr, cc = np.nonzero(pat)
    return CsrProblem(n, rp, cc.astype(np.int32), d[rr, cc].astype(np.float64), "dense")


# ---------------------------------------------------------------------------------------
# Node coordinates (for the distance-Laplacian strength of Sec. 3.1)
# ---------------------------------------------------------------------------------------

def grid_coords(*axes) -> np.ndarray:
    """Coordinates of a tensor grid's nodes, (n, dim) float64, x fastest (the unknown order
    of every generator here); ``axes[d]`` holds the node positions along axis d."""
    mesh = np.meshgrid(*[np.asarray(a, dtype=np.float64) for a in reversed(axes)],
                       indexing="ij")
    return np.stack([g.reshape(-1) for g in reversed(mesh)], axis=1)


def _graded_nodes(nint: int, aspect: float) -> np.ndarray:
    """Interior node positions of a graded axis: node k (1-based) sits at h_0 + ... + h_{k-1}
    (summed in that order from 0.0) with the widths of ``graded_spacing``."""
    h = graded_spacing(nint, aspect)
    z = np.empty(nint)
    acc = 0.0
    for k in range(nint):
        acc = acc + h[k]
        z[k] = acc
    return z


def fd5_coords(nx: int = 64, ny: int = 64, aspect: float = 100.0) -> np.ndarray:
    """Node coordinates of ``fd5_stretched(nx, ny, aspect)``."""
    h = 1.0 / (nx + 1)
    return grid_coords(h * np.arange(1, nx + 1), _graded_nodes(ny, aspect))


def fd7_coords(n: int = 128, aspect: float = 1000.0, nx: int | None = None,
               ny: int | None = None) -> np.ndarray:
    """Node coordinates of ``fd7_stretched(n, aspect, nx, ny)``."""
    nx = n if nx is None else nx
    ny = n if ny is None else ny
    h = 1.0 / (nx + 1)
    return grid_coords(h * np.arange(1, nx + 1), h * np.arange(1, ny + 1),
                       _graded_nodes(n, aspect))


def q1_coords(ne: int = 100, hx=None, hy=None, hz=None, nex: int | None = None,
              ney: int | None = None) -> np.ndarray:
    """Node coordinates of ``q1_hex`` with the same mesh arguments (interior nodes)."""
    nex = ne if nex is None else nex
    ney = ne if ney is None else ney
    if hx is None:
        hx = hy = hz = Fraction(1, ne)
    ax = [float(hx * i) for i in range(1, nex)]
    ay = [float(hy * j) for j in range(1, ney)]
    az = [float(hz * k) for k in range(1, ne)]
    return grid_coords(ax, ay, az)


def random_rhs(n: int, seed: int) -> np.ndarray:
    """b_i ~ U(-1, 1) from numpy PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-1.0, 1.0, size=n)


# ---------------------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------------------

def workload(name: str) -> CsrProblem:
    """The named synthetic workloads.

    * ``fd5_64x64_a100``   2-D 5-pt, 64x64 unknowns, aspect 1:100 (n = 4,096).
    * ``fd7_128_a1000``    3-D 7-pt, 128^3 unknowns, aspect 1:1000 (n = 2,097,152).
    * ``q1_100_randkappa`` 27-pt Q1, 100^3 elements, kappa = 10^U[-3,3] (n = 970,299).
    * ``fd7_160_a1000``    3-D 7-pt, 160^3 unknowns, aspect 1:1000 (n = 4,096,000).
    * ``q1_box24_hz2``     27-pt Q1 on 1x1x2 boxes, 24^3 unknowns (stress problem).
    Any ``fd7_<n>_a<aspect>`` and ``fd5_<n>x<n>_a<aspect>`` is also accepted.
    """
    if name == "q1_100_randkappa":
        return q1_random_kappa(100, seed=3)
    if name == "q1_box24_hz2":
        return q1_stretched_box(24, Fraction(2))
    if name.startswith("fd7_"):
        _, n, a = name.split("_")
        return fd7_stretched(int(n), float(a[1:]))
    if name.startswith("fd5_"):
        _, nn, a = name.split("_")
        nx, ny = nn.split("x")
        return fd5_stretched(int(nx), int(ny), float(a[1:]))
    if name.startswith("q1_") and name.endswith("_randkappa"):
        return q1_random_kappa(int(name.split("_")[1]), seed=3)
    raise KeyError(name)


RHS_SEED = {"fd5_64x64_a100": 1, "fd7_128_a1000": 2, "q1_100_randkappa": 4,
            "fd7_160_a1000": 5, "q1_box24_hz2": 7}


def serving_requests(count: int = 256, seed: int = 6, smin: int = 16, smax: int = 96):
    """Seeded request descriptions for the serving workload.

    Each request is a 7-point z-stretched cube with aspect 10**U[1,3] or a 27-point random
    kappa cube (u ~ U[-3,3]), chosen with probability 1/2, with side s ~ U{smin..smax}
    unknowns per dimension (the 27-point cube then has s+1 elements per dimension).
    Returns a list of dicts; ``build_request`` turns one into (CsrProblem, rhs).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for r in range(count):
        kind = "fd7" if rng.uniform() < 0.5 else "q1"
        s = int(rng.integers(smin, smax + 1))
        aspect = float(10.0 ** rng.uniform(1.0, 3.0))
        sub = int(rng.integers(0, 2**31 - 1))
        out.append({"id": r, "kind": kind, "side": s, "aspect": aspect, "seed": sub})
    return out


def serving_method(req: dict) -> dict:
    """Method settings of a serving request, for both families: OffLmp + 1Norm (plain SA's
    filtered diagonal can vanish on the random-coefficient cubes, and its eigenvalue estimate
    can turn negative on some stretched ones: the failures the adaptations of Sec. 2 address)
    and the Chebyshev interval's upper end 1.1 times the power-method estimate (ten power
    steps can underestimate the largest eigenvalue enough to leave the V-cycle indefinite on
    the 6-decade coefficient jumps).  FP32 V-cycle inside FP64 CG to 1e-10."""
    return {"variants": ("offlmp", "1norm"), "cheb_boost": 1.1, "precision": "fp32",
            "rtol": 1e-10}


def build_request(req: dict):
    if req["kind"] == "fd7":
        p = fd7_stretched(req["side"], req["aspect"])
    else:
        p = q1_random_kappa(req["side"] + 1, seed=req["seed"])
    b = random_rhs(p.n, req["seed"] + 1)
    return p, b
