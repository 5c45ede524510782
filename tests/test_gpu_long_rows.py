"""GPU parity on operators with long rows: the split row-sum order of y = A x (rows of more
than 64 entries as 64 interleaved in-order partial sums, added in order), rows that span the
SpMV's chunks, several long rows in one row block, and the coarse levels they produce.

The matrix is a 100 x 200 five-point Laplacian plus symmetric "hub" couplings: hub h is
coupled (weight -1/2, strong at theta = 0.02) to random far vertices so that its row has
exactly the target length (64, 65, 127, 128, 500, 2047, 2048, 2049, 4500 and 9000 entries;
two hubs are neighbours in index, so one row block holds both).  The diagonal is the absolute
row sum plus 1/10, so the matrix is a symmetric M-matrix.  Both power methods of every level
(D^-1 Abar for the damping factor, D^-1 A for the smoother) run through the SpMV, and their
results are compared bitwise with the oracle, as is every setup array; the solve compares
iterations and x.  The FP32 V-cycle (float products, the same split order) is compared with the
FP64 solve.  A second matrix gives Sprsfy a root row of 5200 entries, longer than its block
kernels hold in LDS.
"""
import numpy as np
import pytest

from paper_2103_10476_amd import problems as pb
from parity import compare_setup, compare_solve, log, run_both

pytestmark = pytest.mark.gpu

TARGETS = [64, 65, 127, 128, 500, 2047, 2048, 2049, 4500, 9000]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()


def hub_problem(nx=100, ny=200, seed=3):
    n = nx * ny
    rng = np.random.Generator(np.random.PCG64(seed))
    nbrs = [set() for _ in range(n)]
    w = {}

    def link(i, j, v):
        nbrs[i].add(j)
        nbrs[j].add(i)
        w[(min(i, j), max(i, j))] = v

    for y in range(ny):
        for x in range(nx):
            i = x + nx * y
            if x + 1 < nx:
                link(i, i + 1, -1.0)
            if y + 1 < ny:
                link(i, i + nx, -1.0)
    # interior hubs spread over the index range, two of them adjacent
    hubs = [nx * (10 + 18 * k) + 50 for k in range(len(TARGETS) - 1)]
    hubs.append(hubs[-1] + 1)
    for h, t in zip(hubs, TARGETS):
        extra = t - 1 - len(nbrs[h])  # row length = off-diagonals + the diagonal
        cand = rng.permutation(n)
        k = 0
        for j in cand:
            if k == extra:
                break
            j = int(j)
            if j == h or j in nbrs[h] or j in hubs:
                continue
            link(h, j, -0.5)
            k += 1
        assert len(nbrs[h]) + 1 == t
    rows, cols, vals = [], [], []
    for i in range(n):
        off = sorted(nbrs[i])
        d = 0.0
        for j in off:
            d += abs(w[(min(i, j), max(i, j))])
        entries = [(j, w[(min(i, j), max(i, j))]) for j in off] + [(i, d + 0.1)]
        entries.sort()
        for j, v in entries:
            rows.append(i)
            cols.append(j)
            vals.append(v)
    rp = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rp, np.asarray(rows) + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    prob = pb.CsrProblem(n, rp, np.asarray(cols, dtype=np.int32), np.asarray(vals),
                         f"hubs_{nx}x{ny}")
    return prob, hubs


def test_hub_matrix_shape():
    p, hubs = hub_problem()
    lens = np.diff(p.rp)
    assert sorted(int(lens[h]) for h in hubs) == sorted(TARGETS)
    assert hubs[-1] == hubs[-2] + 1
    # symmetric, M-matrix, strictly diagonally dominant
    rows = np.repeat(np.arange(p.n), lens)
    a = {(int(r), int(c)): v for r, c, v in zip(rows, p.col, p.val)}
    for (r, c), v in list(a.items())[:20000]:
        assert a[(c, r)] == v
    off = rows != p.col
    assert np.all(p.val[off] < 0) and np.all(p.val[~off] > 0)


@pytest.mark.parametrize("var", [[], ["offlmp", "1norm"], ["sprsfy"]],
                         ids=lambda v: "+".join(v) or "plain")
def test_hub_matrix_parity(var):
    p, _ = hub_problem()
    g, h = run_both(p, theta=0.02, variants=var, rtol=1e-10, max_coarse=200)
    log(f"[long rows] levels {g.info()['levels']} n {g.info()['n']}")
    compare_setup(g, h)
    compare_solve(g, h, pb.random_rhs(p.n, 5))


def test_hub_matrix_fp32_vcycle():
    from paper_2103_10476_amd import solver
    p, _ = hub_problem()
    b = pb.random_rhs(p.n, 6)
    xs = {}
    for prec in ("fp64", "fp32"):
        o = solver.Options(theta=0.02, rtol=1e-10, max_coarse=200, precision=prec)
        g = solver.Hierarchy.from_problem(p, options=o)
        x, it = solver.solve(g, b)
        xs[prec] = x.cpu().numpy()
        log(f"[long rows] {prec}: {it} iterations")
        g.close()
    err = np.linalg.norm(xs["fp32"] - xs["fp64"]) / np.linalg.norm(xs["fp64"])
    assert err < 1e-8, err


def long_root_problem(nx=100, ny=200, span=5200, w=0.01):
    """A 100 x 200 five-point Laplacian whose corner vertex 0 is also coupled weakly (weight
    -w) to every vertex of index below span but its grid neighbours: a 5200-entry row whose grid
    couplings stay strong (at theta = 0.02), so vertex 0 is the first root and its aggregate's
    Sprsfy decisions read a root row longer than the block kernels' LDS holds."""
    n = nx * ny
    nb = [dict() for _ in range(n)]

    def link(i, j, v):
        nb[i][j] = v
        nb[j][i] = v

    for y in range(ny):
        for x in range(nx):
            i = x + nx * y
            if x + 1 < nx:
                link(i, i + 1, -1.0)
            if y + 1 < ny:
                link(i, i + nx, -1.0)
    for j in range(2, span):
        if j != nx:
            link(0, j, -w)
    rp = np.zeros(n + 1, dtype=np.int32)
    cols, vals = [], []
    for i in range(n):
        d = sum(abs(v) for v in nb[i].values()) + 0.1
        ent = sorted(list(nb[i].items()) + [(i, d)])
        rp[i + 1] = rp[i] + len(ent)
        cols += [j for j, _ in ent]
        vals += [v for _, v in ent]
    return pb.CsrProblem(n, rp, np.asarray(cols, dtype=np.int32), np.asarray(vals), "longroot")


def test_sprsfy_long_root_row():
    """Sprsfy on an aggregate whose root row has 5200 entries: every setup array (the drop
    marks among them) bitwise equal to the oracle's, and the solve."""
    p = long_root_problem()
    assert p.rp[1] - p.rp[0] == 5200
    g, h = run_both(p, theta=0.02, variants=["sprsfy"], rtol=1e-10, max_coarse=200)
    L0 = h.levels[0]
    assert L0.is_root[0] == 1 and int(np.sum(L0.mask == 2)) > 0  # the path is exercised
    compare_setup(g, h)
    compare_solve(g, h, pb.random_rhs(p.n, 7))

