"""Pins of the oracle's aggregation, tentative prolongator and Sprsfy.

Sources: Sec. 1.1 (aggregates partition the vertices; tentative prolongator from the constant
near null space) and Sec. 2.5 (root choice, Fig. 1 aggregates, the Sprsfy relabelling).
"""
import numpy as np
import pytest

from paper_2103_10476_amd import problems as pb


def rows_of(rp):
    return np.repeat(np.arange(len(rp) - 1), np.diff(rp))


def graph_from_mask(p, mask):
    r = rows_of(p.rp)
    g = [set() for _ in range(p.n)]
    for e in range(p.nnz):
        if mask[e] in (1, 2):
            g[r[e]].add(int(p.col[e]))
            g[int(p.col[e])].add(int(r[e]))
    return g


def mis2_rounds(g, prio, singletons=False):
    """Independent route to the aggregation roots: rounds of the distance-2 maximal
    independent set rule (a vertex enters when it has the best priority among the undecided
    vertices within distance 2 and no entered vertex is within distance 2).  An isolated
    vertex is alone in its ball: it enters in the first round when isolated vertices are
    singleton aggregates, and never takes part otherwise."""
    n = len(g)
    UND, IN, OUT = 1, 0, 2
    state = [UND if (g[v] or singletons) else OUT for v in range(n)]
    while any(s == UND for s in state):
        key = [(state[v], prio[v]) for v in range(n)]
        k1 = [min([key[v]] + [key[u] for u in g[v]]) for v in range(n)]
        k2 = [min([k1[v]] + [k1[u] for u in g[v]]) for v in range(n)]
        new = list(state)
        for v in range(n):
            if state[v] != UND:
                continue
            if k2[v][0] == IN:
                new[v] = OUT
            elif k2[v] == key[v]:
                new[v] = IN
        state = new
    return [s == IN for s in state]


def dist2_ball(g, v):
    out = {v} | g[v]
    for u in g[v]:
        out |= g[u]
    return out


def check_partition(g, agg, root, nc, singletons=False):
    n = len(g)
    roots = [v for v in range(n) if root[v]]
    assert len(roots) == nc
    assert sorted(agg[v] for v in roots) == list(range(nc))
    # numbering = rank of the root's index
    assert [agg[v] for v in roots] == list(range(nc))
    # eq. (aggregates): the aggregates are disjoint (agg is a function), none is empty, and
    # they cover every vertex with a strong connection -- every vertex at all when isolated
    # vertices are singleton aggregates, which the left-out reading drops
    assert set(a for a in agg if a >= 0) == set(range(nc))
    for v in range(n):
        if g[v]:
            assert 0 <= agg[v] < nc
        elif singletons:
            assert root[v] and list(agg).count(agg[v]) == 1
        else:
            assert agg[v] == -1 and not root[v]
    for a, ra in enumerate(roots):
        for rb in roots[a + 1:]:
            assert rb not in dist2_ball(g, ra)  # roots at graph distance >= 3
        for u in g[ra]:
            assert agg[u] == agg[ra]  # aggregate contains the closed neighbourhood


def random_sym_pattern(rng, n, density):
    d = (rng.uniform(size=(n, n)) < density).astype(float)
    d = np.triu(d, 1)
    d = -(d + d.T)
    d[np.arange(n), np.arange(n)] = 1.0
    return pb.from_dense(d)


@pytest.mark.parametrize("isolated", ["left_out", "singleton"])
@pytest.mark.parametrize("order", [0, 1])
def test_greedy_equals_mis2_rounds(orc, order, isolated):
    """The greedy root choice is the lexicographically-first distance-2 MIS; brute force by
    rounds on random graphs (isolated vertices among them), natural and hashed priority."""
    rng = np.random.default_rng(5 + order)
    sing = isolated == "singleton"
    for trial in range(60):
        n = int(rng.integers(2, 40))
        p = random_sym_pattern(rng, n, rng.uniform(0.02, 0.3))
        mask = np.where(p.col == rows_of(p.rp), 3, 1).astype(np.uint8)
        seed = int(rng.integers(0, 2**63))
        agg, root, nc = orc.aggregate(p.n, p.rp, p.col, mask, order=order, seed=seed, level=2,
                                      isolated=isolated)
        g = graph_from_mask(p, mask)
        if order == 0:
            prio = list(range(n))
        else:
            prio = [((orc.splitmix64(seed, (2 << 56) | (2 << 40) | v) >> 34) << 32) | v
                    for v in range(n)]
        expect = mis2_rounds(g, prio, sing)
        assert [bool(x) for x in root] == expect
        check_partition(g, list(agg), list(root), nc, sing)
        # leftovers join the aggregate they have the most strong edges to (ties: smaller id)
        owner = {}
        for v in range(n):
            if root[v]:
                owner[v] = agg[v]
                for u in g[v]:
                    owner[u] = agg[v]
        for v in range(n):
            if g[v] and v not in owner:
                cnt = {}
                for u in g[v]:
                    if u in owner:
                        cnt[owner[u]] = cnt.get(owner[u], 0) + 1
                best = max(cnt.values())
                assert agg[v] == min(a for a, c in cnt.items() if c == best)


def _periodic9(side, vertical_only):
    st = {}
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            if dx == dy == 0:
                continue
            st[(dx, dy)] = -1.0 if (not vertical_only or dx == 0) else -1e-4
    st[(0, 0)] = -sum(st.values())
    return pb.periodic_stencil_2d(side, side, st)


def test_fig1_all_strong_gives_3x3_squares(orc):
    """Fig. 1 (left): all connections strong on a regular mesh -> perfect square aggregates."""
    side = 12
    p = _periodic9(side, False)
    mask = orc.strength(p.n, p.rp, p.col, p.val, 0.0)
    agg, root, nc = orc.aggregate(p.n, p.rp, p.col, mask)
    assert nc == (side // 3) ** 2
    for a in range(nc):
        members = np.nonzero(agg == a)[0]
        xs = sorted({int(v % side) for v in members})
        ys = sorted({int(v // side) for v in members})
        assert len(members) == 9 and len(xs) == 3 and len(ys) == 3


def test_fig1_vertical_strong_gives_3x1_lines(orc):
    """Fig. 1 (right): only vertical connections strong -> 3-point vertical aggregates."""
    side = 12
    p = _periodic9(side, True)
    mask = orc.strength(p.n, p.rp, p.col, p.val, 0.02)
    agg, root, nc = orc.aggregate(p.n, p.rp, p.col, mask)
    assert nc == side * side // 3
    for a in range(nc):
        members = np.nonzero(agg == a)[0]
        assert len(members) == 3 and len({int(v % side) for v in members}) == 1


def test_tentative_prolongator_properties(orc):
    """Sec. 1.1: Ptent has one unit entry per aggregated row, reproduces the constant there,
    and its column-normalised form Q has orthonormal columns (one nullspace vector: QR =
    scaling)."""
    p = pb.fd5_stretched(20, 20, 100.0)
    mask = orc.strength(p.n, p.rp, p.col, p.val, 0.02)
    agg, root, nc = orc.aggregate(p.n, p.rp, p.col, mask)
    Pt = np.zeros((p.n, nc))
    rows = np.nonzero(agg >= 0)[0]
    Pt[rows, agg[rows]] = 1.0
    assert np.all(Pt.sum(axis=1)[rows] == 1.0)
    assert np.array_equal(Pt @ np.ones(nc), (agg >= 0).astype(float))
    Q = Pt / np.sqrt(Pt.sum(axis=0))
    np.testing.assert_allclose(Q.T @ Q, np.eye(nc), atol=1e-15)


def test_isolated_vertex_left_out_or_singleton(orc):
    """A vertex without strong connections joins no aggregate by default (a zero row of the
    tentative prolongator).  With the covering reading of Sec. 1.1, eq. (aggregates), the
    root rule makes it the root of an aggregate of its own (nothing around it is
    aggregated), numbered by the rank of its index among the roots."""
    d = np.array([[1.0, 0.0, 0.0, -1e-6], [0.0, 2.0, -1.0, 0.0], [0.0, -1.0, 2.0, -1.0],
                  [-1e-6, 0.0, -1.0, 2.0]])
    p = pb.from_dense(d)
    mask = orc.strength(p.n, p.rp, p.col, p.val, 0.1)
    agg, root, nc = orc.aggregate(p.n, p.rp, p.col, mask)
    assert nc == 1 and list(agg) == [-1, 0, 0, 0] and list(root) == [0, 1, 0, 0]
    agg, root, nc = orc.aggregate(p.n, p.rp, p.col, mask, isolated="singleton")
    assert nc == 2 and list(agg) == [0, 1, 1, 1] and list(root) == [1, 1, 0, 0]


def test_singleton_reading_on_a_random_coefficient_cube(orc):
    """Covering reading: a random-coefficient cube with isolated vertices still coarsens
    (the others aggregate), each isolated vertex a coarse unknown of its own; it converges."""
    p = pb.q1_random_kappa(12, seed=3)
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, theta=0.02, variants=["offlmp", "1norm"],
                            max_coarse=50, rtol=1e-8, isolated="singleton")
    L0 = h.levels[0]
    g = graph_from_mask(pb.CsrProblem(p.n, p.rp, p.col, p.val, "q1"), L0.mask)
    iso = [v for v in range(p.n) if not g[v]]
    assert iso, "the random-coefficient cube has vertices without strong connections"
    assert np.all((L0.agg >= 0) & (L0.agg < L0.nc))
    for v in iso:
        assert L0.is_root[v] and np.count_nonzero(L0.agg == L0.agg[v]) == 1
    assert h.levels[1].n == L0.nc < p.n
    r = h.solve(pb.random_rhs(p.n, 4))
    assert r["converged"] and r["iterations"] < 40


def test_left_out_reading_keeps_the_stretched_cube_coarsening(orc):
    """What leaving isolated vertices out buys, on the benchmark family (64^3 z-stretched
    7-point cube, aspect 1:1000, 1Norm): on level 2 a whole z-plane of 64 x 64 vertices has
    no strong connection.  As singleton aggregates (the covering reading) those 4096 vertices
    are carried to every coarser level, so the coarsening stalls: the last levels shrink by
    well under 1% and the coarsest keeps more than 4096 unknowns.  Left out, the plane is
    treated by the smoother alone and the hierarchy reaches a small coarsest level; both
    converge."""
    p = pb.fd7_stretched(64, 1000.0)
    b = pb.random_rhs(p.n, 2)
    kw = dict(theta=0.02, variants=["1norm"], rtol=1e-8)
    left = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, **kw)
    iso = [int(np.count_nonzero(L.agg < 0)) for L in left.levels[:-1]]
    assert 4096 in iso
    plane = np.nonzero(left.levels[iso.index(4096)].agg < 0)[0]
    sing = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, isolated="singleton", **kw)
    ns = [L.n for L in sing.levels]
    assert ns[-1] > 4096 and ns[-2] - ns[-1] < 0.01 * ns[-2]
    assert left.levels[-1].n < 1000 and len(left.levels) < len(sing.levels)
    assert left.solve(b)["converged"] and sing.solve(b)["converged"]
    assert len(plane) == 4096


def _sprsfy_grid(nx=6, ny=6, special=((1, 1), (2, 1))):
    """Vertical strong couplings, weak horizontal ones, plus one strong horizontal edge."""
    n = nx * ny
    d = np.zeros((n, n))
    idx = lambda x, y: x + nx * y  # noqa: E731
    for y in range(ny):
        for x in range(nx):
            i = idx(x, y)
            if y + 1 < ny:
                d[i, idx(x, y + 1)] = d[idx(x, y + 1), i] = -1.0
            if x + 1 < nx:
                d[i, idx(x + 1, y)] = d[idx(x + 1, y), i] = -1e-4
    a, b = idx(*special[0]), idx(*special[1])
    d[a, b] = d[b, a] = -1.0
    d[np.arange(n), np.arange(n)] = -d.sum(axis=1) + 0.1
    return pb.from_dense(d), a, b


def test_sprsfy_drops_lone_strong_link(orc):
    """Sec. 2.5: a non-root member's single strong connection into an aggregate that the
    root reaches only through weak connections is dropped, together with its transpose."""
    p, a, b = _sprsfy_grid()
    mask = orc.strength(p.n, p.rp, p.col, p.val, 0.02)
    agg, root, nc = orc.aggregate(p.n, p.rp, p.col, mask)
    assert not root[a] and not root[b] and agg[a] != agg[b]
    m2 = orc.sprsfy(p.n, p.rp, p.col, mask, agg, root, nc)
    r = rows_of(p.rp)
    changed = np.nonzero(m2 != mask)[0]
    pairs = {(int(r[e]), int(p.col[e])) for e in changed}
    assert pairs == {(a, b), (b, a)}
    assert np.all(m2[changed] == 2)
    # aggregates are not affected; the twice-filtered pattern stays symmetric
    agg2, root2, nc2 = orc.aggregate(p.n, p.rp, p.col, mask)
    assert np.array_equal(agg, agg2)
    rp, col, val = orc.lump(p.n, p.rp, p.col, p.val, m2)
    D = np.zeros((p.n, p.n), bool)
    D[rows_of(rp), col] = True
    assert np.array_equal(D, D.T)


def test_sprsfy_keeps_multiple_links(orc):
    """Two strong connections into the same candidate aggregate are both kept."""
    p, a, b = _sprsfy_grid(special=((1, 1), (2, 1)))
    # add a second strong link from the same aggregate into the same neighbour aggregate
    d = p.to_dense()
    i, j = 1 + 6 * 0, 2 + 6 * 0  # roots (1,0) and (2,0): a root-root link is strong too
    d[i, j] = d[j, i] = -1.0
    d[np.arange(p.n), np.arange(p.n)] = 0.0
    d[np.arange(p.n), np.arange(p.n)] = -d.sum(axis=1) + 0.1
    q = pb.from_dense(d)
    mask = orc.strength(q.n, q.rp, q.col, q.val, 0.02)
    agg, root, nc = orc.aggregate(q.n, q.rp, q.col, mask)
    m2 = orc.sprsfy(q.n, q.rp, q.col, mask, agg, root, nc)
    r = rows_of(q.rp)
    for e in np.nonzero(m2 != mask)[0]:
        assert {int(r[e]), int(q.col[e])} != {a, b}


def test_sprsfy_reduces_coarse_nnz(orc):
    """Sec. 3.1/3.3: Sprsfy lowers operator complexity."""
    p = pb.workload("fd7_16_a1000")
    h0 = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, theta=0.02, max_coarse=50)
    h1 = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, theta=0.02, max_coarse=50,
                             variants=["sprsfy"])
    assert np.array_equal(h0.levels[0].agg, h1.levels[0].agg)
    assert h1.levels[1].nnz <= h0.levels[1].nnz
    assert h1.levels[0].Abar[0][-1] <= h0.levels[0].Abar[0][-1]
