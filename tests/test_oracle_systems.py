"""Oracle pins for systems SA with a multi-vector nullspace (the paper's future work; standard
smoothed aggregation for systems with a QR tentative prolongator).

* Per aggregate, P_t's block is the Q of numpy's QR of the aggregate's rows of B (signs with a
  non-negative R diagonal), P_t^T P_t = I and P_t B_c = B.
* Smoothing: P B_c = (I - omega D^-1 Abar) B.
* bs = 1, k = 1, B = 1 builds the scalar hierarchy up to the column scaling of P: the same
  labels and aggregates, the same iterations, the solution to rounding.
* A (x) I_2 with the two component translations decouples into two copies of the scalar
  problem: the node labels are the scalar labels and the aggregates the scalar aggregates.
* Elasticity: rigid-body modes lie in the kernel of the unconstrained stiffness, and with
  them the solver needs far fewer iterations than with translations alone.
"""
import numpy as np
import pytest
from scipy.sparse import csr_matrix

from paper_2103_10476_amd import problems as pb


def _sp(t, shape):
    return csr_matrix((t[2], t[1], t[0]), shape=shape)


@pytest.fixture(scope="module")
def beam():
    return pb.elastic_beam(16, 5, 5)


def test_qr_tentative_prolongator(orc, beam):
    p, X, B = beam
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, nullspace=B, block_size=3,
                            max_coarse=100)
    L0, L1 = h.levels[0], h.levels[1]
    Pt = _sp(L0.Pt, (p.n, L1.n)).toarray()
    assert np.abs(Pt.T @ Pt - np.eye(L1.n)).max() <= 1e-13
    assert np.abs(Pt @ L1.B - B).max() <= 1e-12
    k = 6
    for J in range(0, L0.nc, max(1, L0.nc // 25)):
        nodes = np.flatnonzero(L0.agg == J)
        dofs = (3 * nodes[:, None] + np.arange(3)).reshape(-1)
        Q, R = np.linalg.qr(B[dofs])
        sg = np.sign(np.diag(R))
        sg[sg == 0] = 1.0
        Q, R = Q * sg, R * sg[:, None]
        assert np.abs(Pt[np.ix_(dofs, k * J + np.arange(k))] - Q).max() <= 1e-12
        assert np.abs(L1.B[k * J:k * J + k] - R).max() <= 1e-12 * np.abs(R).max()
    # smoothed prolongator: P B_c = (I - omega D^-1 Abar) B
    P = _sp(L0.P, (p.n, L1.n)).toarray()
    Ab = _sp(L0.Abar, (p.n, p.n)).toarray()
    want = B - (L0.omega * L0.invD)[:, None] * (Ab @ B)
    assert np.abs(P @ L1.B - want).max() <= 1e-11 * np.abs(want).max()


def test_scalar_problem_as_a_system_of_one(orc):
    """The QR of a column of ones is the unit tentative prolongator scaled by 1/sqrt(|J|) per
    column.  With two levels (an exact coarse solve) the preconditioner is invariant under that
    scaling; deeper, lumping on the rescaled coarse operator differs (it is not invariant under
    diagonal scaling), so only the first two levels' labels must agree."""
    q = pb.fd7_stretched(12, 100.0)
    hs = orc.OracleHierarchy(q.n, q.rp, q.col, q.val, max_coarse=500, rtol=1e-10)
    hq = orc.OracleHierarchy(q.n, q.rp, q.col, q.val, nullspace=np.ones((q.n, 1)),
                             block_size=1, max_coarse=500, rtol=1e-10)
    assert len(hs.levels) == len(hq.levels) == 2
    assert np.array_equal(hs.levels[0].mask, hq.levels[0].mask)
    assert np.array_equal(hs.levels[0].agg, hq.levels[0].agg)
    cnt = np.bincount(hs.levels[0].agg[hs.levels[0].agg >= 0])
    assert np.allclose(hq.levels[1].B[:, 0], np.sqrt(cnt), rtol=1e-15, atol=0)
    bvec = pb.random_rhs(q.n, 3)
    r1, r2 = hs.solve(bvec), hq.solve(bvec)
    assert r1["iterations"] == r2["iterations"]
    assert np.linalg.norm(r1["x"] - r2["x"]) <= 1e-11 * np.linalg.norm(r1["x"])
    deep_s = orc.OracleHierarchy(q.n, q.rp, q.col, q.val, max_coarse=60)
    deep_q = orc.OracleHierarchy(q.n, q.rp, q.col, q.val, nullspace=np.ones((q.n, 1)),
                                 block_size=1, max_coarse=60)
    for l in (0, 1):
        assert np.array_equal(deep_s.levels[l].mask, deep_q.levels[l].mask)
        assert np.array_equal(deep_s.levels[l].agg, deep_q.levels[l].agg)


def test_kronecker_system_decouples(orc):
    q = pb.fd7_stretched(9, 1000.0)
    A = _sp((q.rp, q.col, q.val), (q.n, q.n))
    K = csr_matrix(np.kron(A.toarray(), np.eye(2)))
    K.sort_indices()
    Bm = np.kron(np.ones((q.n, 1)), np.eye(2))
    hs = orc.OracleHierarchy(q.n, q.rp, q.col, q.val, max_coarse=40)
    hk = orc.OracleHierarchy(2 * q.n, K.indptr, K.indices, K.data, nullspace=Bm, block_size=2,
                             max_coarse=80)
    L, M = hs.levels[0], hk.levels[0]
    assert np.array_equal(M.nmask, L.mask)            # node labels = scalar labels
    assert np.array_equal(M.agg, L.agg)
    assert [2 * l.n for l in hs.levels] == [l.n for l in hk.levels]


def test_elasticity_rigid_body_modes(orc, beam):
    g = np.linspace(0.0, 1.0, 5)
    Z, Y, Xg = np.meshgrid(g, g, g, indexing="ij")
    q, _, Bq = pb.q1_elasticity(np.stack([Xg, Y, Z], -1), fixed=np.zeros((5, 5, 5), bool))
    Kq = q.to_dense()
    assert np.abs(Kq @ Bq).max() <= 1e-13 * np.abs(Kq).max()
    ev = np.linalg.eigvalsh(Kq)
    assert np.sum(np.abs(ev) <= 1e-12 * ev.max()) == 6
    p, X, B = beam
    b = pb.random_rhs(p.n, 2)
    it = {}
    for k in (3, 6):
        h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, nullspace=B[:, :k].copy(),
                                block_size=3, max_coarse=100, rtol=1e-8)
        r = h.solve(b)
        assert r["converged"]
        it[k] = r["iterations"]
    assert it[6] < 0.7 * it[3], it


def test_systems_distance_strength_and_errors(orc, beam):
    p, X, B = beam
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, nullspace=B, block_size=3, coords=X,
                            max_coarse=100, theta=0.025)
    L = h.levels[0]
    m = orc.distance_strength(len(X), L.Gn[0], L.Gn[1], X, 0.025)
    assert np.array_equal(L.nmask, m)
    assert h.levels[1].coords.shape == (L.nc, 3)
    assert p.n % 5 != 0
    with pytest.raises(orc.OracleError):      # the block size must divide n
        orc.OracleHierarchy(p.n, p.rp, p.col, p.val, nullspace=B, block_size=5)
    for var in (("sprsfy",), ("cnstrnt",)):
        with pytest.raises(orc.OracleError):
            orc.OracleHierarchy(p.n, p.rp, p.col, p.val, nullspace=B, block_size=3,
                                variants=var, max_coarse=100)
    bad = B.copy()
    bad[3, 2] = np.nan
    with pytest.raises(orc.OracleError):
        orc.OracleHierarchy(p.n, p.rp, p.col, p.val, nullspace=bad, block_size=3)
    # an aggregate with fewer dofs than nullspace vectors (corner aggregates of a cube)
    q = pb.fd7_stretched(8, 1.0)
    with pytest.raises(orc.OracleError) as e:
        orc.OracleHierarchy(q.n, q.rp, q.col, q.val, nullspace=np.random.default_rng(0)
                            .normal(size=(q.n, 6)), block_size=1, max_coarse=2)
    assert "fewer" in str(e.value)
    # re-setup keeps the nullspace: same values reproduce the hierarchy; a new one is refused
    h2 = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, nullspace=B, block_size=3, max_coarse=100)
    ref = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, nullspace=B, block_size=3, max_coarse=100)
    h2.resetup(p.val)
    for a, c in zip(h2.levels, ref.levels):
        assert np.array_equal(a.A[2], c.A[2])
    with pytest.raises(orc.OracleError):
        h2.resetup(p.val, nullspace=B)
