"""Systems SA with a multi-vector nullspace (sa_setup_system) through the C ABI against the
oracle: 3-D Q1 elasticity with its six rigid-body modes (and with translations only), the
block and the distance strength, plain/OffLmp/1Norm, a Kronecker-product system, a scalar
problem as a system of one, FP32 V-cycle, GMRES, re-setup and the error cases.  Every level
bitwise (node graph, labels, aggregates, QR tentative prolongator, nullspaces, P, R, A_l),
equal iterations, solutions to 1e-12."""
import numpy as np
import pytest
from scipy.sparse import csr_matrix

from paper_2103_10476_amd import problems as pb
from parity import compare_setup, compare_solve, log, run_both

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


_BEAMS = {}


def _beam(*args, **kw):
    key = (args, tuple(sorted(kw.items())))
    if key not in _BEAMS:
        _BEAMS[key] = pb.elastic_beam(*args, **kw)
    return _BEAMS[key]


@pytest.mark.parametrize("var", [(), ("offlmp",), ("1norm",), ("offlmp", "1norm")],
                         ids=lambda v: "+".join(v) or "plain")
@pytest.mark.parametrize("k", [6, 3])
def test_elastic_beam_matches_oracle(var, k):
    p, X, B = _beam(24, 6, 6)
    g, h = run_both(p, nullspace=B[:, :k].copy(), block_size=3, variants=var, max_coarse=200,
                    rtol=1e-10)
    assert len(h.levels) >= 2
    compare_setup(g, h)
    it, _ = compare_solve(g, h, pb.random_rhs(p.n, 3))
    log(f"[systems] beam k={k} {'+'.join(var) or 'plain'}: levels {g.info()['n']}, {it} its")
    g.close()


def test_stretched_beam_distance_strength():
    p, X, B = _beam(20, 8, 8, stretch=20.0)
    g, h = run_both(p, nullspace=B, block_size=3, coords=X, theta=0.025, max_coarse=150,
                    variants=("offlmp", "1norm"), rtol=1e-10)
    compare_setup(g, h)
    compare_solve(g, h, pb.random_rhs(p.n, 4))
    g.close()


def test_kronecker_system_and_system_of_one():
    q = pb.fd7_stretched(14, 1000.0)
    A = csr_matrix((q.val, q.col, q.rp), shape=(q.n, q.n)).toarray()
    K = csr_matrix(np.kron(A, np.eye(2)))
    K.sort_indices()
    kp = pb.CsrProblem(2 * q.n, K.indptr.astype(np.int32), K.indices.astype(np.int32), K.data)
    g, h = run_both(kp, nullspace=np.kron(np.ones((q.n, 1)), np.eye(2)), block_size=2,
                    max_coarse=100, rtol=1e-10)
    compare_setup(g, h)
    compare_solve(g, h, pb.random_rhs(kp.n, 5))
    g.close()
    g, h = run_both(q, nullspace=np.ones((q.n, 1)), block_size=1, max_coarse=60, rtol=1e-10,
                    agg_order="hashed", smoother="jacobi")
    compare_setup(g, h)
    compare_solve(g, h, pb.random_rhs(q.n, 6))
    g.close()


def test_systems_fp32_gmres_and_resetup():
    from oracle import oracle as orc
    from paper_2103_10476_amd import solver
    p, X, B = _beam(24, 6, 6)
    kw = dict(max_coarse=200, rtol=1e-10)
    g = solver.Hierarchy.from_problem(p, nullspace=B, block_size=3,
                                      options=solver.Options(precision="fp32", **kw))
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, nullspace=B, block_size=3, **kw)
    b = pb.random_rhs(p.n, 7)
    x, it, rr, st = g.solve(b)
    ref = h.solve(b)
    assert st == "SA_OK" and abs(it - ref["iterations"]) <= 2
    assert np.linalg.norm(x.cpu().numpy() - ref["x"]) <= 1e-8 * np.linalg.norm(ref["x"])
    g.close()
    g, h = run_both(p, nullspace=B, block_size=3, **kw)
    x, it, rr, st = g.solve_gmres(b, restart=30)
    r = h.solve_gmres(b, restart=30)
    assert it == r["iterations"]
    assert np.linalg.norm(x.cpu().numpy() - r["x"]) <= 1e-12 * np.linalg.norm(r["x"])
    rng = np.random.Generator(np.random.PCG64(9))
    d = np.repeat(rng.uniform(0.5, 2.0, size=p.n // 3), 3)
    rows = np.repeat(np.arange(p.n), np.diff(p.rp))
    val2 = (d[rows] * p.val) * d[p.col]
    g.resetup(val2)
    h.resetup(val2)
    compare_setup(g, h)
    compare_solve(g, h, b)
    g.close()


def test_systems_errors_like_the_oracle():
    from oracle import oracle as orc
    from paper_2103_10476_amd import solver
    from paper_2103_10476_amd._lib import SaError
    p, X, B = _beam(12, 4, 4)
    assert p.n % 7 != 0
    cases = [dict(block_size=7, nullspace=B, kw={}),
             dict(block_size=3, nullspace=B, kw=dict(variants=("sprsfy",))),
             dict(block_size=3, nullspace=B, kw=dict(variants=("cnstrnt",))),
             dict(block_size=3, nullspace=np.where(np.arange(B.size).reshape(B.shape) == 7,
                                                   np.nan, B), kw={})]
    for c in cases:
        kw = dict(max_coarse=50, **c["kw"])
        with pytest.raises(orc.OracleError) as eo:
            orc.OracleHierarchy(p.n, p.rp, p.col, p.val, nullspace=c["nullspace"],
                                block_size=c["block_size"], **kw)
        with pytest.raises(SaError) as eg:
            solver.Hierarchy.from_problem(p, nullspace=c["nullspace"],
                                          block_size=c["block_size"],
                                          options=solver.Options(**kw))
        assert eg.value.code == eo.value.code == -1
    # an aggregate with fewer unknowns than nullspace vectors (corner aggregates of a cube)
    q = pb.fd7_stretched(8, 1.0)
    Bq = np.random.default_rng(0).normal(size=(q.n, 6))
    with pytest.raises(orc.OracleError) as eo:
        orc.OracleHierarchy(q.n, q.rp, q.col, q.val, nullspace=Bq, block_size=1, max_coarse=2)
    with pytest.raises(SaError) as eg:
        solver.Hierarchy.from_problem(q, nullspace=Bq, block_size=1,
                                      options=solver.Options(max_coarse=2))
    assert eg.value.code == eo.value.code == -1
    g = solver.Hierarchy.from_problem(p, nullspace=B, block_size=3,
                                      options=solver.Options(max_coarse=50))
    with pytest.raises(SaError):
        g.resetup(p.val, nullspace=B)
    g.close()


def test_elastic_beam_full_size():
    """The benchmark's elasticity cantilever (96 x 24 x 24 elements, 180,000 unknowns) with
    its six rigid-body modes: every level bitwise, CG to 1e-8 with equal iterations."""
    p, X, B = _beam(96, 24, 24)
    g, h = run_both(p, nullspace=B, block_size=3, cheb_boost=1.1, rtol=1e-8)
    compare_setup(g, h)
    it, _ = compare_solve(g, h, pb.random_rhs(p.n, 2))
    log(f"[systems] beam 96x24x24: levels {g.info()['n']}, {it} its, setup "
        f"{g.info()['setup_seconds'] * 1e3:.1f} ms")
    g.close()


def test_grouped_solve_over_systems_and_scalar_hierarchies():
    """sa_solve_many over a systems hierarchy, a scalar one and a distance-strength one gives
    each system's sa_solve result bit for bit."""
    from paper_2103_10476_amd import solver
    import torch
    p, X, B = _beam(16, 5, 5)
    q = pb.fd7_stretched(20, 1000.0)
    hs = [solver.Hierarchy.from_problem(p, nullspace=B, block_size=3,
                                        options=solver.Options(max_coarse=100, rtol=1e-10)),
          solver.Hierarchy.from_problem(q, options=solver.Options(max_coarse=60, rtol=1e-10)),
          solver.Hierarchy.from_problem(q, coords=pb.fd7_coords(20, 1000.0),
                                        options=solver.Options(max_coarse=60, rtol=1e-10,
                                                               precision="fp32"))]
    bs = [pb.random_rhs(p.n, 1), pb.random_rhs(q.n, 2), pb.random_rhs(q.n, 3)]
    alone = [h.solve(b) for h, b in zip(hs, bs)]
    grouped = solver.solve_many(hs, bs)
    for (xa, ia, ra, sa_), (xg, ig, rg, sg) in zip(alone, grouped):
        assert ia == ig and ra == rg and sa_ == sg
        assert torch.equal(xa, xg)
    for h in hs:
        h.close()
