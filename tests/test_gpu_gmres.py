"""GMRES (sa_solve_gmres) and the LU coarse solver through the C ABI against the oracle:
restarted flexible GMRES with the V-cycle as right preconditioner (the paper's solver for its
nonsymmetric systems, Sec. 3.4) on nonsymmetric upwind convection-diffusion cubes and on a
symmetric cube.  Hierarchies bitwise (the coarsest inverse to rounding, against numpy),
equal Arnoldi step counts, solutions to 1e-12; FP32 V-cycle within its bar; the error and
edge cases; a dense nonsymmetric coarsest level of 4096 unknowns; the 128^3 cube at full
size."""
import numpy as np
import pytest

from paper_2103_10476_amd import problems as pb
from parity import TOL_X, compare_setup, log, run_both

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def compare_gmres(g, h, b, restart, tol=TOL_X, its_slack=0):
    x, it, rr, status = g.solve_gmres(b, restart=restart)
    ref = h.solve_gmres(b, restart=restart)
    xg = x.cpu().numpy()
    err = np.linalg.norm(xg - ref["x"]) / np.linalg.norm(ref["x"])
    log(f"[gmres]   restart {restart}: steps gpu {it} oracle {ref['iterations']} rel err "
        f"{err:.2e} relres {rr:.3e} / {ref['rel_residual']:.3e}")
    assert abs(it - ref["iterations"]) <= its_slack, (it, ref["iterations"])
    assert (status == "SA_OK") == ref["converged"]
    assert err <= tol, err
    return it


CASES = [
    ("cd7 16^3 b(2,1,.5)", lambda: pb.cd7_upwind(16, 1.0, (2.0, 1.0, 0.5)), dict(max_coarse=60)),
    ("cd7 20^3 a100 strong convection", lambda: pb.cd7_upwind(20, 100.0, (40.0, -20.0, 10.0)),
     dict(max_coarse=80, variants=("offlmp", "1norm"))),
    ("cd7 17^3 all variants", lambda: pb.cd7_upwind(17, 10.0, (5.0, 5.0, -5.0)),
     dict(max_coarse=50, variants=("sprsfy", "offlmp", "1norm", "cnstrnt"))),
    ("cd7 24^3 hashed jacobi", lambda: pb.cd7_upwind(24, 1000.0, (1.0, 2.0, 3.0)),
     dict(max_coarse=100, agg_order="hashed", smoother="jacobi")),
]


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_gmres_nonsymmetric_matches_oracle(name, make, kw):
    p = make()
    g, h = run_both(p, coarse_solver="lu", rtol=1e-10, **kw)
    assert len(h.levels) >= 2
    compare_setup(g, h)
    b = pb.random_rhs(p.n, 11)
    for restart in (5, 30):
        compare_gmres(g, h, b, restart)
    g.close()


def test_gmres_symmetric_cholesky_and_restart_one():
    p = pb.fd7_stretched(17, 1000.0)
    g, h = run_both(p, max_coarse=40, rtol=1e-9, max_iter=300)
    compare_setup(g, h)
    b = pb.random_rhs(p.n, 4)
    for restart in (1, 3, 50):
        compare_gmres(g, h, b, restart)
    g.close()


def test_gmres_fp32_vcycle():
    from oracle import oracle as orc
    from paper_2103_10476_amd import solver
    p = pb.cd7_upwind(20, 100.0, (4.0, 2.0, 1.0))
    kw = dict(max_coarse=80, rtol=1e-10, coarse_solver="lu")
    g = solver.Hierarchy.from_problem(p, options=solver.Options(precision="fp32", **kw))
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, **kw)
    b = pb.random_rhs(p.n, 5)
    x, it, rr, st = g.solve_gmres(b, restart=30)
    ref = h.solve_gmres(b, restart=30)
    xg = x.cpu().numpy()
    A = p.to_dense() if p.n <= 4000 else None
    assert st == "SA_OK" and abs(it - ref["iterations"]) <= 2
    assert np.linalg.norm(xg - ref["x"]) <= 1e-8 * np.linalg.norm(ref["x"])
    rows = np.repeat(np.arange(p.n), np.diff(p.rp))
    Ax = np.zeros(p.n)
    np.add.at(Ax, rows, p.val * xg[p.col])
    assert np.linalg.norm(b - Ax) <= 2e-10 * np.linalg.norm(b)
    log(f"[gmres] fp32 V-cycle: {it} steps (fp64 oracle {ref['iterations']})")
    g.close()


def test_gmres_edges_and_errors():
    from oracle import oracle as orc
    from paper_2103_10476_amd import solver
    from paper_2103_10476_amd._lib import SaError
    p = pb.cd7_upwind(12, 10.0, (3.0, 1.0, 1.0))
    kw = dict(max_coarse=40, rtol=1e-14, max_iter=7, coarse_solver="lu")
    g, h = run_both(p, **kw)
    b = pb.random_rhs(p.n, 6)
    # the iteration cap, across a restart
    x, it, rr, st = g.solve_gmres(b, restart=3)
    ref = h.solve_gmres(b, restart=3)
    assert st == "SA_NOT_CONVERGED" and it == 7 and not ref["converged"]
    assert np.linalg.norm(x.cpu().numpy() - ref["x"]) <= 1e-12 * np.linalg.norm(ref["x"])
    # no iterations allowed: x = 0, not converged, on both sides
    g0, h0 = run_both(p, **dict(kw, max_iter=0))
    x, it, rr, st = g0.solve_gmres(b, restart=3)
    r0 = h0.solve_gmres(b, restart=3)
    assert it == 0 == r0["iterations"] and st == "SA_NOT_CONVERGED" and not r0["converged"]
    assert float(x.abs().max()) == 0.0 and np.all(r0["x"] == 0.0)
    g0.close()
    # zero right-hand side
    x, it, rr, st = g.solve_gmres(np.zeros(p.n), restart=3)
    assert st == "SA_OK" and it == 0 and float(x.abs().max()) == 0.0
    # restart out of range
    for r in (0, -2, 1025):
        with pytest.raises(SaError) as e:
            g.solve_gmres(b, restart=r)
        assert e.value.code == -1
    # a nonsymmetric coarsest operator under Cholesky fails on both sides
    with pytest.raises(SaError) as eg:
        solver.Hierarchy.from_problem(p, options=solver.Options(max_coarse=40))
    with pytest.raises(orc.OracleError) as eo:
        orc.OracleHierarchy(p.n, p.rp, p.col, p.val, max_coarse=40)
    assert eg.value.code == eo.value.code == -6
    g.close()


def test_dense_nonsymmetric_coarsest_of_4096():
    """A single level of 4096 unknowns solved by the blocked LU (64 blocks): the inverse
    against numpy's, and GMRES converging in one step."""
    from paper_2103_10476_amd import solver
    p = pb.cd7_upwind(16, 10.0, (8.0, -3.0, 2.0))
    g = solver.Hierarchy.from_problem(
        p, options=solver.Options(max_coarse=5000, coarse_solver="lu", rtol=1e-12))
    assert g.info()["levels"] == 1
    A = p.to_dense()
    inv = g.export(0, "coarse_inv").reshape(p.n, p.n)
    ref = np.linalg.inv(A)
    err = np.abs(inv - ref).max() / np.abs(ref).max()
    log(f"[gmres] dense LU 4096: max rel err of the inverse {err:.2e}")
    assert err <= 1e-12
    x, it, rr, st = g.solve_gmres(pb.random_rhs(p.n, 7), restart=10)
    assert st == "SA_OK" and it == 1
    g.close()


def test_gmres_full_size_cd7_128():
    """128^3 graded convection-diffusion cube (2,097,152 unknowns), OffLmp + 1Norm, LU coarse
    solver: hierarchy bitwise, GMRES(30) steps equal, solution to 1e-12."""
    p = pb.cd7_upwind(128, 1000.0, (1.0, 0.5, 0.25))
    g, h = run_both(p, coarse_solver="lu", variants=("offlmp", "1norm"), rtol=1e-8)
    compare_setup(g, h)
    it = compare_gmres(g, h, pb.random_rhs(p.n, 2), 30)
    log(f"[gmres] 128^3: levels {g.info()['n']} steps {it}")
    g.close()
