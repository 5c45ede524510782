"""Oracle pins for restarted flexible GMRES with the SA V-cycle as right preconditioner (the
solver the paper uses for its nonsymmetric wind-turbine systems, Sec. 3.4).

* With an exact preconditioner (a single level, solved directly) GMRES converges in one step
  to A^{-1} b.
* Minimal-residual property: after k Arnoldi steps (no restart) the reported residual equals
  min ||b - A x|| over x in M^{-1} K_k(A M^{-1}, b), computed independently with numpy's least
  squares on an explicit Krylov basis.
* Within a cycle the residual never grows; a converged solve meets the tolerance on the true
  residual; any restart length at least the iteration count gives the same iterate; the
  iteration cap, a zero right-hand side and bad arguments behave as documented.
"""
import numpy as np
import pytest

from paper_2103_10476_amd import problems as pb


def _dense(p):
    return p.to_dense()


def test_exact_preconditioner_one_step(orc):
    p = pb.cd7_upwind(6, 1.0, (3.0, -2.0, 1.0))
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, max_coarse=1000, rtol=1e-12,
                            coarse_solver="lu")
    assert len(h.levels) == 1
    b = pb.random_rhs(p.n, 1)
    r = h.solve_gmres(b, restart=10)
    assert r["converged"] and r["iterations"] == 1
    ref = np.linalg.solve(_dense(p), b)
    assert np.linalg.norm(r["x"] - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("beta", [(0.0, 0.0, 0.0), (2.0, 1.0, -4.0)])
def test_minimal_residual_property(orc, beta):
    p = pb.cd7_upwind(9, 10.0, beta)
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, max_coarse=50, rtol=1e-14, max_iter=6,
                            coarse_solver="lu")
    assert len(h.levels) >= 2
    A = _dense(p)
    b = pb.random_rhs(p.n, 2)
    r = h.solve_gmres(b, restart=30, history=True)
    hist = r["history"]
    assert r["iterations"] == 6 and len(hist) == 7
    # explicit Krylov basis of A M^-1, orthonormalised column by column
    U = np.zeros((p.n, 6))
    u = b / np.linalg.norm(b)
    for k in range(6):
        U[:, k] = u
        U[:, : k + 1], _ = np.linalg.qr(U[:, : k + 1])
        u = A @ h.vcycle(U[:, k])
        u /= np.linalg.norm(u)
    for k in range(1, 7):
        X = np.stack([h.vcycle(U[:, i]) for i in range(k)], axis=1)   # M^-1 U_k
        y, *_ = np.linalg.lstsq(A @ X, b, rcond=None)
        best = np.linalg.norm(b - A @ (X @ y))
        assert abs(hist[k] - best) <= 1e-7 * np.linalg.norm(b), (k, hist[k], best)
    assert np.all(np.diff(hist) <= 1e-14 * hist[0])


def test_converged_solution_and_restarts(orc):
    p = pb.cd7_upwind(12, 100.0, (2.0, 1.0, 0.5))
    A = _dense(p)
    b = pb.random_rhs(p.n, 3)
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, max_coarse=60, rtol=1e-10,
                            variants=("offlmp", "1norm"), coarse_solver="lu")
    full = h.solve_gmres(b, restart=200)
    assert full["converged"]
    it = full["iterations"]
    assert np.linalg.norm(b - A @ full["x"]) <= 1.0001e-10 * np.linalg.norm(b)
    ref = np.linalg.solve(A, b)
    assert np.linalg.norm(full["x"] - ref) <= 1e-8 * np.linalg.norm(ref)
    # any restart length >= the iteration count runs the same single cycle
    again = h.solve_gmres(b, restart=it)
    assert again["iterations"] == it and np.array_equal(again["x"], full["x"])
    # short restarts still converge (more steps), and the reported residual is the true one
    # after the last restart or the cycle's least-squares one
    short = h.solve_gmres(b, restart=3, history=True)
    assert short["converged"] and short["iterations"] >= it
    assert np.linalg.norm(b - A @ short["x"]) <= 1.0001e-10 * np.linalg.norm(b)


def test_iteration_cap_zero_rhs_and_arguments(orc):
    p = pb.cd7_upwind(10, 10.0)
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, max_coarse=50, rtol=1e-14, max_iter=4,
                            coarse_solver="lu")
    r = h.solve_gmres(pb.random_rhs(p.n, 5), restart=3)
    assert not r["converged"] and r["iterations"] == 4
    z = h.solve_gmres(np.zeros(p.n), restart=3)
    assert z["converged"] and z["iterations"] == 0 and np.all(z["x"] == 0)
    with pytest.raises(orc.OracleError):
        h.solve_gmres(pb.random_rhs(p.n, 5), restart=0)


def test_symmetric_problem_matches_cg_solution(orc):
    p = pb.fd7_stretched(12, 1000.0)
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, max_coarse=60, rtol=1e-11)
    b = pb.random_rhs(p.n, 6)
    g = h.solve_gmres(b, restart=50)
    c = h.solve(b)
    assert g["converged"] and c["converged"]
    assert np.linalg.norm(g["x"] - c["x"]) <= 1e-8 * np.linalg.norm(c["x"])


def test_cd7_generator_is_the_upwind_operator():
    # zero velocity gives the diffusion matrix; otherwise rows sum to zero inside, the
    # velocity part is skew-symmetric up to the upwind diagonal, and the matrix is an M-matrix
    assert np.array_equal(pb.cd7_upwind(7, 10.0, (0, 0, 0)).val, pb.fd7_stretched(7, 10.0).val)
    p = pb.cd7_upwind(7, 1.0, (3.0, 0.0, 0.0))
    A = _dense(p)
    off = A - np.diag(np.diag(A))
    assert np.all(off <= 0.0)
    inner = [i + 7 * (j + 7 * k) for i in range(1, 6) for j in range(1, 6) for k in range(1, 6)]
    assert np.abs(A.sum(axis=1)[inner]).max() <= 1e-13
    D = pb.fd7_stretched(7, 1.0).to_dense()
    C = A - D                                  # the convective part
    h = 1.0 / 8
    # upstream (west) neighbour carries -beta_x * face area, downstream nothing
    i = inner[0]
    assert abs(C[i, i - 1] + 3.0 * h * h) <= 1e-15 and C[i, i + 1] == 0.0
    assert abs(C[i, i] - 3.0 * h * h) <= 1e-15


def test_coarse_lu_solver(orc):
    """The LU coarse solver: a single level is solved exactly (vs numpy), the Cholesky solver
    refuses a nonsymmetric coarsest operator, and on a symmetric problem both solvers give the
    same hierarchy and the same solution to rounding."""
    p = pb.cd7_upwind(5, 3.0, (4.0, -1.0, 2.0))
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, max_coarse=1000, coarse_solver="lu")
    f = pb.random_rhs(p.n, 9)
    ref = np.linalg.solve(_dense(p), f)
    assert np.linalg.norm(h.vcycle(f) - ref) <= 1e-13 * np.linalg.norm(ref)
    with pytest.raises(orc.OracleError) as e:
        orc.OracleHierarchy(p.n, p.rp, p.col, p.val, max_coarse=1000)
    assert e.value.code == -6
    # the nonsymmetric coarsest level of a two-level hierarchy, too
    q = pb.cd7_upwind(10, 3.0, (4.0, -1.0, 2.0))
    with pytest.raises(orc.OracleError):
        orc.OracleHierarchy(q.n, q.rp, q.col, q.val, max_coarse=200)
    s = pb.fd7_stretched(10, 100.0)
    hc = orc.OracleHierarchy(s.n, s.rp, s.col, s.val, max_coarse=200, rtol=1e-10)
    hl = orc.OracleHierarchy(s.n, s.rp, s.col, s.val, max_coarse=200, rtol=1e-10,
                             coarse_solver="lu")
    b = pb.random_rhs(s.n, 4)
    rc, rl = hc.solve(b), hl.solve(b)
    assert rc["iterations"] == rl["iterations"]
    assert np.linalg.norm(rc["x"] - rl["x"]) <= 1e-12 * np.linalg.norm(rc["x"])
