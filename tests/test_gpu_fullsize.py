"""GPU parity at the benchmark's full sizes, in the configuration bench.py times: the whole
hierarchy (every level's arrays and scalars) is compared bit for bit with the oracle's, and the
solve gives the same iteration count and x within 1e-12 relative."""
import pytest

from paper_2103_10476_amd import problems as pb
from parity import compare_setup, compare_solve, run_both

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def c2():
    return pb.workload("fd7_128_a1000"), pb.random_rhs(2097152, pb.RHS_SEED["fd7_128_a1000"])


@pytest.mark.parametrize("var", [[], ["sprsfy"], ["offlmp"], ["1norm"], ["cnstrnt"]],
                         ids=lambda v: "+".join(v) or "plain")
def test_fd7_128_a1000_each_variant(c2, var):
    """The 128^3 z-stretched cube (aspect 1:1000), theta = 0.02, one setup per variant."""
    p, b = c2
    g, h = run_both(p, theta=0.02, variants=var, rtol=1e-8)
    compare_setup(g, h)
    compare_solve(g, h, b)


def test_q1_100_randkappa_offlmp_1norm():
    """27-point Q1 cube, 100^3 elements, kappa = 10^U[-3,3]: OffLmp + 1Norm."""
    p = pb.workload("q1_100_randkappa")
    b = pb.random_rhs(p.n, pb.RHS_SEED["q1_100_randkappa"])
    g, h = run_both(p, theta=0.02, variants=["offlmp", "1norm"], rtol=1e-8)
    compare_setup(g, h)
    compare_solve(g, h, b)


def test_stress_box_24_all_variants():
    from fractions import Fraction
    p = pb.q1_stretched_box(24, Fraction(2))
    b = pb.random_rhs(p.n, 7)
    g, h = run_both(p, theta=0.15, variants=["offlmp", "1norm", "cnstrnt", "sprsfy"], rtol=1e-10)
    compare_setup(g, h)
    compare_solve(g, h, b)


@pytest.fixture(scope="module")
def c4():
    return pb.workload("fd7_160_a1000"), pb.random_rhs(4096000, pb.RHS_SEED["fd7_160_a1000"])


def test_fd7_160_a1000_fp64_and_fp32_vcycle(c4):
    """The 160^3 z-stretched cube (aspect 1:1000) at rtol 1e-10: the FP64 hierarchy bit for
    bit and its solve (iterations equal, x within 1e-12); then the FP32-V-cycle solve of the
    same hierarchy against the FP64 oracle's solution, to the FP32 mode's stated tolerances
    (iterations within 2, true relative residual at most 2 rtol, x within 1e-8)."""
    import numpy as np
    import scipy.sparse as sp
    from paper_2103_10476_amd import solver
    from parity import log
    p, b = c4
    rtol = 1e-10
    g, h = run_both(p, theta=0.02, rtol=rtol)
    compare_setup(g, h)
    compare_solve(g, h, b)
    g.close()
    ref = h.solve(b)
    f = solver.Hierarchy.from_problem(p, options=solver.Options(theta=0.02, rtol=rtol,
                                                                precision="fp32"))
    x, it, rr, st = f.solve(b)
    xg = x.cpu().numpy()
    f.close()
    A = sp.csr_matrix((p.val, p.col, p.rp), shape=(p.n, p.n))
    true_res = np.linalg.norm(b - A @ xg) / np.linalg.norm(b)
    err = np.linalg.norm(xg - ref["x"]) / np.linalg.norm(ref["x"])
    log(f"[fp32] fd7_160_a1000: iterations {it} (oracle FP64 {ref['iterations']}), true "
        f"residual {true_res:.2e}, error vs oracle {err:.2e}")
    assert st == "SA_OK" and ref["converged"]
    assert abs(it - ref["iterations"]) <= 2
    assert true_res <= 2 * rtol
    assert err <= 1e-8
