"""FP32 V-cycle mode through the C ABI, against the FP64 oracle.

In this mode the hierarchy is built exactly as in FP64 (the setup is bitwise the oracle's);
P, R, every level operator and the smoother diagonals are then stored and applied in FP32,
while CG, the fine residual, the eigenvalue estimates and the coarsest solve stay FP64.  So
the solve differs from the oracle's by the FP32 rounding of the preconditioner only: CG
(flexible, Polak-Ribiere) still reaches the same residual, in about the same number of
iterations, at a solution the residual bound ties to the oracle's.

Tolerances (written out here): iterations within 2 of the FP64 oracle's; true relative
residual ||b - A x|| / ||b|| at most 2 rtol; ||x - x_oracle|| / ||x_oracle|| at most 1e-8
(two solutions with residuals below 1e-10 on these matrices, whose condition numbers stay
below ~1e6, cannot differ by more)."""
import numpy as np
import pytest

from paper_2103_10476_amd import problems as pb
from parity import compare_setup, log, run_both

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


CASES = [
    ("fd5_64x64_a100", dict(variants=())),
    ("fd7_24_a1000", dict(variants=())),
    ("fd7_24_a1000_1norm", dict(variants=("1norm",))),
    ("q1_randkappa_14", dict(variants=("offlmp", "1norm"), cheb_boost=1.1)),
]


def _problem(name):
    if name == "fd5_64x64_a100":
        return pb.workload(name)
    if name.startswith("fd7_24"):
        return pb.fd7_stretched(24, 1000.0)
    return pb.q1_random_kappa(15, seed=3)


@pytest.mark.parametrize("name,kw", CASES, ids=[c[0] for c in CASES])
def test_fp32_vcycle_against_fp64_oracle(name, kw):
    import scipy.sparse as sp
    p = _problem(name)
    b = pb.random_rhs(p.n, 9)
    rtol = 1e-10
    g, h = run_both(p, theta=0.02, rtol=rtol, precision="fp32", pcg_beta="pr", **kw)
    compare_setup(g, h)  # the FP32 mode builds the same hierarchy
    x, it, rr, st = g.solve(b)
    ref = h.solve(b)
    xg = x.cpu().numpy()
    A = sp.csr_matrix((p.val, p.col, p.rp), shape=(p.n, p.n))
    true_res = np.linalg.norm(b - A @ xg) / np.linalg.norm(b)
    err = np.linalg.norm(xg - ref["x"]) / np.linalg.norm(ref["x"])
    log(f"[fp32] {name}: iterations {it} (oracle FP64 {ref['iterations']}), true residual "
        f"{true_res:.2e}, error vs oracle {err:.2e}")
    assert st == "SA_OK" and ref["converged"]
    assert abs(it - ref["iterations"]) <= 2
    assert true_res <= 2 * rtol
    assert err <= 1e-8


def test_fp32_and_fp64_modes_share_the_hierarchy():
    """Switching precision changes nothing in setup: every exported array is identical."""
    from paper_2103_10476_amd import solver
    p = pb.fd7_stretched(17, 1000.0)
    a = solver.Hierarchy.from_problem(p, options=solver.Options(precision="fp64"))
    f = solver.Hierarchy.from_problem(p, options=solver.Options(precision="fp32"))
    assert a.info()["levels"] == f.info()["levels"]
    for l in range(a.info()["levels"]):
        for part in ("A_val", "P_val", "R_val", "sm_invD"):
            assert np.array_equal(a.export(l, part), f.export(l, part)), (l, part)
