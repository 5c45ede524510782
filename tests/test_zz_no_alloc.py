"""sa_solve_gmres_noalloc (no device allocation; workspace in the library's fixed scratch
array) against sa_solve_gmres through the C ABI: the same kernels in the same order on the
same hierarchy, so iterations, residual and x must be identical bit for bit.  Two calls in a
row, the second on a smaller system with a shorter restart, so the second call runs over
what the first left in the array; an FP32-V-cycle hierarchy; a nonsymmetric operator; and
a workspace beyond the array's 128 MiB refused before anything runs."""
import numpy as np
import pytest

from paper_2103_10476_amd import problems as pb

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _pair(h, b, restart):
    xa, ita, rra, sta = h.solve_gmres(b, restart=restart)
    xn, itn, rrn, stn = h.solve_gmres(b, restart=restart, noalloc=True)
    xa, xn = xa.cpu().numpy(), xn.cpu().numpy()
    print(f"[noalloc] n={h.n} restart={restart}: {ita} steps {sta} / {itn} steps {stn}",
          flush=True)
    assert (ita, rra, sta) == (itn, rrn, stn)
    assert np.array_equal(xa.view(np.uint64), xn.view(np.uint64))
    return ita


def test_noalloc_matches_allocating_gmres_twice_shrinking():
    from paper_2103_10476_amd import solver
    big = pb.fd7_stretched(40, 1000.0)        # n = 64,000, restart 30: about 32 MB
    small = pb.fd7_stretched(18, 100.0)       # n = 5,832, restart 12
    hb = solver.Hierarchy.from_problem(big, options=solver.Options(rtol=1e-10))
    hs = solver.Hierarchy.from_problem(small, options=solver.Options(rtol=1e-10))
    assert _pair(hb, pb.random_rhs(big.n, 3), 30) > 0
    assert _pair(hs, pb.random_rhs(small.n, 4), 12) > 0
    # and back to the larger one, over the smaller call's leftovers
    assert _pair(hb, pb.random_rhs(big.n, 5), 30) > 0
    hb.close()
    hs.close()


def test_noalloc_fp32_vcycle_and_nonsymmetric():
    from paper_2103_10476_amd import solver
    p = pb.cd7_upwind(20, 100.0, (1.0, 0.5, 0.25))
    o = solver.Options(variants=("offlmp", "1norm"), coarse_solver="lu", rtol=1e-8,
                       precision="fp32")
    h = solver.Hierarchy.from_problem(p, options=o)
    assert _pair(h, pb.random_rhs(p.n, 6), 20) > 0
    h.close()


def test_noalloc_refuses_a_workspace_beyond_the_array():
    from paper_2103_10476_amd import solver
    from paper_2103_10476_amd._lib import SaError
    p = pb.fd7_stretched(40, 1000.0)          # n = 64,000: restart 200 needs about 206 MB
    h = solver.Hierarchy.from_problem(p, options=solver.Options(rtol=1e-10))
    with pytest.raises(SaError) as e:
        h.solve_gmres(pb.random_rhs(p.n, 3), restart=200, noalloc=True)
    assert e.value.code == -1 and "scratch" in str(e.value)
    x, it, _, st = h.solve_gmres(pb.random_rhs(p.n, 3), restart=200)  # the allocating call runs
    assert st == "SA_OK" and it > 0
    h.close()
