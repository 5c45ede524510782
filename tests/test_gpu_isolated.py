"""The covering reading of the aggregates (Sec. 1.1, eq. (aggregates); option isolated =
"singleton"): every vertex without strong connections becomes an aggregate of its own, on
the GPU exactly as in the oracle -- every level's arrays bitwise, the solve with equal
iterations and x within 1e-12, or the same failure status on both sides."""
import numpy as np
import pytest

from paper_2103_10476_amd import problems as pb
from parity import compare_setup, compare_solve, log, run_both

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _jitter(X, scale, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return X + rng.uniform(-scale, scale, size=X.shape)


CASES = [
    ("q1 kappa 14 offlmp+1norm", lambda: (pb.q1_random_kappa(14, seed=3), None),
     dict(variants=("offlmp", "1norm"), max_coarse=50, cheb_boost=1.1)),
    ("q1 kappa 14 sprsfy+cnstrnt+offlmp+1norm", lambda: (pb.q1_random_kappa(14, seed=5), None),
     dict(variants=("sprsfy", "cnstrnt", "offlmp", "1norm"), max_coarse=50, cheb_boost=1.1)),
    ("fd7 32 a1000 1norm", lambda: (pb.fd7_stretched(32, 1000.0), None),
     dict(variants=("1norm",))),
    ("fd7 24 a1000 hashed (coarsening stalls)", lambda: (pb.fd7_stretched(24, 1000.0), None),
     dict(agg_order="hashed", seed=5, max_coarse=60)),
    ("q1 18 distance theta .08 hashed 1norm",
     lambda: (pb.q1_hex(18), _jitter(pb.q1_coords(18), 0.02, 4)),
     dict(theta=0.08, max_coarse=40, agg_order="hashed", seed=77, variants=("1norm",))),
]


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_singleton_reading_matches_oracle(name, make, kw):
    p, X = make()
    kw = dict(kw)
    kw.setdefault("theta", 0.02)
    g, h = run_both(p, coords=X, rtol=1e-10, isolated="singleton", **kw)
    assert len(h.levels) >= 2
    compare_setup(g, h)
    compare_solve(g, h, pb.random_rhs(p.n, 23))
    g.close()


def test_singleton_zero_lumped_diagonal_fails_like_the_oracle():
    """Plain SA with the covering reading on a jittered Q1 mesh (distance strength, theta
    0.08): a singleton on a coarse level whose row sums to zero gets a zero filtered diagonal
    under plain lumping (the small-diagonal failure of Sec. 1.2); both sides report it."""
    from oracle import oracle as orc
    from paper_2103_10476_amd import solver
    from paper_2103_10476_amd._lib import SaError
    p, X = pb.q1_hex(18), _jitter(pb.q1_coords(18), 0.02, 4)
    kw = dict(theta=0.08, max_coarse=40, agg_order="hashed", seed=77, isolated="singleton")
    with pytest.raises(orc.OracleError) as eo:
        orc.OracleHierarchy(p.n, p.rp, p.col, p.val, coords=X, rtol=1e-10, **kw)
    with pytest.raises(SaError) as eg:
        solver.Hierarchy.from_problem(p, options=solver.Options(rtol=1e-10, **kw), coords=X)
    log(f"[isolated] both fail: oracle {eo.value.code}, gpu {eg.value.code}")
    assert eo.value.code == eg.value.code == -3
