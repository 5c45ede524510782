"""All 16 combinations of the four adaptations (Sprsfy, OffLmp, 1Norm, Cnstrnt; the layout of
the paper's Table 1) against the oracle, on the Sec. 1.2 stress problem (Q1 on 1x1x2 boxes,
theta = 0.15) and a random-coefficient Q1 cube: bitwise hierarchies, equal iterations,
solutions to 1e-12, or the same failure on both sides."""
import itertools

import pytest

from paper_2103_10476_amd import problems as pb
from parity import compare_setup, compare_solve, log, run_both

pytestmark = pytest.mark.gpu

NAMES = ("sprsfy", "offlmp", "1norm", "cnstrnt")
COMBOS = [tuple(n for n, on in zip(NAMES, bits) if on)
          for bits in itertools.product((0, 1), repeat=4)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _both_or_same_failure(p, b, **kw):
    from oracle import oracle as orc
    from paper_2103_10476_amd._lib import SaError
    try:
        g, h = run_both(p, **kw)
    except (orc.OracleError, SaError) as e:
        # the method can fail on these inputs (Sec. 1.2); then both sides must fail alike
        from paper_2103_10476_amd import solver
        with pytest.raises(orc.OracleError) as eo:
            orc.OracleHierarchy(p.n, p.rp, p.col, p.val, **kw)
        with pytest.raises(SaError) as eg:
            solver.Hierarchy.from_problem(p, options=solver.Options(**kw))
        assert eg.value.code == eo.value.code
        log(f"[sweep]   both fail with {eg.value.code}")
        return
    compare_setup(g, h)
    compare_solve(g, h, b)


@pytest.mark.parametrize("var", COMBOS, ids=lambda v: "+".join(v) or "plain")
def test_stress_box_all_combinations(var):
    from fractions import Fraction
    p = pb.q1_stretched_box(12, Fraction(2))
    _both_or_same_failure(p, pb.random_rhs(p.n, 7), theta=0.15, variants=var, max_coarse=30,
                          rtol=1e-10)


@pytest.mark.parametrize("var", COMBOS, ids=lambda v: "+".join(v) or "plain")
def test_random_kappa_all_combinations(var):
    p = pb.q1_random_kappa(14, seed=9)
    _both_or_same_failure(p, pb.random_rhs(p.n, 8), theta=0.02, variants=var, max_coarse=60,
                          rtol=1e-10, cheb_boost=1.1)
