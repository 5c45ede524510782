"""The paper's test families (Sec. 3.2-3.3, App. A-B) against the oracle, with the
distance-Laplacian strength (theta = 0.025; weights 1/d and 1/d^2), Dirichlet right-hand
sides and CG to 1e-10:

* the randomly perturbed cube (Q1 on perturbed hexahedra, z stretched 100:1): all 16
  combinations of the adaptations on three seeds at 16^3 elements, and the paper's 60^3
  elements for three combinations;
* the triaxially stretched reaction-diffusion cube: the ten (kx, ky, kz) configurations at
  two reaction rates at 14^3 elements, and one configuration at 60^3 (Chebyshev interval end
  1.1 times the power estimate).

Every case: bitwise hierarchy (coordinates included), equal iterations, solution to 1e-12, or
the same failure status on both sides."""
import itertools

import pytest

from paper_2103_10476_amd import problems as pb
from parity import compare_setup, compare_solve, log, run_both

pytestmark = pytest.mark.gpu

NAMES = ("sprsfy", "offlmp", "1norm", "cnstrnt")
COMBOS = [tuple(n for n, on in zip(NAMES, bits) if on)
          for bits in itertools.product((0, 1), repeat=4)]
PAPER = dict(theta=0.025, max_coarse=1000, rtol=1e-10)
# the stretched cube with the literal [lambda/10, lambda] breaks CG down in most runs (ten power
# steps underestimate lambda on these meshes); its runs take the interval's end 1.1 lambda
STRETCH = dict(PAPER, cheb_boost=1.1)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _check(p, b, X, **kw):
    from oracle import oracle as orc
    from paper_2103_10476_amd import solver
    from paper_2103_10476_amd._lib import SaError
    try:
        g, h = run_both(p, coords=X, **kw)
    except (orc.OracleError, SaError):
        with pytest.raises(orc.OracleError) as eo:
            orc.OracleHierarchy(p.n, p.rp, p.col, p.val, coords=X, **kw)
        with pytest.raises(SaError) as eg:
            solver.Hierarchy.from_problem(p, options=solver.Options(**kw), coords=X)
        assert eg.value.code == eo.value.code
        log(f"[families]   both fail with {eg.value.code}")
        return None
    compare_setup(g, h)
    it, _ = compare_solve(g, h, b)
    g.close()
    return it


_MESHES = {}


def _perturbed(ne, seed):
    key = ("p", ne, seed)
    if key not in _MESHES:
        _MESHES[key] = pb.perturbed_cube(ne, seed)
    return _MESHES[key]


@pytest.mark.parametrize("var", COMBOS, ids=lambda v: "+".join(v) or "plain")
def test_perturbed_cube_all_combinations(var):
    for seed in range(3):
        p, b, X = _perturbed(16, seed)
        for pw in (1, 2):
            _check(p, b, X, variants=var, max_coarse=100, theta=0.025, rtol=1e-10,
                   dist_power=pw)


@pytest.mark.parametrize("var,pw", [((), 1), ((), 2), (("offlmp", "cnstrnt"), 2), (NAMES, 1)],
                         ids=["plain-1/d", "plain-1/d2", "offlmp+cnstrnt-1/d2", "all-1/d"])
def test_perturbed_cube_paper_size(var, pw):
    p, b, X = _perturbed(60, 1)
    it = _check(p, b, X, variants=var, dist_power=pw, **PAPER)
    log(f"[families] perturbed 60^3 seed 1 {'+'.join(var) or 'plain'} 1/d^{pw}: "
        f"iterations {it}")


@pytest.mark.parametrize("cfg", pb.STRETCH_CONFIGS, ids=lambda c: "k%d%d%d" % c)
def test_stretched_cube_configurations(cfg):
    for sigma in (1e1, 1e5):
        p, b, X = pb.stretched_cube(*cfg, sigma, ne=14)
        for var, pw in (((), 1), (("1norm",), 1), (("offlmp",), 1), ((), 2), (("1norm",), 2)):
            _check(p, b, X, variants=var, dist_power=pw, **dict(STRETCH, max_coarse=100))


def test_stretched_cube_paper_size():
    p, b, X = pb.stretched_cube(1, 5, 10, 1e3, ne=60)
    for var, pw in (((), 1), (("1norm",), 1), ((), 2), (("1norm",), 2)):
        it = _check(p, b, X, variants=var, dist_power=pw, **STRETCH)
        log(f"[families] stretched (1,5,10) sigma 1e3 60^3 {'+'.join(var) or 'plain'} "
            f"1/d^{pw}: iterations {it}")
