"""Distance-Laplacian strength (Sec. 3.1) through sa_setup_coords against the oracle: the
labels, aggregates, every level's arrays and the coarse coordinates (aggregate centroids)
bitwise, the solve to 1e-12 with equal iterations; the same failures on bad coordinates; the
numeric re-setup keeps the distance labels; the 128^3 stretched cube at full size."""
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
    ("fd7 17^3 a1000", lambda: (pb.fd7_stretched(17, 1000.0), pb.fd7_coords(17, 1000.0)),
     dict(max_coarse=40)),
    ("fd7 17^3 a1000 all variants",
     lambda: (pb.fd7_stretched(17, 1000.0), pb.fd7_coords(17, 1000.0)),
     dict(max_coarse=40, variants=("sprsfy", "offlmp", "1norm", "cnstrnt"))),
    ("fd5 64x64 a100 (2-D)", lambda: (pb.fd5_stretched(64, 64, 100.0), pb.fd5_coords(64, 64, 100.0)),
     dict(max_coarse=50)),
    ("fd7 1x1x300 (1-D)", lambda: (pb.fd7_stretched(300, 50.0, nx=1, ny=1),
                                   pb.fd7_coords(300, 50.0, nx=1, ny=1)[:, 2:].copy()),
     dict(max_coarse=10)),
    ("q1 box 12 theta .15", lambda: (pb.q1_stretched_box(12), pb.q1_coords(13, 1, 1, 2)),
     dict(theta=0.15, max_coarse=30, variants=("offlmp", "1norm"), cheb_boost=1.1)),
    ("q1 kappa 14 jittered mesh", lambda: (pb.q1_random_kappa(14, seed=9),
                                           _jitter(pb.q1_coords(14), 0.01, 3)),
     dict(max_coarse=60, variants=("offlmp", "1norm"), cheb_boost=1.1)),
    ("q1 18 theta .08 hashed order", lambda: (pb.q1_hex(18), _jitter(pb.q1_coords(18), 0.02, 4)),
     dict(theta=0.08, max_coarse=40, agg_order="hashed", seed=77)),
    # weights 1/d^2 (no square root)
    ("fd7 17^3 a1000 power 2", lambda: (pb.fd7_stretched(17, 1000.0), pb.fd7_coords(17, 1000.0)),
     dict(max_coarse=40, dist_power=2)),
    ("q1 kappa 14 jittered power 2", lambda: (pb.q1_random_kappa(14, seed=9),
                                              _jitter(pb.q1_coords(14), 0.01, 3)),
     dict(max_coarse=60, variants=("offlmp", "1norm"), cheb_boost=1.1, dist_power=2)),
    ("perturbed cube 20 power 2", lambda: pb.perturbed_cube(20, 5)[::2],
     dict(theta=0.025, max_coarse=100, variants=("offlmp",), dist_power=2)),
]


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_distance_strength_matches_oracle(name, make, kw):
    p, X = make()  # (problem, coordinates)
    g, h = run_both(p, coords=X, rtol=1e-10, **kw)
    assert len(h.levels) >= 2, name
    compare_setup(g, h)
    compare_solve(g, h, pb.random_rhs(p.n, 21))
    g.close()


def test_single_level_keeps_coordinates():
    p = pb.fd7_stretched(6, 10.0)
    X = pb.fd7_coords(6, 10.0)
    g, h = run_both(p, coords=X, max_coarse=1000)
    assert g.info()["levels"] == 1
    assert np.array_equal(g.export(0, "coords").reshape(p.n, 3), X)
    compare_setup(g, h)
    compare_solve(g, h, pb.random_rhs(p.n, 2))


def test_bad_coordinates_fail_like_the_oracle():
    from oracle import oracle as orc
    from paper_2103_10476_amd import solver
    from paper_2103_10476_amd._lib import SaError
    p = pb.fd7_stretched(8, 10.0)
    X = pb.fd7_coords(8, 10.0)
    bad_same = X.copy()
    bad_same[9] = bad_same[10]          # x-neighbours at one point
    bad_nan = X.copy()
    bad_nan[5, 2] = np.inf
    for Y, pw in ((bad_same, 1), (bad_same, 2), (bad_nan, 1),
                  (np.zeros((p.n, 4)) + np.arange(p.n)[:, None], 1), (X, 3)):
        with pytest.raises(orc.OracleError) as eo:
            orc.OracleHierarchy(p.n, p.rp, p.col, p.val, coords=Y, max_coarse=20,
                                dist_power=pw)
        with pytest.raises(SaError) as eg:
            solver.Hierarchy.from_problem(p, options=solver.Options(max_coarse=20,
                                                                    dist_power=pw), coords=Y)
        assert eg.value.code == eo.value.code == -1
    # the library still works afterwards
    g = solver.Hierarchy.from_problem(p, options=solver.Options(max_coarse=20), coords=X)
    assert g.solve(pb.random_rhs(p.n, 1))[3] == "SA_OK"


def test_resetup_keeps_distance_labels():
    from oracle import oracle as orc
    from paper_2103_10476_amd import solver
    p = pb.q1_random_kappa(13, seed=5)
    X = _jitter(pb.q1_coords(13), 0.01, 8)
    kw = dict(max_coarse=60, variants=("offlmp", "1norm"), cheb_boost=1.1, rtol=1e-10)
    g = solver.Hierarchy.from_problem(p, options=solver.Options(**kw), coords=X)
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, coords=X, **kw)
    rng = np.random.Generator(np.random.PCG64(3))
    d = rng.uniform(0.5, 2.0, size=p.n)
    rows = np.repeat(np.arange(p.n), np.diff(p.rp))
    val2 = (d[rows] * p.val) * d[p.col]
    g.resetup(val2)
    h.resetup(val2)
    compare_setup(g, h)
    compare_solve(g, h, pb.random_rhs(p.n, 5))
    # the distance labels do not depend on the values: a fresh setup on the new values takes
    # the same symbolic decisions on level 0
    fresh = solver.Hierarchy.from_problem(
        pb.CsrProblem(p.n, p.rp, p.col, val2), options=solver.Options(**kw), coords=X)
    assert np.array_equal(fresh.export(0, "mask"), g.export(0, "mask"))
    assert np.array_equal(fresh.export(0, "agg"), g.export(0, "agg"))
    g.close()
    fresh.close()


def test_full_size_fd7_128_distance():
    """128^3 graded cube with its node coordinates.  Weights 1/d: plain SA's prolongator
    eigenvalue estimate turns negative on both sides (the failure the adaptations address);
    weights 1/d^2: every level bitwise, solve to 1e-12."""
    from oracle import oracle as orc
    from paper_2103_10476_amd import solver
    from paper_2103_10476_amd._lib import SaError
    p = pb.workload("fd7_128_a1000")
    X = pb.fd7_coords(128, 1000.0)
    with pytest.raises(SaError) as eg:
        solver.Hierarchy.from_problem(p, options=solver.Options(), coords=X)
    with pytest.raises(orc.OracleError) as eo:
        orc.OracleHierarchy(p.n, p.rp, p.col, p.val, coords=X)
    assert eg.value.code == eo.value.code == -4
    g, h = run_both(p, coords=X, dist_power=2)
    compare_setup(g, h)
    it, _ = compare_solve(g, h, pb.random_rhs(p.n, pb.RHS_SEED["fd7_128_a1000"]))
    log(f"[distance] 128^3: levels {g.info()['n']} iterations {it} setup "
        f"{g.info()['setup_seconds'] * 1e3:.1f} ms")
    g.close()
