"""Numeric re-setup (sa_resetup) through the C ABI against the oracle's re-setup: after new
values on the setup's pattern, every level array is bitwise the oracle's, and the solve
matches to 1e-12 with equal iterations.  Also: on two-level hierarchies the re-setup equals a
fresh GPU setup on the new values bit for bit, a failed re-setup leaves the hierarchy
refusing solves until a good one, and at 128^3 the re-setup skips root selection."""
import time

import numpy as np
import pytest

from paper_2103_10476_amd import problems as pb
from parity import compare_setup, compare_solve, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dad(p, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    d = rng.uniform(0.5, 2.0, size=p.n)
    rows = np.repeat(np.arange(p.n), np.diff(p.rp))
    return (d[rows] * p.val) * d[p.col]


CASES = [
    ("fd7 17^3 plain", lambda: pb.fd7_stretched(17, 1000.0), dict(max_coarse=40)),
    ("fd7 17^3 all variants", lambda: pb.fd7_stretched(17, 1000.0),
     dict(max_coarse=40, variants=("sprsfy", "offlmp", "1norm", "cnstrnt"))),
    ("q1 kappa 12 offlmp+1norm", lambda: pb.q1_random_kappa(13, seed=5),
     dict(max_coarse=60, variants=("offlmp", "1norm"))),
    ("fd5 64x64 nullspace", lambda: pb.workload("fd5_64x64_a100"), dict(max_coarse=50)),
]


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_resetup_matches_oracle(name, make, kw):
    from oracle import oracle as orc
    from paper_2103_10476_amd import solver
    p = make()
    B = None
    if "nullspace" in name:
        B = 1.0 + 0.5 * np.sin(np.arange(p.n) * 0.1)
    g = solver.Hierarchy.from_problem(p, nullspace=B, options=solver.Options(**kw))
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, nullspace=B, **kw)
    for k, val in enumerate([_dad(p, 3), 3.0 * p.val + 0.0, _dad(p, 4)]):
        B2 = None if B is None else B[::-1].copy()
        g.resetup(val, nullspace=B2)
        h.resetup(val, nullspace=B2)
        log(f"[resetup] {name}: values set {k}")
        compare_setup(g, h)
        compare_solve(g, h, pb.random_rhs(p.n, 10 + k))
    g.close()


def test_resetup_equals_fresh_setup_two_levels():
    from paper_2103_10476_amd import solver
    p = pb.fd7_stretched(20, 1000.0)
    o = solver.Options(max_coarse=3000, variants=("offlmp", "1norm"))
    val2 = _dad(p, 8)
    g = solver.Hierarchy.from_problem(p, options=o)
    assert g.info()["levels"] == 2
    fresh = solver.Hierarchy(p.n, p.rp, p.col, val2, options=o)
    assert np.array_equal(g.export(0, "agg"), fresh.export(0, "agg"))
    g.resetup(val2)
    for l in range(2):
        for part in ("A_val", "P_val", "R_val", "Abar_val", "invD", "sm_invD", "coarse_inv"):
            a, b = g.export(l, part), fresh.export(l, part)
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), (l, part)
    x1 = g.solve(pb.random_rhs(p.n, 1))[0].cpu().numpy()
    x2 = fresh.solve(pb.random_rhs(p.n, 1))[0].cpu().numpy()
    assert np.array_equal(x1, x2)


def test_failed_resetup_then_recovery():
    from paper_2103_10476_amd import solver
    from paper_2103_10476_amd._lib import SaError
    p = pb.fd7_stretched(12, 100.0)
    g = solver.Hierarchy.from_problem(p, options=solver.Options(max_coarse=40))
    bad = p.val.copy()
    bad[7] = np.inf
    with pytest.raises(SaError) as e:
        g.resetup(bad)
    assert e.value.code == -1
    with pytest.raises(SaError):
        g.solve(pb.random_rhs(p.n, 1))
    g.resetup(p.val)
    assert g.solve(pb.random_rhs(p.n, 1))[3] == "SA_OK"


def test_resetup_full_size_fd7_128():
    """128^3 z-stretched cube: re-setup with new values equals the oracle's re-setup on every
    level, and takes less time than the setup (no strength test, no root selection)."""
    import torch
    from oracle import oracle as orc
    from paper_2103_10476_amd import solver
    p = pb.workload("fd7_128_a1000")
    g = solver.Hierarchy.from_problem(p, options=solver.Options())
    t_setup = g.info()["setup_seconds"]
    val2 = _dad(p, 5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.resetup(val2)
    torch.cuda.synchronize()
    t_re = time.perf_counter() - t0
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val)
    h.resetup(val2)
    compare_setup(g, h)
    compare_solve(g, h, pb.random_rhs(p.n, 2))
    # the second re-setup takes the Galerkin values through the plans the first one built
    val3 = _dad(p, 6)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.resetup(val3)
    torch.cuda.synchronize()
    t_re2 = time.perf_counter() - t0
    h.resetup(val3)
    compare_setup(g, h)
    compare_solve(g, h, pb.random_rhs(p.n, 3))
    log(f"[resetup] 128^3: setup {t_setup * 1e3:.1f} ms (first, cold), re-setup "
        f"{t_re * 1e3:.1f} ms (builds the plans), next re-setup {t_re2 * 1e3:.1f} ms")


PARTS = ("A_val", "P_val", "R_val", "Abar_val", "invD", "sm_invD", "coarse_inv")


@pytest.mark.parametrize("name,make,kw", CASES[1:3], ids=[c[0] for c in CASES[1:3]])
def test_planned_resetups_equal_full_ones(name, make, kw, monkeypatch):
    """Four re-setups in a row with the Galerkin plans (built by the first, used by the
    others) against the same four with the full products (SAAMG_RESETUP_PLAN=0): every level
    array bit for bit."""
    from paper_2103_10476_amd import solver
    p = make()
    vals = [_dad(p, 11), 2.0 * p.val, _dad(p, 12), _dad(p, 13)]
    out = {}
    for mode in ("plans", "full"):
        if mode == "full":
            monkeypatch.setenv("SAAMG_RESETUP_PLAN", "0")
        else:
            monkeypatch.delenv("SAAMG_RESETUP_PLAN", raising=False)
        g = solver.Hierarchy.from_problem(p, options=solver.Options(**kw))
        nl = g.info()["levels"]
        out[mode] = []
        for v in vals:
            g.resetup(v)
            out[mode].append([[g.export(l, part) for part in PARTS] for l in range(nl)])
        g.close()
    for k in range(len(vals)):
        for l, (a_l, b_l) in enumerate(zip(out["plans"][k], out["full"][k])):
            for part, a, b in zip(PARTS, a_l, b_l):
                a, b = np.asarray(a), np.asarray(b)
                assert a.shape == b.shape, (k, l, part)
                assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), (k, l, part)
