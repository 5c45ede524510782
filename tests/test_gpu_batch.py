"""Grouped solve (sa_solve_many) through the C ABI: many hierarchies advanced in lockstep by
grouped launches must give, for every system, exactly what sa_solve gives for it alone (x bit
for bit, iteration count, residual, status), whatever else is in the group: other sizes and
depths, FP32 or FP64 V-cycles, Chebyshev or Jacobi of several degrees, FR or PR beta,
systems that stop early, a zero right-hand side, a single-level hierarchy, iteration caps."""
import numpy as np
import pytest

from paper_2103_10476_amd import problems as pb

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def log(msg):
    print(msg, flush=True)


def _cases():
    from paper_2103_10476_amd import solver as S
    O = S.Options
    return [
        ("fd7 20^3 fp64", pb.fd7_stretched(20, 1000.0), O(rtol=1e-10)),
        ("fd7 24^3 fp32", pb.fd7_stretched(24, 100.0), O(rtol=1e-10, precision="fp32")),
        ("q1 13^3 offlmp+1norm fp32", pb.q1_random_kappa(14, seed=5),
         O(rtol=1e-10, variants=("offlmp", "1norm"), cheb_boost=1.1, precision="fp32")),
        ("fd5 64x64 jacobi3", pb.workload("fd5_64x64_a100"),
         O(rtol=1e-8, smoother="jacobi", degree=3)),
        ("fd7 16^3 cheb3 pr", pb.fd7_stretched(16, 10.0), O(rtol=1e-9, degree=3, pcg_beta="pr")),
        ("fd7 12^3 cheb1", pb.fd7_stretched(12, 1000.0), O(rtol=1e-8, degree=1)),
        ("fd7 9^3 single level", pb.fd7_stretched(9, 10.0), O(rtol=1e-10, max_coarse=1000)),
        ("fd7 18^3 cap 3", pb.fd7_stretched(18, 1000.0), O(rtol=1e-14, max_iter=3)),
        ("fd7 10^3 cap 0", pb.fd7_stretched(10, 100.0), O(rtol=1e-8, max_iter=0)),
        ("fd7 22^3 sprsfy+cnstrnt", pb.fd7_stretched(22, 1000.0),
         O(rtol=1e-10, variants=("sprsfy", "cnstrnt"), max_coarse=100)),
    ]


def test_grouped_equals_alone():
    from paper_2103_10476_amd import solver
    cases = _cases()
    hs, bs = [], []
    for k, (name, p, o) in enumerate(cases):
        hs.append(solver.Hierarchy.from_problem(p, options=o))
        b = pb.random_rhs(p.n, 40 + k)
        if name.startswith("fd7 12^3"):
            b = np.zeros(p.n)  # zero right-hand side: x = 0 after no iteration
        bs.append(b)
    alone = [h.solve(b) for h, b in zip(hs, bs)]
    alone = [(x.cpu().numpy(), it, rr, st) for x, it, rr, st in alone]
    grouped = solver.solve_many(hs, bs)
    for (name, p, o), (xa, ia, ra, sa), (xg, ig, rg, sg) in zip(cases, alone, grouped):
        xg = xg.cpu().numpy()
        log(f"[batch] {name}: levels {hs[cases.index((name, p, o))].info()['levels']}, "
            f"alone {ia} its {sa}, grouped {ig} its {sg}")
        assert sg == sa and ig == ia and rg == ra, (name, (ia, ra, sa), (ig, rg, sg))
        assert np.array_equal(xa.view(np.uint64), xg.view(np.uint64)), name
    assert grouped[7][3] == "SA_NOT_CONVERGED" and grouped[7][1] == 3
    assert grouped[8][3] == "SA_NOT_CONVERGED" and grouped[8][1] == 0
    assert grouped[5][1] == 0 and grouped[5][3] == "SA_OK"
    for h in hs:
        h.close()


def test_grouped_repeated_and_reordered():
    """The same systems in another order, twice: identical results each time."""
    from paper_2103_10476_amd import solver
    cases = _cases()[:6]
    hs = [solver.Hierarchy.from_problem(p, options=o) for _, p, o in cases]
    bs = [pb.random_rhs(p.n, 60 + k) for k, (_, p, _) in enumerate(cases)]
    first = solver.solve_many(hs, bs)
    order = list(reversed(range(len(hs))))
    second = solver.solve_many([hs[i] for i in order], [bs[i] for i in order])
    for j, i in enumerate(order):
        x1, i1, r1, s1 = first[i]
        x2, i2, r2, s2 = second[j]
        assert (i1, r1, s1) == (i2, r2, s2)
        assert np.array_equal(x1.cpu().numpy().view(np.uint64), x2.cpu().numpy().view(np.uint64))
    for h in hs:
        h.close()


def test_grouped_full_size_fd7_128():
    """The 128^3 benchmark system next to two small ones: still bitwise sa_solve's result."""
    from paper_2103_10476_amd import solver
    big = pb.workload("fd7_128_a1000")
    small = [pb.fd7_stretched(17, 1000.0), pb.q1_random_kappa(12, seed=8)]
    opts = [solver.Options(rtol=1e-8), solver.Options(rtol=1e-8),
            solver.Options(rtol=1e-8, variants=("offlmp", "1norm"))]
    probs = [big] + small
    hs = [solver.Hierarchy.from_problem(p, options=o) for p, o in zip(probs, opts)]
    bs = [pb.random_rhs(p.n, 2 + k) for k, p in enumerate(probs)]
    alone = [h.solve(b) for h, b in zip(hs, bs)]
    grouped = solver.solve_many(hs, bs)
    for (xa, ia, ra, sa), (xg, ig, rg, sg) in zip(alone, grouped):
        assert (ia, ra, sa) == (ig, rg, sg)
        assert bool((xa == xg).all())
    log(f"[batch] 128^3 next to two small systems: {grouped[0][1]} its, bitwise equal")
    for h in hs:
        h.close()
