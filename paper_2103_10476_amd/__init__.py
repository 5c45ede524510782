"""MI355X-native smoothed-aggregation AMG with the prolongator adaptations of Hu, Siefert and
Tuminaro (arXiv 2103.10476): setup and CG + V-cycle solve behind a C ABI (include/saamg.h).

    from paper_2103_10476_amd import setup, Options, problems
    h = setup(problems.workload("fd7_128_a1000"), options=Options(variants=["1norm"]))
    x, iterations = h.solve(b)[:2]
"""
from . import problems  # noqa: F401  (pure numpy, no GPU)

__all__ = ["Options", "Hierarchy", "setup", "solve", "problems"]


def __getattr__(name):
    if name in ("Options", "Hierarchy", "setup", "solve"):
        from . import solver
        return getattr(solver, name)
    raise AttributeError(name)
