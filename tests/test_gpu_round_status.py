"""GPU parity of the root selection's ways of running rounds.

On the grid, rounds are launched back to back and the host learns where the selection ends
from status words that the first pass of each round writes into pinned host memory; when a
word does not arrive in time, the host synchronises and reads the device flags instead
(SAAMG_STATUS_SPIN_NS=0 takes that fallback at every wait).  Levels up to
SAAMG_MIS_WG_MAX_N vertices run every round after the first in one workgroup instead, and
grid levels from SAAMG_MIS_V_MIN_N vertices on give each thread 4 vertices.  All four are
compared with the oracle (aggregates, roots and every setup array bitwise) and with each
other (rounds per level), on the 64 x 64 stretched 5-point grid, a 24^3 stretched
7-point cube, a 14^3 random-coefficient 27-point cube and, in hashed order, a 20^3 cube.
"""
import os

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
    torch.cuda.init()


CASES = [
    (lambda: pb.workload("fd5_64x64_a100"), dict(theta=0.02)),
    (lambda: pb.fd7_stretched(24, 1000.0), dict(theta=0.02, max_coarse=50)),
    (lambda: pb.q1_random_kappa(14, seed=3), dict(theta=0.02, variants=["offlmp", "1norm"],
                                                  max_coarse=40)),
    (lambda: pb.fd7_stretched(20, 1000.0), dict(theta=0.02, max_coarse=50, agg_order="hashed",
                                                seed=31)),
]

ENV = ("SAAMG_MIS_WG_MAX_N", "SAAMG_STATUS_SPIN_NS", "SAAMG_MIS_V_MIN_N")
MODES = {  # values for ENV (None: unset)
    "grid, status ring": ("0", None, None),
    "grid, device flags": ("0", "0", None),
    "one workgroup": ("1073741824", None, None),
    "grid, 4 vertices per thread": ("0", None, "0"),
}


@pytest.mark.parametrize("case", range(len(CASES)))
def test_round_paths_agree(case, monkeypatch):
    make, opts = CASES[case]
    p = make()
    rounds = {}
    for mode, values in MODES.items():
        for var, v in zip(ENV, values):
            if v is None:
                monkeypatch.delenv(var, raising=False)
            else:
                monkeypatch.setenv(var, v)
        g, h = run_both(p, **opts)
        compare_setup(g, h)
        rounds[mode] = list(g.info()["mis_rounds"])
        log(f"[rounds] {mode}: {rounds[mode]}")
        g.close()
    first = rounds["grid, status ring"]
    assert all(r == first for r in rounds.values()), rounds
    if opts.get("agg_order") != "hashed":  # hashed order needs few rounds
        assert max(first) > 6  # more rounds than the launch-ahead window
