"""GPU parity of the root selection's end detection.

Rounds are launched back to back and the host learns where the selection ends from status
words that the first pass of each round writes into pinned host memory; when a word does not
arrive in time, the host synchronises and reads the device flags instead.  With
SAAMG_STATUS_SPIN_NS=0 the fallback is taken at every wait, so both ways of finding the end
are compared with the oracle (aggregates, roots and every setup array bitwise) and with each
other (rounds per level), on the 64 x 64 stretched 5-point grid, a 24^3 stretched 7-point cube
and a 14^3 random-coefficient 27-point cube.
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
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_status_ring_and_fallback_agree(case, monkeypatch):
    make, opts = CASES[case]
    p = make()
    rounds = {}
    for spin in (None, "0"):
        if spin is None:
            monkeypatch.delenv("SAAMG_STATUS_SPIN_NS", raising=False)
        else:
            monkeypatch.setenv("SAAMG_STATUS_SPIN_NS", spin)
        g, h = run_both(p, **opts)
        compare_setup(g, h)
        rounds[spin] = list(g.info()["mis_rounds"])
        log(f"[status] spin {spin}: rounds {rounds[spin]}")
        g.close()
    assert rounds[None] == rounds["0"]
    assert max(rounds[None]) > 6  # more rounds than the launch-ahead window
