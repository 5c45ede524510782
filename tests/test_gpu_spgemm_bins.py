"""GPU parity of the Galerkin product's wavefront-per-row bins (eq. Galerkin, Sec. 1.1): both
widths of their sort keys, and both ways of redoing the rows that overflow the hash bin.

Rows of more than 64 products are taken by one wavefront each; a step's 64 products are
sorted across the lanes by (column << 6 | lane).  The keys are 32 bits wide while the columns
stay below 2^26 (every workload here) and 64 bits wide otherwise; SAAMG_SPGEMM_KEY64=1 takes
the 64-bit keys at any width.  Rows of more than 1024 products whose output is wider than the
LDS go to a 2048-slot hash table; those with more than 1024 distinct columns are redone over
their column windows in LDS tiles, or with SAAMG_SPGEMM_MAX_TILES=0 with a dense accumulator
in global memory.  Each mode is compared with the oracle (every setup array bitwise, the
solve to the usual tolerance).

The 400 x 400 hub matrix (a five-point Laplacian with ten far-coupled hubs of 64 to 9000
entries) sends its level-0 hub rows, with more than 1024 products over 27,418 coarse columns
(wider than any LDS window), to the hash kernel, and the hubs with more than 1024 distinct
columns on to the tiles (two of them) or the dense accumulator; its coarser levels and the
24^3 stretched cube use the LDS window kernel and the 512-slot hash kernel.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_2103_10476_amd import problems as pb
from parity import compare_setup, compare_solve, log, run_both
from test_gpu_long_rows import hub_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()


CASES = {
    "hubs 400x400": (lambda: hub_problem(400, 400)[0], dict(theta=0.02, rtol=1e-10,
                                                            max_coarse=200)),
    "fd7 24 a1000": (lambda: pb.fd7_stretched(24, 1000.0), dict(theta=0.02, max_coarse=50)),
}


def _products(lv):
    """Per-row product counts and output row lengths of A P on one oracle level, and the width
    of P."""
    A = sp.csr_matrix((lv.A[2], lv.A[1], lv.A[0]), shape=(lv.n, lv.n))
    P = sp.csr_matrix((lv.P[2], lv.P[1], lv.P[0]), shape=(lv.n, lv.nc))
    ylen = np.diff(P.indptr)
    t = np.zeros(lv.n, dtype=np.int64)
    rows = np.repeat(np.arange(lv.n), np.diff(A.indptr))
    np.add.at(t, rows, ylen[A.indices])
    return t, np.diff((A @ P).tocsr().indptr), lv.nc


MODES = {  # environment for each mode (None: unset)
    "keys 32, tiles": {"SAAMG_SPGEMM_KEY64": None, "SAAMG_SPGEMM_MAX_TILES": None},
    "keys 64": {"SAAMG_SPGEMM_KEY64": "1", "SAAMG_SPGEMM_MAX_TILES": None},
    "dense overflow": {"SAAMG_SPGEMM_KEY64": None, "SAAMG_SPGEMM_MAX_TILES": "0"},
}


@pytest.mark.parametrize("mode", list(MODES))
@pytest.mark.parametrize("name", list(CASES))
def test_wave_bins_match_oracle(name, mode, monkeypatch):
    make, opts = CASES[name]
    p = make()
    for var, v in MODES[mode].items():
        if v is None:
            monkeypatch.delenv(var, raising=False)
        else:
            monkeypatch.setenv(var, v)
    g, h = run_both(p, **opts)
    if name.startswith("hubs"):
        t, d, width = _products(h.levels[0])
        # level 0's A P reaches the hash kernel (rows over 1024 products, wider than 19,661
        # columns: 160 KB of LDS at 8 bytes and a bit per column), and some overflow it
        assert width > 19661 and int(np.sum(t > 1024)) >= 4, (width, int(np.sum(t > 1024)))
        assert int(np.sum((t > 1024) & (d > 1024))) >= 4
    log(f"[spgemm bins] {name} {mode}: levels {g.info()['levels']}")
    compare_setup(g, h)
    compare_solve(g, h, pb.random_rhs(p.n, 11))
    g.close()
