"""GPU parity of the Galerkin product's wavefront-per-row bins (eq. Galerkin, Sec. 1.1) with
both widths of their sort keys.

Rows of more than 64 products are taken by one wavefront each; a step's 64 products are
sorted across the lanes by (column << 6 | lane).  The keys are 32 bits wide while the columns
stay below 2^26 (every workload here) and 64 bits wide otherwise; SAAMG_SPGEMM_KEY64=1 takes
the 64-bit keys at any width, so both are compared with the oracle (every setup array
bitwise, the solve to the usual tolerance).

The 400 x 400 hub matrix (a five-point Laplacian with ten far-coupled hubs of 64 to 9000
entries) sends its level-0 hub rows, with more than 1024 products over 27,418 coarse columns
(wider than any LDS window), to the 2048-slot hash kernel, and the hubs with more than 1024
distinct columns on to the dense global accumulator; its coarser levels and the 24^3
stretched cube use the LDS window kernel and the 512-slot hash kernel.
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
    """Per-row product counts of A P on one oracle level, and the width of P."""
    A = sp.csr_matrix((lv.A[2], lv.A[1], lv.A[0]), shape=(lv.n, lv.n))
    ylen = np.diff(lv.P[0])
    t = np.zeros(lv.n, dtype=np.int64)
    rows = np.repeat(np.arange(lv.n), np.diff(A.indptr))
    np.add.at(t, rows, ylen[A.indices])
    return t, lv.nc


@pytest.mark.parametrize("key64", [False, True], ids=["keys 32", "keys 64"])
@pytest.mark.parametrize("name", list(CASES))
def test_wave_bins_match_oracle(name, key64, monkeypatch):
    make, opts = CASES[name]
    p = make()
    if key64:
        monkeypatch.setenv("SAAMG_SPGEMM_KEY64", "1")
    else:
        monkeypatch.delenv("SAAMG_SPGEMM_KEY64", raising=False)
    g, h = run_both(p, **opts)
    if name.startswith("hubs"):
        t, width = _products(h.levels[0])
        # level 0's A P reaches the hash kernel: rows over 1024 products, wider than 19,661
        # columns (160 KB of LDS at 8 bytes and a bit per column)
        assert width > 19661 and int(np.sum(t > 1024)) >= 4, (width, int(np.sum(t > 1024)))
    log(f"[spgemm bins] {name} key64={key64}: levels {g.info()['levels']}")
    compare_setup(g, h)
    compare_solve(g, h, pb.random_rhs(p.n, 11))
    g.close()
