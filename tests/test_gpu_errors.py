"""GPU error paths through the C ABI: malformed input is rejected by host checks and by the
validation kernel's bounds-checked reads (no kernel indexes with unvalidated data)."""
import numpy as np
import pytest

from paper_2103_10476_amd import problems as pb

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _setup(p_tuple, **kw):
    from paper_2103_10476_amd import solver
    n, rp, col, val = p_tuple
    return solver.Hierarchy(n, rp, col, val, options=solver.Options(**kw))


def _code(fn):
    from paper_2103_10476_amd._lib import SaError
    with pytest.raises(SaError) as e:
        fn()
    return e.value.code


def test_bad_csr_rejected():
    p = pb.fd5_stretched(8, 8, 10.0)
    base = (p.n, p.rp.copy(), p.col.copy(), p.val.copy())
    # unsorted columns in row 5
    n, rp, col, val = (x.copy() if hasattr(x, "copy") else x for x in base)
    a, b = rp[5], rp[5] + 1
    col[a], col[b] = col[b], col[a]
    assert _code(lambda: _setup((n, rp, col, val))) == -2
    # out-of-range column
    n, rp, col, val = (x.copy() if hasattr(x, "copy") else x for x in base)
    col[7] = p.n + 3
    assert _code(lambda: _setup((n, rp, col, val))) == -2
    # missing diagonal: drop row 0's diagonal entry
    d = p.to_dense()
    d[0, 0] = 0.0
    q = pb.from_dense(d)
    keep = ~((np.repeat(np.arange(q.n), np.diff(q.rp)) == 0) & (q.col == 0))
    rows = np.repeat(np.arange(q.n), np.diff(q.rp))[keep]
    rp2 = np.zeros(q.n + 1, np.int32)
    rp2[1:] = np.cumsum(np.bincount(rows, minlength=q.n))
    assert _code(lambda: _setup((q.n, rp2, q.col[keep], q.val[keep]))) == -2
    # row pointers that do not span nnz
    n, rp, col, val = (x.copy() if hasattr(x, "copy") else x for x in base)
    rp[-1] -= 1
    assert _code(lambda: _setup((n, rp, col[:-1], val[:-1]))) in (-2,)
    # row pointers not starting at 0, or ending short of the arrays' length
    n, rp, col, val = (x.copy() if hasattr(x, "copy") else x for x in base)
    rp[0] = 1
    assert _code(lambda: _setup((n, rp, col, val))) == -2
    n, rp, col, val = (x.copy() if hasattr(x, "copy") else x for x in base)
    assert _code(lambda: _setup((n, rp, np.append(col, 0).astype(np.int32),
                                 np.append(val, 1.0)))) == -2
    # a decreasing row pointer inside the matrix
    n, rp, col, val = (x.copy() if hasattr(x, "copy") else x for x in base)
    rp[6] = rp[5] - 1
    assert _code(lambda: _setup((n, rp, col, val))) == -2
    # non-finite value
    n, rp, col, val = (x.copy() if hasattr(x, "copy") else x for x in base)
    val[3] = np.nan
    assert _code(lambda: _setup((n, rp, col, val))) == -1


def test_bad_options_rejected():
    p = pb.fd5_stretched(8, 8, 10.0)
    assert _code(lambda: _setup((p.n, p.rp, p.col, p.val), theta=1.5)) == -1
    assert _code(lambda: _setup((p.n, p.rp, p.col, p.val), degree=0)) == -1


def test_zero_rhs_and_iteration_cap():
    from paper_2103_10476_amd import solver
    p = pb.fd7_stretched(12, 100.0)
    h = solver.Hierarchy.from_problem(p, options=solver.Options(max_coarse=20, max_iter=2,
                                                                 rtol=1e-14))
    x, it, rr, st = h.solve(np.zeros(p.n))
    assert it == 0 and st == "SA_OK" and float(x.abs().max()) == 0.0
    x, it, rr, st = h.solve(pb.random_rhs(p.n, 1))
    assert st == "SA_NOT_CONVERGED" and it == 2


def test_indefinite_matrix_breaks_down():
    """A negative-definite matrix: smoother diagonal check fails at setup."""
    p = pb.fd7_stretched(8, 10.0)
    assert _code(lambda: _setup((p.n, p.rp, p.col, -p.val), max_coarse=20)) in (-3, -4)


def test_nullspace_with_zero_rejected():
    from paper_2103_10476_amd import solver
    p = pb.fd5_stretched(8, 8, 10.0)
    B = np.ones(p.n)
    B[3] = 0.0
    assert _code(lambda: solver.Hierarchy.from_problem(p, nullspace=B)) == -1
