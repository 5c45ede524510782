"""Serving through the C ABI (sa_server_*): requests of the serving workload's two families
(7-point z-stretched cubes, 27-point random-kappa cubes) run concurrently on one GPU under an
HBM budget.  Each request must come back bitwise equal to the same setup + solve run alone,
match the CPU oracle, stay within its admission estimate, and fail on its own without
disturbing the others."""
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


def _requests(count, smin, smax, seed=11):
    """Small-side members of the serving workload with the serving method (OffLmp + 1Norm),
    plus other settings in rotation so that the mix holds several code paths."""
    from paper_2103_10476_amd import solver
    extra = [{"precision": "fp32"}, {}, {"variants": ("sprsfy", "cnstrnt"), "max_coarse": 200},
             {"smoother": "jacobi", "rtol": 1e-8}]
    out = []
    for i, req in enumerate(pb.serving_requests(count, seed=seed, smin=smin, smax=smax)):
        p, b = pb.build_request(req)
        kw = dict(pb.serving_method(req))
        kw.update(extra[i % len(extra)])
        kw["variants"] = tuple(sorted(set(kw.get("variants", ())) | {"offlmp", "1norm"}))
        out.append((req, p, b, solver.Options(**kw)))
    return out


def _alone(p, b, o):
    from paper_2103_10476_amd import solver
    h = solver.Hierarchy.from_problem(p, options=o)
    x, it, rr, st = h.solve(b)
    xh = x.cpu().numpy()
    h.close()
    return xh, it, rr, st


def _serve(reqs, budget, slots, borrow=False):
    from paper_2103_10476_amd import solver
    srv = solver.Server(hbm_budget=budget, max_slots=slots)
    tickets = [srv.submit(p, b, o, borrow=borrow) for (_, p, b, o) in reqs]
    out = [srv.wait(t, p.n) for t, (_, p, _, _) in zip(tickets, reqs)]
    st = srv.stats()
    srv.close()
    return out, st


def test_mix_is_bitwise_equal_to_alone():
    reqs = _requests(12, 10, 26)
    log(f"[serving] {len(reqs)} requests, n = {[p.n for _, p, _, _ in reqs]}")
    served, st = _serve(reqs, budget=8 << 30, slots=4)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    for (req, p, b, o), (x, r) in zip(reqs, served):
        xa, it, rr, sta = _alone(p, b, o)
        assert r["status"] == sta, (req, r["status"], sta)
        assert r["iterations"] == it and r["rel_residual"] == rr, (req, r, it, rr)
        assert np.array_equal(x.view(np.uint64), xa.view(np.uint64)), req
        assert 0 < r["peak_bytes"] <= r["reserved_bytes"], r
        assert r["latency_seconds"] >= r["setup_seconds"] + r["solve_seconds"]
    assert st["peak_reserved_bytes"] <= st["budget_bytes"]


def test_borrowed_inputs_match_copied_ones():
    """sa_server_submit_borrowed reads the caller's arrays instead of copies: same bits."""
    reqs = _requests(8, 10, 24, seed=23)
    copied, _ = _serve(reqs, budget=8 << 30, slots=3)
    borrowed, st = _serve(reqs, budget=8 << 30, slots=3, borrow=True)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    for req, (xc, rc), (xb, rb) in zip(reqs, copied, borrowed):
        assert rb["status"] == rc["status"] and rb["iterations"] == rc["iterations"], req
        assert rb["rel_residual"] == rc["rel_residual"], req
        assert np.array_equal(xb.view(np.uint64), xc.view(np.uint64)), req


def test_borrowed_device_inputs_match_copied_ones():
    """sa_server_submit_borrowed with A and b in device memory (A->loc = SA_DEVICE), called
    through the C ABI: the setup copies the matrix device to device and the solve reads b
    there; results equal those of host inputs copied at submission, bit for bit."""
    import ctypes as C
    import torch
    from paper_2103_10476_amd import _lib, solver
    reqs = _requests(6, 10, 22, seed=29)
    copied, _ = _serve(reqs, budget=8 << 30, slots=3)
    types = (np.int32, np.int32, np.float64, np.float64)
    held = [[torch.from_numpy(np.ascontiguousarray(a, dtype=t)).cuda()
             for a, t in zip((p.rp, p.col, p.val, b), types)] for _, p, b, _ in reqs]
    torch.cuda.synchronize()  # the server's streams read them
    srv = solver.Server(hbm_budget=8 << 30, max_slots=3)
    tickets = []
    for (_, p, b, o), d in zip(reqs, held):
        csr = _lib.SaCsr(int(p.n), int(p.nnz), d[0].data_ptr(), d[1].data_ptr(),
                         d[2].data_ptr(), _lib.SA_DEVICE)
        opts = o.to_c()
        t = C.c_uint64()
        _lib.check(_lib.lib().sa_server_submit_borrowed(srv._s, C.byref(csr),
                                                        C.c_void_p(d[3].data_ptr()),
                                                        C.byref(opts), C.byref(t)),
                   "sa_server_submit_borrowed")
        tickets.append(t.value)
    served = [srv.wait(t, p.n) for t, (_, p, _, _) in zip(tickets, reqs)]
    srv.close()
    del held
    for req, (xc, rc), (xb, rb) in zip(reqs, copied, served):
        assert rb["status"] == rc["status"] and rb["iterations"] == rc["iterations"], req
        assert rb["rel_residual"] == rc["rel_residual"], req
        assert np.array_equal(xb.view(np.uint64), xc.view(np.uint64)), req


def test_served_requests_match_oracle():
    """Small requests of both families, plus one of each family with side >= 64."""
    from oracle import oracle as orc
    from paper_2103_10476_amd import solver
    reqs = []
    large = pb.serving_requests(12, seed=15, smin=64, smax=72)
    pick = [next(r for r in large if r["kind"] == k) for k in ("fd7", "q1")]
    both = [(req, *pb.build_request(req), None) for req in pick]
    for (req, p, b, _) in _requests(6, 10, 18, seed=12) + both:
        kw = dict(pb.serving_method(req), precision="fp64")  # the oracle computes in FP64
        reqs.append((req, p, b, solver.Options(**kw)))
    served, _ = _serve(reqs, budget=8 << 30, slots=3)
    for (req, p, b, o), (x, r) in zip(reqs, served):
        m = pb.serving_method(req)
        h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, theta=0.02, rtol=m["rtol"],
                                variants=m["variants"], cheb_boost=m["cheb_boost"])
        ref = h.solve(b)
        err = np.linalg.norm(x - ref["x"]) / np.linalg.norm(ref["x"])
        log(f"[serving] {req['kind']} s={req['side']} its {r['iterations']} "
            f"oracle {ref['iterations']} err {err:.1e}")
        assert r["iterations"] == ref["iterations"]
        assert err <= 1e-12


def test_tight_budget_serialises_and_matches():
    """A budget of 1.5 times the largest request's estimate admits one large request at a
    time; results equal the roomy run's bit for bit."""
    from paper_2103_10476_amd import solver
    reqs = _requests(8, 10, 24, seed=13)
    biggest = max(solver.estimate_bytes(p.n, p.nnz) for _, p, _, _ in reqs)
    roomy, _ = _serve(reqs, budget=8 << 30, slots=4)
    tight, st = _serve(reqs, budget=int(1.5 * biggest), slots=4)
    assert st["peak_reserved_bytes"] <= int(1.5 * biggest)
    assert st["completed"] == len(reqs)
    for (x1, r1), (x2, r2) in zip(roomy, tight):
        assert np.array_equal(x1.view(np.uint64), x2.view(np.uint64))
        assert r1["iterations"] == r2["iterations"]


def test_largest_requests_fit_their_estimate():
    """The largest members of both families (side 96: 884,736 unknowns; the 27-point one
    has 23.4M entries) hold at most their admission estimate of device memory."""
    from paper_2103_10476_amd import solver
    reqs = []
    for kind, seed in (("fd7", 21), ("q1", 22)):
        req = {"id": 0, "kind": kind, "side": 96, "aspect": 1000.0, "seed": seed}
        p, b = pb.build_request(req)
        reqs.append((req, p, b, solver.Options(**pb.serving_method(req))))
    served, st = _serve(reqs, budget=64 << 30, slots=2)
    for (req, p, _, _), (x, r) in zip(reqs, served):
        log(f"[serving] {req['kind']} n={p.n} nnz={p.nnz}: peak {r['peak_bytes'] / 2**20:.0f} "
            f"MiB, estimate {r['reserved_bytes'] / 2**20:.0f} MiB, {r['iterations']} its, "
            f"{r['status']}")
        assert r["status"] == "SA_OK"
        assert r["peak_bytes"] <= r["reserved_bytes"]


def test_failure_is_isolated_and_oversize_rejected():
    from paper_2103_10476_amd import solver
    from paper_2103_10476_amd._lib import SaError
    good = pb.fd7_stretched(12, 100.0)
    bad = pb.fd7_stretched(8, 10.0)
    b_good = pb.random_rhs(good.n, 3)
    b_bad = pb.random_rhs(bad.n, 4)
    srv = solver.Server(hbm_budget=4 << 30, max_slots=2)
    o = solver.Options(max_coarse=20)
    t1 = srv.submit(good, b_good, o)
    t2 = srv.submit((bad.n, bad.rp, bad.col, -bad.val), b_bad, o)  # negative definite
    t3 = srv.submit(good, b_good, o)
    x1, r1 = srv.wait(t1, good.n)
    with pytest.raises(SaError) as e:
        srv.wait(t2, bad.n)
    assert e.value.code in (-3, -4)
    x3, r3 = srv.wait(t3, good.n)
    assert np.array_equal(x1, x3) and r1["status"] == "SA_OK"
    with pytest.raises(SaError):  # ticket already collected
        srv.poll(t1, good.n)
    st = srv.stats()
    assert st["completed"] == 2 and st["failed"] == 1
    srv.close()
    small = solver.Server(hbm_budget=1 << 20, max_slots=1)
    with pytest.raises(SaError) as e:
        small.submit(good, b_good)
    assert e.value.code == -7  # SA_ERR_OOM: larger than the whole budget
    small.close()
