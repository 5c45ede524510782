"""Helpers for GPU-vs-oracle parity tests (imported by the gpu-marked tests only)."""
from __future__ import annotations

import sys
import time

import numpy as np

TOL_X = 1e-12  # relative error of the solution vs the oracle's (FP64)


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_both(p, b=None, nullspace=None, coords=None, block_size=None, **opts):
    """Set up on the GPU and in the oracle with the same inputs (``coords``: node
    coordinates for the distance-Laplacian strength)."""
    from oracle import oracle as orc
    from paper_2103_10476_amd import solver
    log(f"[parity] {p.name} n={p.n} nnz={p.nnz} opts={opts}")
    g_opts = dict(opts)
    pcg = g_opts.pop("pcg_beta", "fr")
    o = solver.Options(**g_opts, pcg_beta=pcg)
    t = time.time()
    g = solver.Hierarchy.from_problem(p, nullspace=nullspace, options=o, coords=coords,
                                      block_size=block_size)
    tg = time.time() - t
    t = time.time()
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, nullspace=nullspace, coords=coords,
                            block_size=block_size, **opts)
    to = time.time() - t
    log(f"[parity]   setup gpu {tg:.3f}s oracle {to:.3f}s levels {len(h.levels)}")
    return g, h


def assert_same(a, b, what):
    a = np.asarray(a)
    b = np.asarray(b)
    assert a.shape == b.shape, f"{what}: shape {a.shape} vs {b.shape}"
    if a.dtype.kind == "f":
        bad = np.nonzero(a != b)[0]
        assert bad.size == 0, (f"{what}: {bad.size} of {a.size} values differ; first at "
                               f"{bad[0]}: {a[bad[0]]!r} vs {b[bad[0]]!r}")
    else:
        bad = np.nonzero(a != b)[0]
        assert bad.size == 0, (f"{what}: {bad.size} of {a.size} differ; first at {bad[0]}: "
                               f"{a[bad[0]]} vs {b[bad[0]]}")


def compare_setup(g, h, check_values=True):
    """Bitwise comparison of every level's arrays and scalars."""
    info = g.info()
    assert info["levels"] == len(h.levels), (info["levels"], len(h.levels))
    for l, L in enumerate(h.levels):
        tag = f"level {l}"
        assert info["n"][l] == L.n and info["nnz"][l] == L.nnz, (tag, info["n"][l], L.n)
        for name, arr in zip(("A_rp", "A_col", "A_val"), L.A):
            assert_same(g.export(l, name), arr, f"{tag} {name}")
        if getattr(h, "dim", 0):
            assert_same(g.export(l, "coords"), L.coords.reshape(-1), f"{tag} coords")
        if getattr(h, "system", False):
            assert_same(g.export(l, "nullspace"), L.B.reshape(-1), f"{tag} nullspace")
        if L.coarsest:
            inv = g.export(l, "coarse_inv").reshape(L.n, L.n)
            A = np.zeros((L.n, L.n))
            A[np.repeat(np.arange(L.n), np.diff(L.A[0])), L.A[1]] = L.A[2]
            ref = np.linalg.inv(A)
            err = np.abs(inv - ref).max() / np.abs(ref).max()
            assert err <= 1e-11 * max(1.0, np.linalg.cond(A) / 1e4), (tag, "coarse inverse", err)
            continue
        assert_same(g.export(l, "mask"), L.mask, f"{tag} mask")
        assert_same(g.export(l, "agg"), L.agg, f"{tag} agg")
        assert_same(g.export(l, "root"), L.is_root, f"{tag} root")
        for name, arr in zip(("Abar_rp", "Abar_col", "Abar_val"), L.Abar):
            assert_same(g.export(l, name), arr, f"{tag} {name}")
        assert_same(g.export(l, "invD"), L.invD, f"{tag} invD")
        for name, arr in zip(("P_rp", "P_col", "P_val"), L.P):
            assert_same(g.export(l, name), arr, f"{tag} {name}")
        for name, arr in zip(("R_rp", "R_col", "R_val"), L.R):
            assert_same(g.export(l, name), arr, f"{tag} {name}")
        assert_same(g.export(l, "sm_invD"), L.sm_invD, f"{tag} sm_invD")
        if getattr(h, "system", False):
            for name, arr in zip(("Pt_rp", "Pt_col", "Pt_val"), L.Pt):
                assert_same(g.export(l, name), arr, f"{tag} {name}")
            assert_same(g.export(l, "node_mask"), L.nmask, f"{tag} node labels")
            assert_same(g.export(l, "node_rp"), L.Gn[0], f"{tag} node graph rp")
            assert_same(g.export(l, "node_col"), L.Gn[1], f"{tag} node graph col")
        assert info["lambda"][l] == L.lam, (tag, "lambda", info["lambda"][l], L.lam)
        assert info["omega"][l] == L.omega, (tag, "omega")
        assert info["smoother_lambda"][l] == L.sm_lam, (tag, "smoother lambda")


def compare_solve(g, h, b, tol=TOL_X):
    x, it, rr, status = g.solve(b)
    ref = h.solve(b)
    xg = x.cpu().numpy()
    err = np.linalg.norm(xg - ref["x"]) / np.linalg.norm(ref["x"])
    log(f"[parity]   iterations gpu {it} oracle {ref['iterations']} rel err {err:.2e} "
        f"relres {rr:.3e}")
    assert it == ref["iterations"], (it, ref["iterations"])
    assert (status == "SA_OK") == ref["converged"]
    assert err <= tol, err
    return it, err
