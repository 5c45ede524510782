"""Pins of the oracle's Galerkin product, smoother, V-cycle, coarse solve, PCG and the
inner-product convention.

Sources: Sec. 1.1 (Galerkin coarse operator; Algorithm 1 V-cycle), Sec. 2.5 (coarse fill-in
pattern), Sec. 3.1 (Chebyshev degree 2 on [lambda/10, lambda]; direct coarse solve; CG).
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_2103_10476_amd import problems as pb


def rows_of(rp):
    return np.repeat(np.arange(len(rp) - 1), np.diff(rp))


def dense(csr, n, m=None):
    rp, col, val = csr
    d = np.zeros((n, n if m is None else m))
    d[rows_of(rp), col] = val
    return d


@pytest.mark.parametrize("name,var", [("fd5_16x16_a100", []), ("fd7_8_a1000", ["sprsfy"]),
                                      ("fd7_8_a1000", ["cnstrnt", "offlmp", "1norm"])])
def test_galerkin_dense_brute_force(orc, name, var):
    """A_{l+1} = P^T A_l P (Sec. 1.1): dense product, symbolic pattern, symmetry."""
    p = pb.workload(name)
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, theta=0.02, max_coarse=20, variants=var)
    assert len(h.levels) >= 2
    for l in range(len(h.levels) - 1):
        L, Lc = h.levels[l], h.levels[l + 1]
        A = dense(L.A, L.n)
        P = dense(L.P, L.n, L.nc)
        R = dense(L.R, L.nc, L.n)
        assert np.array_equal(R, P.T)
        Ac = dense(Lc.A, Lc.n)
        ref = P.T @ A @ P
        assert np.abs(Ac - ref).max() <= 1e-13 * np.abs(ref).max()
        # stored pattern = boolean product pattern (cancellations stay stored)
        pat = ((P != 0).T.astype(int) @ (A != 0).astype(int) @ (P != 0).astype(int)) > 0
        patL = np.zeros_like(pat)
        patL[rows_of(Lc.A[0]), Lc.A[1]] = True
        Ppat = np.zeros((L.n, L.nc), bool)
        Ppat[rows_of(L.P[0]), L.P[1]] = True
        Apat = np.zeros((L.n, L.n), bool)
        Apat[rows_of(L.A[0]), L.A[1]] = True
        sym = (Ppat.T.astype(int) @ Apat.astype(int) @ Ppat.astype(int)) > 0
        assert np.array_equal(patL, sym) and np.array_equal(sym, sym.T)
        assert np.abs(Ac - Ac.T).max() <= 1e-14 * np.abs(Ac).max()


def test_galerkin_preserves_null_space(orc):
    """A 1 = 0 and P 1 = 1 (constant in range(P)) give A_c 1_c = 0 (Sec. 1.1)."""
    p = pb.periodic_stencil_2d(9, 9, {(0, 0): 4.0, (1, 0): -1.0, (-1, 0): -1.0,
                                      (0, 1): -1.0, (0, -1): -1.0})
    m = orc.strength(p.n, p.rp, p.col, p.val, 0.0)
    agg, root, nc = orc.aggregate(p.n, p.rp, p.col, m)
    Ab = orc.lump(p.n, p.rp, p.col, p.val, m)
    invD = orc.diag(p.n, *Ab)
    lam = orc.power(p.n, *Ab, invD)
    P = orc.prolongator(p.n, *Ab, invD, agg, 4.0 / (3.0 * lam))
    A = (p.rp, p.col, p.val)
    AP_rows = [orc.spgemm_row(A, P, nc, i) for i in range(p.n)]
    AP = np.zeros((p.n, nc))
    for i, (c, v) in enumerate(AP_rows):
        AP[i, c] = v
    Ac = dense(P, p.n, nc).T @ AP
    assert np.abs(Ac @ np.ones(nc)).max() <= 1e-13 * np.abs(Ac).max()


def test_coarse_fill_distance_three(orc):
    """Sec. 2.5: coarse (i,j) is nonzero iff Ptent_i^T Abar^T A Abar Ptent_j != 0."""
    p = pb.workload("fd5_16x16_a100")
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, theta=0.02, max_levels=2, max_coarse=20)
    L = h.levels[0]
    Pt = np.zeros((L.n, L.nc), int)
    ok = L.agg >= 0
    Pt[np.nonzero(ok)[0], L.agg[ok]] = 1
    Abp = (dense(L.Abar, L.n) != 0).astype(int)
    Ap = (dense(L.A, L.n) != 0).astype(int)
    pat = (Pt.T @ Abp.T @ Ap @ Abp @ Pt) > 0
    Lc = h.levels[1]
    got = np.zeros_like(pat)
    got[rows_of(Lc.A[0]), Lc.A[1]] = True
    assert np.array_equal(got, pat)


def cheb_poly_matrix(A, invD, lam, ratio, deg):
    """Closed form of the degree-`deg` Chebyshev error propagator p(D^{-1}A) with
    p(t) = T_deg((theta - t)/delta) / T_deg(theta/delta) on [lam/ratio, lam]."""
    lo = lam / ratio
    theta, delta = (lam + lo) / 2, (lam - lo) / 2
    M = np.diag(invD) @ A
    X = (theta * np.eye(len(A)) - M) / delta
    T0, T1 = np.eye(len(A)), X
    for _ in range(deg - 1):
        T0, T1 = T1, 2 * X @ T1 - T0
    Tk = T1 if deg >= 1 else T0
    t = theta / delta
    c0, c1 = 1.0, t
    for _ in range(deg - 1):
        c0, c1 = c1, 2 * t * c1 - c0
    return Tk / c1


@pytest.mark.parametrize("smoother", ["chebyshev", "jacobi"])
def test_two_level_error_propagator(orc, smoother):
    """Algorithm 1 with two levels: E = S (I - P A_c^{-1} P^T A) S, S the smoother's error
    propagator in closed form; the oracle's V-cycle reproduces it and converges."""
    p = pb.workload("fd5_12x12_a100")
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, theta=0.02, max_levels=2, max_coarse=5,
                            smoother=smoother)
    L = h.levels[0]
    A = dense(L.A, L.n)
    B = np.column_stack([h.vcycle(e) for e in np.eye(L.n)])
    E = np.eye(L.n) - B @ A
    if smoother == "chebyshev":
        S = cheb_poly_matrix(A, L.sm_invD, L.sm_lam, 10.0, 2)
        # p(lam*) ~ 0.503 and |p| <= 1 on [0, 1.1 lam*] (degree 2, ratio 10)
        ts = np.linspace(0, 1.1 * L.sm_lam, 200)
        lo = L.sm_lam / 10
        th, de = (L.sm_lam + lo) / 2, (L.sm_lam - lo) / 2
        pv = (2 * ((th - ts) / de) ** 2 - 1) / (2 * (th / de) ** 2 - 1)
        assert np.all(np.abs(pv) <= 1 + 1e-12)
    else:
        w = 4.0 / (3.0 * L.sm_lam)
        J = np.eye(L.n) - w * np.diag(L.sm_invD) @ A
        S = J @ J
    P = dense(L.P, L.n, L.nc)
    Ac = P.T @ A @ P
    CG = np.eye(L.n) - P @ np.linalg.solve(Ac, P.T @ A)
    Eref = S @ CG @ S
    assert np.abs(E - Eref).max() <= 1e-10
    # energy-norm contraction
    w_, V = np.linalg.eigh(A)
    Ah = V @ np.diag(np.sqrt(w_)) @ V.T
    rho = np.abs(np.linalg.eigvals(Ah @ E @ np.linalg.inv(Ah))).max()
    assert rho < 0.9
    # symmetric preconditioner (same smoother before and after)
    assert np.abs(B - B.T).max() <= 1e-10 * np.abs(B).max()


def test_single_level_is_direct_solve(orc):
    """n <= max_coarse: the V-cycle is the dense direct solve (Sec. 3.1)."""
    p = pb.workload("fd5_16x16_a100")
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, max_coarse=1000)
    assert len(h.levels) == 1
    f = pb.random_rhs(p.n, 9)
    u = h.vcycle(f)
    ref = np.linalg.solve(p.to_dense(), f)
    assert np.abs(u - ref).max() <= 1e-12 * np.abs(ref).max()


def _dense_pcg(A, M, b, rtol, max_iter):
    x = np.zeros_like(b)
    r = b.copy()
    g0 = r @ r
    z = M @ r
    p = z.copy()
    rho = r @ z
    for k in range(1, max_iter + 1):
        q = A @ p
        a = rho / (p @ q)
        x += a * p
        r -= a * q
        rr = r @ r
        if rr <= rtol * rtol * g0:
            return x, k, rr / (rtol * rtol * g0)
        z = M @ r
        rho1 = r @ z
        p = z + (rho1 / rho) * p
        rho = rho1
    return x, max_iter, None


@pytest.mark.parametrize("name", ["fd5_16x16_a100", "fd7_8_a1000"])
def test_pcg_matches_dense_pcg(orc, name):
    """CG preconditioned by the V-cycle (Sec. 3.1): the same iteration count as dense CG with
    the V-cycle as an explicit matrix, and the true residual meets the tolerance."""
    p = pb.workload(name)
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, theta=0.02, max_coarse=20, rtol=1e-10)
    A = p.to_dense()
    M = np.column_stack([h.vcycle(e) for e in np.eye(p.n)])
    b = pb.random_rhs(p.n, 11)
    x_d, k_d, margin = _dense_pcg(A, M, b, 1e-10, 200)
    r = h.solve(b)
    assert r["converged"]
    if margin is not None and margin < 0.5:
        assert r["iterations"] == k_d
    else:
        assert abs(r["iterations"] - k_d) <= 1
    assert np.linalg.norm(b - A @ r["x"]) / np.linalg.norm(b) <= 1.5e-10
    assert np.linalg.norm(r["x"] - x_d) <= 1e-8 * np.linalg.norm(x_d)


def test_pcg_zero_rhs_and_not_converged(orc):
    p = pb.workload("fd5_16x16_a100")
    h = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, max_coarse=20, max_iter=2, rtol=1e-12)
    r = h.solve(np.zeros(p.n))
    assert r["iterations"] == 0 and np.all(r["x"] == 0)
    r = h.solve(pb.random_rhs(p.n, 1))
    assert not r["converged"] and r["iterations"] == 2


def test_nullspace_scaling_invariance(orc):
    """Reading: a nullspace vector B is handled by the exact scaling D_B A D_B; with B a power
    of two the scaled problem is exact, and the hierarchy equals the unscaled one with
    P_1 = D_B Phat_1."""
    p = pb.workload("fd5_16x16_a100")
    B = np.where(np.arange(p.n) % 3 == 0, 2.0, 0.5)
    h0 = orc.OracleHierarchy(p.n, p.rp, p.col, p.val, max_coarse=20)
    # A' = D_B^{-1} A D_B^{-1} has near-nullspace B; scaling it back gives A exactly
    val = p.val / B[rows_of(p.rp)] / B[p.col]
    h1 = orc.OracleHierarchy(p.n, p.rp, p.col, val, nullspace=B, max_coarse=20)
    assert np.array_equal(h0.levels[0].agg, h1.levels[0].agg)
    P0 = dense(h0.levels[0].P, p.n, h0.levels[0].nc)
    P1 = dense(h1.levels[0].P, p.n, h1.levels[0].nc)
    assert np.array_equal(P1, B[:, None] * P0)
    for l in range(1, len(h0.levels)):
        assert np.array_equal(h0.levels[l].A[2], h1.levels[l].A[2])
    # P_1 reproduces the nullspace on aggregated rows before smoothing: Ptent 1 = B
    ok = h1.levels[0].agg >= 0
    Pt = np.zeros((p.n, h1.levels[0].nc))
    Pt[np.nonzero(ok)[0], h1.levels[0].agg[ok]] = B[ok]
    assert np.array_equal(Pt @ np.ones(h1.levels[0].nc), np.where(ok, B, 0))


# ---- inner products and the generator ---------------------------------------------------

def test_canonical_dot_exact_cases(orc):
    for n in (1, 255, 4096, 4097, 70000):
        x = np.arange(n, dtype=float) % 7 - 3
        y = np.ones(n)
        assert orc.dot(x, y) == float(x.sum())  # integers: every partial sum exact
    assert orc.dot(np.zeros(0), np.zeros(0)) == 0.0


def test_canonical_dot_error_bound(orc):
    """|dot - exact| <= gamma_k sum |x_i y_i| with k = the tree depth (16 + 8 per level)."""
    rng = np.random.default_rng(4)
    for n in (10, 5000, 300000):
        x = rng.normal(size=n) * 10.0 ** rng.uniform(-3, 3, n)
        y = rng.normal(size=n)
        exact = math.fsum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, y)) \
            if n <= 5000 else math.fsum((x * y).tolist())
        exact = float(exact)
        levels = 1 + int(n > 4096) + int(n > 4096**2)
        k = levels * 24 + 1
        u = 2.0**-53
        bound = k * u / (1 - k * u) * np.abs(x * y).sum() + 2 * u * abs(exact)
        assert abs(orc.dot(x, y) - exact) <= bound


def test_splitmix64_published_vector(orc):
    """SplitMix64 started from state 0: the first output is 0xE220A8397B1DCDAF."""
    assert orc.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    u = np.array([orc.splitmix64(7, k) >> 11 for k in range(20000)], dtype=float) * 2.0**-53
    assert abs(u.mean() - 0.5) < 0.01 and u.min() >= 0 and u.max() < 1
