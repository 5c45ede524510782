"""ctypes front end of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import this module.
It never imports the GPU package, and the GPU package never imports it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

VARIANT_BITS = {"sprsfy": 1, "offlmp": 2, "1norm": 4, "cnstrnt": 8}


class OrcOptions(C.Structure):
    _fields_ = [("theta", C.c_double), ("variants", C.c_int32), ("one_norm_power", C.c_int32),
                ("tau", C.c_double), ("sigma", C.c_double), ("power_iters", C.c_int32),
                ("agg_order", C.c_int32), ("seed", C.c_uint64), ("max_levels", C.c_int32),
                ("max_coarse", C.c_int32), ("smoother", C.c_int32), ("degree", C.c_int32),
                ("cheb_ratio", C.c_double), ("cheb_boost", C.c_double), ("rtol", C.c_double),
                ("max_iter", C.c_int32), ("pcg_beta", C.c_int32), ("dist_power", C.c_int32),
                ("coarse_solver", C.c_int32), ("singletons", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = C.CDLL(LIB_PATH)
        _setup_prototypes(_lib)
    return _lib


def _setup_prototypes(L):
    P = C.c_void_p
    L.orc_default_options.argtypes = [C.POINTER(OrcOptions)]
    L.orc_last_error.restype = C.c_char_p
    L.orc_setup.argtypes = [C.c_int32, P, P, P, P, C.POINTER(OrcOptions), C.POINTER(C.c_void_p)]
    L.orc_setup_coords.argtypes = [C.c_int32, P, P, P, P, P, C.c_int32,
                                   C.POINTER(OrcOptions), C.POINTER(C.c_void_p)]
    L.orc_setup_system.argtypes = [C.c_int32, P, P, P, C.c_int32, P, C.c_int32, P, C.c_int32,
                                   C.POINTER(OrcOptions), C.POINTER(C.c_void_p)]
    L.orc_level_block.argtypes = [P, C.c_int, P]
    L.orc_resetup.argtypes = [P, P, P]
    L.orc_resetup.restype = C.c_int
    L.orc_num_levels.argtypes = [P]
    L.orc_level_sizes.argtypes = [P, C.c_int, P]
    L.orc_level_scalars.argtypes = [P, C.c_int, P]
    L.orc_export.argtypes = [P, C.c_int, C.c_int, P]
    L.orc_vcycle.argtypes = [P, P, P]
    L.orc_solve.argtypes = [P, P, P, P, P, P]
    L.orc_solve_gmres.argtypes = [P, P, P, C.c_int32, P, P, P]
    L.orc_destroy.argtypes = [P]
    L.orc_strength.argtypes = [C.c_int32, P, P, P, C.c_double, P]
    L.orc_distance_strength.argtypes = [C.c_int32, P, P, P, C.c_int32, C.c_double, C.c_int32,
                                        P]
    L.orc_aggregate.argtypes = [C.c_int32, P, P, P, C.c_int32, C.c_uint64, C.c_int32, C.c_int32,
                                P, P, P]
    L.orc_sprsfy.argtypes = [C.c_int32, P, P, P, P, P, C.c_int32]
    L.orc_lump.argtypes = [C.c_int32, P, P, P, P, C.c_int32, C.c_double, P, P, P]
    L.orc_diag.argtypes = [C.c_int32, P, P, P, C.c_int32, C.c_double, P]
    L.orc_spmv.argtypes = [C.c_int32, C.c_int32, P, P, P, P, P]
    L.orc_power.argtypes = [C.c_int32, P, P, P, P, C.c_int32, C.c_uint64, C.c_int32,
                            C.c_int32, P]
    L.orc_prolongator.argtypes = [C.c_int32, P, P, P, P, P, C.c_double, P, P, P]
    L.orc_cnstrnt.argtypes = [C.c_int32, P, P, P, P]
    L.orc_spgemm_row.argtypes = [P, P, P, P, P, P, C.c_int32, C.c_int32, P, P]
    L.orc_dot.argtypes = [C.c_int64, P, P]
    L.orc_dot.restype = C.c_double
    L.orc_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
    L.orc_splitmix64.restype = C.c_uint64


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


class OracleError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"oracle status {code}: {msg}")
        self.code = code


def _check(code):
    if code < 0:
        raise OracleError(code, lib().orc_last_error().decode())
    return code


def make_options(theta=0.02, variants=(), one_norm_power=0, tau=1.1, sigma=1.0 / 3.0,
                 power_iters=10, agg_order=0, seed=12345, max_levels=10, max_coarse=1000,
                 smoother="chebyshev", degree=2, cheb_ratio=10.0, cheb_boost=1.0, rtol=1e-8,
                 max_iter=500, pcg_beta="fr", dist_power=1, coarse_solver="cholesky",
                 isolated="left_out", **_ignored) -> OrcOptions:
    o = OrcOptions()
    lib().orc_default_options(C.byref(o))
    o.theta = theta
    bits = 0
    for v in variants:
        bits |= VARIANT_BITS[v.lower()]
    o.variants = bits
    o.one_norm_power = one_norm_power
    o.tau = tau
    o.sigma = sigma
    o.power_iters = power_iters
    o.agg_order = 1 if agg_order in (1, "hashed") else 0
    o.seed = seed
    o.max_levels = max_levels
    o.max_coarse = max_coarse
    o.smoother = 1 if smoother in (1, "jacobi") else 0
    o.degree = degree
    o.cheb_ratio = cheb_ratio
    o.cheb_boost = cheb_boost
    o.rtol = rtol
    o.max_iter = max_iter
    o.pcg_beta = 1 if pcg_beta in (1, "pr") else 0
    o.dist_power = dist_power
    o.coarse_solver = 1 if coarse_solver in (1, "lu") else 0
    o.singletons = 1 if isolated in (1, "singleton") else 0
    return o


class Level:
    pass


class OracleHierarchy:
    """Runs the oracle setup; every level's arrays are exported into numpy."""

    def __init__(self, n, rp, col, val, nullspace=None, coords=None, block_size=None, **opts):
        """``coords`` (points x dim, dim 1..3) selects the distance-Laplacian strength.
        ``block_size`` selects systems SA: ``nullspace`` is then an n x k matrix (node-major
        dofs) and coordinates are per node."""
        self.opts = make_options(**opts)
        self._keep = (_i32(rp), _i32(col), _f64(val))
        self.system = block_size is not None
        npts = n // block_size if self.system else n
        X, self.dim = None, 0
        if coords is not None:
            X = _f64(coords).reshape(npts, -1)
            self.dim = X.shape[1]
        h = C.c_void_p()
        if self.system:
            Bm = _f64(nullspace).reshape(n, -1)
            self.k = Bm.shape[1]
            _check(lib().orc_setup_system(n, _p(self._keep[0]), _p(self._keep[1]),
                                          _p(self._keep[2]), block_size, _p(Bm), self.k,
                                          None if X is None else _p(X), self.dim,
                                          C.byref(self.opts), C.byref(h)))
        else:
            B = None if nullspace is None else _f64(nullspace)
            _check(lib().orc_setup_coords(n, _p(self._keep[0]), _p(self._keep[1]),
                                          _p(self._keep[2]), None if B is None else _p(B),
                                          None if X is None else _p(X), self.dim,
                                          C.byref(self.opts), C.byref(h)))
        self.h = h
        self.levels = [self._export(l) for l in range(lib().orc_num_levels(h))]

    def _export(self, l):
        L = lib()
        s = np.zeros(8, dtype=np.int64)
        _check(L.orc_level_sizes(self.h, l, _p(s)))
        sc = np.zeros(4)
        _check(L.orc_level_scalars(self.h, l, _p(sc)))
        n, nnz, nc, nab, nP, nR, nG, last = (int(v) for v in s)
        lv = Level()
        lv.n, lv.nnz, lv.nc, lv.coarsest = n, nnz, nc, bool(last)
        lv.nnzG = nG

        def ex(what, count, dtype):
            a = np.empty(count, dtype=dtype)
            if count:
                _check(L.orc_export(self.h, l, what, _p(a)))
            return a

        lv.A = (ex(0, n + 1, np.int32), ex(1, nnz, np.int32), ex(2, nnz, np.float64))
        npts = n
        lv.bs = 1
        ncd = nc  # coarse unknowns: aggregates, times k for systems
        if self.system:
            bl = np.zeros(6, dtype=np.int64)
            _check(L.orc_level_block(self.h, l, _p(bl)))
            lv.bs, k, nPt, nodes, nG, nB = (int(v) for v in bl)
            npts = n // lv.bs
            ncd = nc * k
            lv.B = ex(22, nB, np.float64).reshape(n, k)
            if not last:
                lv.Pt = (ex(19, n + 1, np.int32), ex(20, nPt, np.int32), ex(21, nPt, np.float64))
                lv.nmask = ex(23, nG, np.uint8)
                lv.Gn = (ex(24, nodes + 1, np.int32), ex(25, nG, np.int32))
        if not last:
            lv.mask = ex(3, nnz, np.uint8)
            lv.agg = ex(4, npts, np.int32)
            lv.is_root = ex(5, npts, np.uint8)
            lv.Abar = (ex(6, n + 1, np.int32), ex(7, nab, np.int32), ex(8, nab, np.float64))
            lv.invD = ex(9, n, np.float64)
            lv.P = (ex(10, n + 1, np.int32), ex(11, nP, np.int32), ex(12, nP, np.float64))
            lv.R = (ex(13, ncd + 1, np.int32), ex(14, nR, np.int32), ex(15, nR, np.float64))
            lv.sm_invD = ex(16, n, np.float64)
            lv.As_val = ex(17, nnz, np.float64)
            lv.lam, lv.omega, lv.sm_lam = float(sc[0]), float(sc[1]), float(sc[2])
        if self.dim:
            lv.coords = ex(18, npts * self.dim, np.float64).reshape(npts, self.dim)
        return lv

    @property
    def operator_complexity(self):
        return sum(l.nnz for l in self.levels) / self.levels[0].nnz

    def vcycle(self, f):
        f = _f64(f)
        u = np.empty_like(f)
        _check(lib().orc_vcycle(self.h, _p(f), _p(u)))
        return u

    def resetup(self, val, nullspace=None):
        """Numeric re-setup (orc_resetup): new values on the setup's pattern, the setup's
        symbolic decisions kept; every level is exported again."""
        v = _f64(val)
        B = None if nullspace is None else _f64(nullspace)
        self._keep = (self._keep[0], self._keep[1], v)
        _check(lib().orc_resetup(self.h, _p(v), None if B is None else _p(B)))
        self.levels = [self._export(l) for l in range(lib().orc_num_levels(self.h))]

    def solve(self, b, history=False):
        b = _f64(b)
        x = np.empty_like(b)
        it = C.c_int32()
        rr = C.c_double()
        hist = np.zeros(self.opts.max_iter + 1) if history else None
        code = _check(lib().orc_solve(self.h, _p(b), _p(x), C.byref(it), C.byref(rr),
                                      None if hist is None else _p(hist)))
        out = {"x": x, "iterations": it.value, "rel_residual": rr.value,
               "converged": code == 0}
        if history:
            out["history"] = hist[: it.value + 1]
        return out

    def solve_gmres(self, b, restart=30, history=False):
        """Restarted flexible GMRES with the V-cycle as right preconditioner; ``history``
        holds the residual norm after each Arnoldi step (index 0: ||b||)."""
        b = _f64(b)
        x = np.empty_like(b)
        it = C.c_int32()
        rr = C.c_double()
        hist = np.zeros(self.opts.max_iter + 1) if history else None
        code = _check(lib().orc_solve_gmres(self.h, _p(b), _p(x), restart, C.byref(it),
                                            C.byref(rr), None if hist is None else _p(hist)))
        out = {"x": x, "iterations": it.value, "rel_residual": rr.value,
               "converged": code == 0}
        if history:
            out["history"] = hist[: it.value + 1]
        return out

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().orc_destroy(self.h)
                self.h = None
        except Exception:
            pass


# ---- single steps ---------------------------------------------------------------------

def strength(n, rp, col, val, theta):
    m = np.empty(int(rp[n]), dtype=np.uint8)
    rp, col, val = _i32(rp), _i32(col), _f64(val)
    _check(lib().orc_strength(n, _p(rp), _p(col), _p(val), theta, _p(m)))
    return m


def distance_strength(n, rp, col, coords, theta, dist_power=1):
    rp, col, X = _i32(rp), _i32(col), _f64(coords).reshape(n, -1)
    m = np.empty(int(rp[n]), dtype=np.uint8)
    _check(lib().orc_distance_strength(n, _p(rp), _p(col), _p(X), X.shape[1], theta,
                                       dist_power, _p(m)))
    return m


def aggregate(n, rp, col, mask, order=0, seed=12345, level=0, isolated="left_out"):
    """isolated: "left_out" (agg -1 for a vertex without strong connections) or "singleton"
    (a singleton aggregate each)."""
    rp, col, mask = _i32(rp), _i32(col), _u8(mask)
    agg = np.empty(n, dtype=np.int32)
    root = np.empty(n, dtype=np.uint8)
    nc = C.c_int32()
    _check(lib().orc_aggregate(n, _p(rp), _p(col), _p(mask), order, seed, level,
                               1 if isolated in (1, "singleton") else 0, _p(agg), _p(root),
                               C.byref(nc)))
    return agg, root, nc.value


def sprsfy(n, rp, col, mask, agg, is_root, nc):
    rp, col, agg, is_root = _i32(rp), _i32(col), _i32(agg), _u8(is_root)
    m = _u8(mask).copy()
    _check(lib().orc_sprsfy(n, _p(rp), _p(col), _p(m), _p(agg), _p(is_root), nc))
    return m


def lump(n, rp, col, val, mask, offlmp=False, tau=1.1):
    rp, col, val, mask = _i32(rp), _i32(col), _f64(val), _u8(mask)
    orp = np.empty(n + 1, dtype=np.int32)
    ocol = np.empty(int(rp[n]), dtype=np.int32)
    oval = np.empty(int(rp[n]), dtype=np.float64)
    _check(lib().orc_lump(n, _p(rp), _p(col), _p(val), _p(mask), int(offlmp), tau, _p(orp),
                          _p(ocol), _p(oval)))
    m = int(orp[n])
    return orp, ocol[:m].copy(), oval[:m].copy()


def diag(n, rp, col, val, one_norm=False, sigma=1.0 / 3.0):
    rp, col, val = _i32(rp), _i32(col), _f64(val)
    d = np.empty(n)
    _check(lib().orc_diag(n, _p(rp), _p(col), _p(val), int(one_norm), sigma, _p(d)))
    return d


def spmv(rp, col, val, x, ncols=None):
    """y = A x, each row's products added sequentially in ascending column order from 0.0."""
    rp, col, val, x = _i32(rp), _i32(col), _f64(val), _f64(x)
    nr = len(rp) - 1
    nc = len(x) if ncols is None else ncols
    y = np.empty(nr)
    _check(lib().orc_spmv(nr, nc, _p(rp), _p(col), _p(val), _p(x), _p(y)))
    return y


def power(n, rp, col, val, invD, iters=10, seed=12345, level=0, stream=0):
    rp, col, val, invD = _i32(rp), _i32(col), _f64(val), _f64(invD)
    lam = C.c_double()
    _check(lib().orc_power(n, _p(rp), _p(col), _p(val), _p(invD), iters, seed, level, stream,
                           C.byref(lam)))
    return lam.value


def prolongator(n, rp, col, val, invD, agg, omega):
    rp, col, val, invD, agg = _i32(rp), _i32(col), _f64(val), _f64(invD), _i32(agg)
    orp = np.empty(n + 1, dtype=np.int32)
    ocol = np.empty(int(rp[n]), dtype=np.int32)
    oval = np.empty(int(rp[n]), dtype=np.float64)
    _check(lib().orc_prolongator(n, _p(rp), _p(col), _p(val), _p(invD), _p(agg), omega,
                                 _p(orp), _p(ocol), _p(oval)))
    m = int(orp[n])
    return orp, ocol[:m].copy(), oval[:m].copy()


def cnstrnt(n, rp, col, val, agg):
    rp, col, agg = _i32(rp), _i32(col), _i32(agg)
    v = _f64(val).copy()
    _check(lib().orc_cnstrnt(n, _p(rp), _p(col), _p(v), _p(agg)))
    return v


def spgemm_row(X, Y, ncols_y, row):
    """Row ``row`` of X*Y; X, Y are (rp, col, val) tuples."""
    xrp, xcol, xval = _i32(X[0]), _i32(X[1]), _f64(X[2])
    yrp, ycol, yval = _i32(Y[0]), _i32(Y[1]), _f64(Y[2])
    cap = 0
    for e in range(int(xrp[row]), int(xrp[row + 1])):
        k = int(xcol[e])
        cap += int(yrp[k + 1] - yrp[k])
    oc = np.empty(max(cap, 1), dtype=np.int32)
    ov = np.empty(max(cap, 1))
    c = _check(lib().orc_spgemm_row(_p(xrp), _p(xcol), _p(xval), _p(yrp), _p(ycol), _p(yval),
                                    ncols_y, row, _p(oc), _p(ov)))
    return oc[:c].copy(), ov[:c].copy()


def dot(x, y):
    x, y = _f64(x), _f64(y)
    return lib().orc_dot(x.size, _p(x), _p(y))


def splitmix64(seed, k):
    return lib().orc_splitmix64(seed, k)
