"""Python front end of the SA-AMG library: options, setup, solve, exports.

PyTorch provides device memory and the stream; every computation runs in libsaamg.so.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import Sequence

import numpy as np

from . import _lib

VARIANT_BITS = {"sprsfy": 1, "offlmp": 2, "1norm": 4, "cnstrnt": 8}


@dataclass
class Options:
    """Mirror of sa_options (include/saamg.h); defaults follow the paper where it states them."""

    theta: float = 0.02
    variants: Sequence[str] = field(default_factory=tuple)
    tau: float = 1.1
    sigma: float = 1.0 / 3.0
    one_norm_power: int = 0
    power_iters: int = 10
    seed: int = 12345
    agg_order: str = "natural"
    max_levels: int = 10
    max_coarse: int = 1000
    smoother: str = "chebyshev"
    degree: int = 2
    precision: str = "fp64"
    cheb_ratio: float = 10.0
    cheb_boost: float = 1.0
    rtol: float = 1e-8
    max_iter: int = 500
    pcg_beta: str = "auto"
    dist_power: int = 1
    coarse_solver: str = "cholesky"
    isolated: str = "left_out"

    def to_c(self) -> _lib.SaOptions:
        o = _lib.SaOptions()
        _lib.lib().sa_default_options(C.byref(o))
        bits = 0
        for v in self.variants:
            bits |= VARIANT_BITS[v.lower()]
        o.variants = bits
        o.theta = self.theta
        o.tau = self.tau
        o.sigma = self.sigma
        o.one_norm_power = self.one_norm_power
        o.power_iters = self.power_iters
        o.seed = self.seed
        o.agg_order = 1 if self.agg_order in ("hashed", 1) else 0
        o.max_levels = self.max_levels
        o.max_coarse = self.max_coarse
        o.smoother = 1 if self.smoother in ("jacobi", 1) else 0
        o.degree = self.degree
        o.precision = 1 if self.precision in ("fp32", "fp32_vcycle", 1) else 0
        o.cheb_ratio = self.cheb_ratio
        o.cheb_boost = self.cheb_boost
        o.rtol = self.rtol
        o.max_iter = self.max_iter
        o.pcg_beta = {"auto": -1, "fr": 0, "pr": 1}[self.pcg_beta]
        o.dist_power = self.dist_power
        o.coarse_solver = 1 if self.coarse_solver in ("lu", 1) else 0
        o.isolated = 1 if self.isolated in ("singleton", 1) else 0
        return o

    def as_dict(self) -> dict:
        d = dict(self.__dict__)
        d["variants"] = list(self.variants)
        return d


def _torch():
    import torch
    return torch


def _stream_handle(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev(a, dtype):
    torch = _torch()
    if isinstance(a, torch.Tensor):
        t = a.to(device="cuda", dtype=dtype)
    else:
        t = torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)
    return t.contiguous()


class Hierarchy:
    """A device-resident SA-AMG hierarchy (sa_hierarchy)."""

    def __init__(self, n, rp, col, val, nullspace=None, options: Options | None = None,
                 stream=None, coords=None, block_size=None):
        """``coords`` (points x dim node coordinates, dim 1..3) selects the distance-Laplacian
        strength test (sa_setup_coords).  ``block_size`` selects systems SA
        (sa_setup_system): ``nullspace`` is then n x k, node-major unknowns."""
        torch = _torch()
        self.options = options or Options()
        self.n = int(n)
        self._stream = stream
        L = _lib.lib()
        drp = _dev(rp, torch.int32)
        dcol = _dev(col, torch.int32)
        dval = _dev(val, torch.float64)
        csr = _lib.SaCsr(self.n, int(dcol.numel()), drp.data_ptr(), dcol.data_ptr(),
                         dval.data_ptr(), _lib.SA_DEVICE)
        dB = None if (nullspace is None or block_size is not None) else _dev(nullspace,
                                                                             torch.float64)
        ctx = _lib.SaContext(_stream_handle(stream))
        opts = self.options.to_c()
        h = C.c_void_p()
        self.block_size = block_size
        if block_size is not None:
            dB = _dev(nullspace, torch.float64).reshape(self.n, -1).contiguous()
            k = int(dB.shape[1])
            dX = None if coords is None else _dev(coords, torch.float64).reshape(
                self.n // block_size, -1).contiguous()
            self.dim = 0 if dX is None else int(dX.shape[1])
            code = L.sa_setup_system(C.byref(ctx), C.byref(csr), block_size,
                                     C.c_void_p(dB.data_ptr()), k,
                                     None if dX is None else C.c_void_p(dX.data_ptr()), self.dim,
                                     C.byref(opts), C.byref(h))
            _lib.check(code, "sa_setup_system")
        elif coords is None:
            code = L.sa_setup(C.byref(ctx), C.byref(csr),
                              None if dB is None else C.c_void_p(dB.data_ptr()),
                              C.byref(opts), C.byref(h))
            _lib.check(code, "sa_setup")
        else:
            dX = _dev(coords, torch.float64).reshape(self.n, -1).contiguous()
            self.dim = int(dX.shape[1])
            code = L.sa_setup_coords(C.byref(ctx), C.byref(csr),
                                     None if dB is None else C.c_void_p(dB.data_ptr()),
                                     C.c_void_p(dX.data_ptr()), self.dim, C.byref(opts),
                                     C.byref(h))
            _lib.check(code, "sa_setup_coords")
        self._h = h

    @classmethod
    def from_problem(cls, p, nullspace=None, options=None, stream=None, coords=None,
                     block_size=None):
        return cls(p.n, p.rp, p.col, p.val, nullspace=nullspace, options=options, stream=stream,
                   coords=coords, block_size=block_size)

    # ---- numeric re-setup ---------------------------------------------------------------
    def resetup(self, val, nullspace=None):
        """New matrix values on the setup's pattern (sa_resetup): keeps strength labels,
        aggregates and every sparsity pattern, recomputes all numbers."""
        torch = _torch()
        dval = _dev(val, torch.float64)
        dB = None if nullspace is None else _dev(nullspace, torch.float64)
        _lib.check(_lib.lib().sa_resetup(self._h, C.c_void_p(dval.data_ptr()),
                                         None if dB is None else C.c_void_p(dB.data_ptr()),
                                         _lib.SA_DEVICE), "sa_resetup")

    # ---- solve ------------------------------------------------------------------------
    def solve(self, b, x=None):
        """CG + V-cycle; b may be numpy or a CUDA tensor.  Returns (x, iterations, relres,
        status) with x a float64 CUDA tensor."""
        torch = _torch()
        db = _dev(b, torch.float64)
        if x is None:
            x = torch.empty(self.n, dtype=torch.float64, device="cuda")
        it = C.c_int32()
        rr = C.c_double()
        code = _lib.lib().sa_solve(self._h, C.c_void_p(db.data_ptr()), C.c_void_p(x.data_ptr()),
                                   _lib.SA_DEVICE, C.byref(it), C.byref(rr))
        _lib.check(code, "sa_solve")
        return x, it.value, rr.value, _lib.STATUS_NAMES[code]

    def solve_gmres(self, b, x=None, restart: int = 30, noalloc: bool = False):
        """Restarted flexible GMRES with the V-cycle as right preconditioner
        (sa_solve_gmres; with noalloc, sa_solve_gmres_noalloc, whose workspace is the
        library's fixed scratch array).  Returns (x, iterations, relres, status)."""
        torch = _torch()
        db = _dev(b, torch.float64)
        if x is None:
            x = torch.empty(self.n, dtype=torch.float64, device="cuda")
        it = C.c_int32()
        rr = C.c_double()
        name = "sa_solve_gmres_noalloc" if noalloc else "sa_solve_gmres"
        code = getattr(_lib.lib(), name)(self._h, C.c_void_p(db.data_ptr()),
                                         C.c_void_p(x.data_ptr()), _lib.SA_DEVICE, restart,
                                         C.byref(it), C.byref(rr))
        _lib.check(code, name)
        return x, it.value, rr.value, _lib.STATUS_NAMES[code]

    def vcycle(self, f):
        torch = _torch()
        df = _dev(f, torch.float64)
        z = torch.empty_like(df)
        _lib.check(_lib.lib().sa_vcycle(self._h, C.c_void_p(df.data_ptr()),
                                        C.c_void_p(z.data_ptr())), "sa_vcycle")
        return z

    # ---- inspection -----------------------------------------------------------------------
    def info(self) -> dict:
        inf = _lib.SaInfo()
        _lib.check(_lib.lib().sa_hierarchy_info(self._h, C.byref(inf)), "sa_hierarchy_info")
        nl = inf.levels
        return {"levels": nl, "n": list(inf.n[:nl]), "nnz": list(inf.nnz[:nl]),
                "nnz_p": list(inf.nnz_p[:nl]), "lambda": list(inf.lambda_[:nl]),
                "omega": list(inf.omega[:nl]), "smoother_lambda": list(inf.smoother_lambda[:nl]),
                "mis_rounds": list(inf.mis_rounds[:nl]),
                "operator_complexity": inf.operator_complexity,
                "device_bytes": inf.device_bytes, "setup_seconds": inf.setup_seconds}

    def export(self, level: int, what: str) -> np.ndarray:
        L = _lib.lib()
        cnt = C.c_int64()
        _lib.check(L.sa_export_size(self._h, level, _lib.PARTS[what], C.byref(cnt)),
                   "sa_export_size")
        out = np.empty(cnt.value, dtype=_lib.PART_DTYPE[what])
        if cnt.value:
            _lib.check(L.sa_export_level(self._h, level, _lib.PARTS[what],
                                         out.ctypes.data_as(C.c_void_p), out.nbytes),
                       "sa_export_level")
        return out

    def export_csr(self, level: int, name: str):
        return (self.export(level, f"{name}_rp"), self.export(level, f"{name}_col"),
                self.export(level, f"{name}_val"))

    def profile(self, on: bool = True):
        """Enable/disable HIP-event timing of the fine-level SpMV launches in solve()."""
        _lib.check(_lib.lib().sa_profile_enable(self._h, 1 if on else 0), "sa_profile_enable")

    def profile_read(self) -> dict:
        n = C.c_int64()
        ms = C.c_double()
        by = C.c_double()
        _lib.check(_lib.lib().sa_profile_read(self._h, C.byref(n), C.byref(ms), C.byref(by)),
                   "sa_profile_read")
        return {"launches": n.value, "ms": ms.value, "bytes": by.value}

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().sa_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_many(hierarchies, rhs):
    """Solves every (hierarchy, b) pair in lockstep (sa_solve_many): one grouped launch per
    CG/V-cycle step for all of them.  Returns a list of (x, iterations, rel_residual, status),
    each equal to what Hierarchy.solve gives for that system alone."""
    torch = _torch()
    k = len(hierarchies)
    bs = [_dev(b, torch.float64) for b in rhs]
    xs = [torch.empty(h.n, dtype=torch.float64, device="cuda") for h in hierarchies]
    H = (C.c_void_p * k)(*[h._h.value for h in hierarchies])
    B = (C.c_void_p * k)(*[b.data_ptr() for b in bs])
    X = (C.c_void_p * k)(*[x.data_ptr() for x in xs])
    its = (C.c_int32 * k)()
    rr = (C.c_double * k)()
    st = (C.c_int * k)()
    _lib.check(_lib.lib().sa_solve_many(H, k, B, X, _lib.SA_DEVICE, its, rr, st),
               "sa_solve_many")
    return [(xs[i], its[i], rr[i], _lib.STATUS_NAMES[st[i]]) for i in range(k)]


def estimate_bytes(n: int, nnz: int) -> int:
    """Device bytes a serving request is charged at admission (sa_estimate_bytes)."""
    return int(_lib.lib().sa_estimate_bytes(int(n), int(nnz)))


class Server:
    """Many independent setup+solve requests on one GPU (sa_server_*): FIFO admission under
    an HBM budget, max_slots requests in flight, each on its own stream.  Inputs are host
    numpy arrays, copied at submit, or with borrow=True (sa_server_submit_borrowed) kept by
    reference until the result has been collected; results come back as host numpy arrays."""

    def __init__(self, hbm_budget: int = 8 << 30, max_slots: int = 4):
        h = C.c_void_p()
        _lib.check(_lib.lib().sa_server_create(None, int(hbm_budget), int(max_slots),
                                               C.byref(h)), "sa_server_create")
        self._s = h
        self._held = {}  # ticket -> the borrowed arrays, alive until the result is collected

    def submit(self, A, b, options: Options | None = None, borrow: bool = False) -> int:
        """A: CsrProblem or (n, rp, col, val) of host arrays; returns the ticket."""
        if hasattr(A, "rp"):
            n, rp, col, val = A.n, A.rp, A.col, A.val
        else:
            n, rp, col, val = A
        rp = np.ascontiguousarray(rp, dtype=np.int32)
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        b = np.ascontiguousarray(b, dtype=np.float64)
        csr = _lib.SaCsr(int(n), int(col.size), rp.ctypes.data, col.ctypes.data,
                         val.ctypes.data, _lib.SA_HOST)
        opts = (options or Options()).to_c()
        t = C.c_uint64()
        fn = _lib.lib().sa_server_submit_borrowed if borrow else _lib.lib().sa_server_submit
        _lib.check(fn(self._s, C.byref(csr), C.c_void_p(b.ctypes.data), C.byref(opts),
                      C.byref(t)), "sa_server_submit")
        if borrow:
            self._held[t.value] = (rp, col, val, b)
        return t.value

    def _collect(self, fn, ticket, n):
        x = np.empty(n, dtype=np.float64)
        r = _lib.SaResult()
        code = fn(self._s, C.c_uint64(ticket), C.c_void_p(x.ctypes.data), _lib.SA_HOST,
                  C.byref(r))
        return code, x, r

    def wait(self, ticket: int, n: int):
        """Blocks until the request is done: (x, result dict).  A failed request raises."""
        code, x, r = self._collect(_lib.lib().sa_server_wait, ticket, n)
        self._held.pop(ticket, None)
        _lib.check(code, "sa_server_wait")
        return x, r.as_dict()

    def poll(self, ticket: int, n: int):
        """None while pending, else (x, result dict).  A failed request raises."""
        code, x, r = self._collect(_lib.lib().sa_server_poll, ticket, n)
        if code == _lib.SA_PENDING:
            return None
        self._held.pop(ticket, None)
        _lib.check(code, "sa_server_poll")
        return x, r.as_dict()

    def drain(self):
        _lib.check(_lib.lib().sa_server_drain(self._s), "sa_server_drain")

    def stats(self) -> dict:
        st = _lib.SaServerStats()
        _lib.check(_lib.lib().sa_server_get_stats(self._s, C.byref(st)), "sa_server_get_stats")
        return st.as_dict()

    def close(self):
        if getattr(self, "_s", None):
            _lib.lib().sa_server_destroy(self._s)
            self._s = None
        self._held = {}  # destroy has returned: no request reads the borrowed arrays any more

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def setup(A, nullspace=None, options: Options | None = None, stream=None) -> Hierarchy:
    """setup(A, nullspace, options) -> hierarchy.  A is a CsrProblem or an (n, rp, col, val)
    tuple (numpy or CUDA tensors)."""
    if hasattr(A, "rp"):
        return Hierarchy.from_problem(A, nullspace, options, stream)
    n, rp, col, val = A
    return Hierarchy(n, rp, col, val, nullspace, options, stream)


def solve(h: Hierarchy, b):
    """solve(hierarchy, b) -> (x, iterations)."""
    x, it, _, _ = h.solve(b)
    return x, it
