"""Python binding of libhot (argument marshalling only).

Every numerical step runs in the HIP kernels of ``lib/libhot.so``; this module
only moves pointers, sizes and streams across the C ABI declared in
``include/hot.h``.  PyTorch provides device memory and the current stream.
If the library is missing the import of ``lib()`` raises: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libhot.so")

HOT_OK, HOT_E_INVALID, HOT_E_NOMEM, HOT_E_DEVICE, HOT_E_NOT_CONVERGED = 0, 1, 2, 3, 4
HOT_E_BUSY, HOT_E_CANCELLED, HOT_E_NUMERIC = 5, 6, 7
HOT_FP64, HOT_FP32_STREAM = 0, 1
HOT_FLAG_RESTART, HOT_FLAG_FIXED_ITERS, HOT_FLAG_ADMM, HOT_FLAG_ABS_KKT = 0x1, 0x2, 0x4, 0x8
HOT_FLAG_SIGMA_UPDATE, HOT_FLAG_ESCALATE = 0x10, 0x20
HOT_SERVER_SHARED = 0x1

EXPORTED = [
    "hot_ctx_create", "hot_ctx_destroy", "hot_ctx_last_error", "hot_status_string",
    "hot_footprint_bytes", "hot_ctx_footprint_bytes", "hot_plan_capacity", "hot_solve", "hot_solution_export",
    "hot_solution_free", "hot_recover_plan", "hot_aat_solve", "hot_batch_submit",
    "hot_batch_wait", "hot_server_create", "hot_server_submit", "hot_server_poll",
    "hot_server_stats", "hot_server_destroy", "hot_server_drain", "hot_ctx_set_profiling",
    "hot_ctx_profile_read", "hot_autotune", "hot_autotune_load", "hot_solution_anchor",
    "hot_solve_noalloc", "hot_noalloc_capacity", "hot_server_cancel",
]


class ServerConfig(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_slots", C.c_int32),
                ("flags", C.c_uint32)]


class Problem(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("mu1", C.c_void_p), ("mu2", C.c_void_p),
                ("tol", C.c_double), ("max_iter", C.c_int32), ("check_every", C.c_int32),
                ("sigma", C.c_double), ("prec", C.c_int32), ("flags", C.c_uint32),
                ("relax", C.c_double), ("coord_row", C.c_void_p), ("coord_col", C.c_void_p)]


class Result(C.Structure):
    _fields_ = [("primal_obj", C.c_double), ("dual_obj", C.c_double), ("kkt", C.c_double),
                ("res_primal", C.c_double), ("res_dual", C.c_double), ("res_comp", C.c_double),
                ("sigma", C.c_double), ("seconds", C.c_double), ("kkt_abs", C.c_double),
                ("iters", C.c_int32),
                ("restarts", C.c_int32), ("status", C.c_int32), ("escalated_at", C.c_int32),
                ("feaserr", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


class HotError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status_string(status)} ({status}): {msg}")
        self.status = status


def lib():
    """Load libhot.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libhot.so not built at {LIB_PATH}; run __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.hot_ctx_create.argtypes = [C.c_int, C.POINTER(vp)]
    L.hot_ctx_destroy.argtypes = [vp]
    L.hot_ctx_last_error.argtypes = [vp]
    L.hot_ctx_last_error.restype = C.c_char_p
    L.hot_status_string.argtypes = [C.c_int]
    L.hot_status_string.restype = C.c_char_p
    L.hot_footprint_bytes.argtypes = [i32, i32, i32, C.c_uint32]
    L.hot_footprint_bytes.restype = C.c_size_t
    L.hot_ctx_footprint_bytes.argtypes = [vp, i32, i32, i32, C.c_uint32]
    L.hot_ctx_footprint_bytes.restype = C.c_size_t
    L.hot_plan_capacity.argtypes = [i32, i32]
    L.hot_plan_capacity.restype = i64
    L.hot_solve.argtypes = [vp, C.POINTER(Problem), vp, C.POINTER(vp), C.POINTER(Result)]
    L.hot_solution_export.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.hot_solution_free.argtypes = [vp]
    L.hot_aat_solve.argtypes = [vp, i32, i32, vp, vp, vp]
    L.hot_batch_submit.argtypes = [vp, C.POINTER(Problem), i32, vp, C.POINTER(vp)]
    L.hot_batch_wait.argtypes = [vp, C.POINTER(Result)]
    L.hot_server_create.argtypes = [vp, C.POINTER(ServerConfig), C.POINTER(vp)]
    L.hot_server_submit.argtypes = [vp, C.POINTER(Problem), C.c_uint64]
    L.hot_server_poll.argtypes = [vp, C.POINTER(Result), C.POINTER(C.c_uint64),
                                  C.POINTER(dbl), i32]
    L.hot_server_poll.restype = i32
    L.hot_server_drain.argtypes = [vp, dbl]
    L.hot_server_stats.argtypes = [vp, C.POINTER(dbl)]
    L.hot_server_destroy.argtypes = [vp]
    L.hot_autotune.argtypes = [vp, C.POINTER(Problem), i32, i32, C.c_char_p, C.POINTER(dbl)]
    L.hot_autotune_load.argtypes = [vp, C.c_char_p]
    L.hot_ctx_set_profiling.argtypes = [vp, C.c_int]
    L.hot_ctx_profile_read.argtypes = [vp, C.POINTER(dbl)]
    L.hot_recover_plan.argtypes = [vp, vp, vp, vp, vp, vp, i64, C.POINTER(i64),
                                   C.POINTER(dbl)]
    L.hot_solution_anchor.argtypes = [vp, vp, vp, vp, C.POINTER(dbl)]
    L.hot_solve_noalloc.argtypes = [vp, C.POINTER(Problem), vp, vp, vp, C.POINTER(Result)]
    L.hot_noalloc_capacity.argtypes = []
    L.hot_noalloc_capacity.restype = C.c_size_t
    L.hot_server_cancel.argtypes = [vp]
    for name in EXPORTED:
        getattr(L, name).restype = getattr(L, name).restype or C.c_int
    L.hot_ctx_destroy.restype = None
    L.hot_solution_free.restype = None
    L.hot_server_destroy.restype = None
    L.hot_server_poll.restype = i32
    _lib = L
    return L


def status_string(s):
    try:
        return lib().hot_status_string(int(s)).decode()
    except Exception:  # pragma: no cover - only while the library is missing
        return str(s)


def footprint_bytes(m, n, prec=HOT_FP64, flags=HOT_FLAG_RESTART):
    return int(lib().hot_footprint_bytes(m, n, prec, flags))


def plan_capacity(m, n):
    return int(lib().hot_plan_capacity(m, n))


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_f64(t):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return t


class Context:
    """Owns a hot_ctx on one device."""

    def __init__(self, device: int = 0):
        L = lib()
        h = C.c_void_p()
        st = L.hot_ctx_create(device, C.byref(h))
        if st != HOT_OK:
            raise HotError(st, "hot_ctx_create failed (no usable GPU?)")
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            lib().hot_ctx_destroy(self.h)
            self.h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def set_profiling(self, on=True):
        lib().hot_ctx_set_profiling(self.h, 1 if on else 0)

    def profile(self):
        out = (C.c_double * 4)()
        lib().hot_ctx_profile_read(self.h, out)
        return {"slab_launches": out[0], "slab_seconds": out[1], "slab_bytes": out[2],
                "iterations_launched": out[3]}

    def last_error(self):
        return lib().hot_ctx_last_error(self.h).decode()

    def problem(self, mu1, mu2, tol=1e-6, max_iter=100000, check_every=10, sigma=0.0,
                prec=HOT_FP64, flags=HOT_FLAG_RESTART, relax=0.0, coord_row=None,
                coord_col=None):
        """Build a hot_problem.  The tensors it points to must stay alive
        while the problem is in use (callers keep a reference)."""
        mu1, mu2 = _dev_f64(mu1), _dev_f64(mu2)
        m, n = mu1.shape
        if tuple(mu2.shape) != (m, n):
            raise ValueError("histogram shapes differ")
        cu = None if coord_row is None else _dev_f64(coord_row).reshape(-1)
        cv = None if coord_col is None else _dev_f64(coord_col).reshape(-1)
        if cu is not None and cu.numel() != m:
            raise ValueError("coord_row must have m entries")
        if cv is not None and cv.numel() != n:
            raise ValueError("coord_col must have n entries")
        prob = Problem(m, n, mu1.data_ptr(), mu2.data_ptr(), tol, max_iter, check_every, sigma,
                       prec, flags, relax, None if cu is None else cu.data_ptr(),
                       None if cv is None else cv.data_ptr())
        prob._keep = (mu1, mu2, cu, cv)
        return prob

    def footprint_bytes(self, m, n, prec=HOT_FP64, flags=HOT_FLAG_RESTART):
        """Device bytes of one problem under this context's launch-shape tuning."""
        return int(lib().hot_ctx_footprint_bytes(self.h, m, n, prec, flags))

    def solve(self, mu1, mu2, keep=False, stream=None, raise_on_error=True, **kw):
        """Run hot_solve; returns (result dict, Solution or None)."""
        prob = self.problem(mu1, mu2, **kw)
        res = Result()
        sol = C.c_void_p()
        st = lib().hot_solve(self.h, C.byref(prob), _stream_ptr(stream),
                             C.byref(sol) if keep else None, C.byref(res))
        if st not in (HOT_OK, HOT_E_NOT_CONVERGED) and raise_on_error:
            raise HotError(st, self.last_error())
        out = res.as_dict()
        out["return_status"] = st
        solution = Solution(self, sol, prob.m, prob.n, (mu1, mu2)) if keep and sol else None
        return out, solution

    def solve_noalloc(self, mu1, mu2, outputs=True, stream=None, **kw):
        """Run hot_solve_noalloc; returns (result dict, xbar, ybar) with the
        final iterate in caller-owned tensors (None unless outputs)."""
        import torch
        prob = self.problem(mu1, mu2, **kw)
        m, n = prob.m, prob.n
        xb = yb = None
        if outputs:
            xb = torch.empty(m * m * n + m * n * n, dtype=torch.float64, device=mu1.device)
            yb = torch.empty(3 * m * n - 1, dtype=torch.float64, device=mu1.device)
        res = Result()
        st = lib().hot_solve_noalloc(self.h, C.byref(prob), _stream_ptr(stream),
                                     None if xb is None else C.c_void_p(xb.data_ptr()),
                                     None if yb is None else C.c_void_p(yb.data_ptr()),
                                     C.byref(res))
        if st not in (HOT_OK, HOT_E_NOT_CONVERGED):
            raise HotError(st, self.last_error())
        out = res.as_dict()
        out["return_status"] = st
        return out, xb, yb

    def aat_solve(self, m, n, R, stream=None):
        import torch
        R = _dev_f64(R)
        y = torch.empty(3 * m * n - 1, dtype=torch.float64, device=R.device)
        st = lib().hot_aat_solve(self.h, m, n, C.c_void_p(R.data_ptr()),
                                 C.c_void_p(y.data_ptr()), _stream_ptr(stream))
        if st != HOT_OK:
            raise HotError(st, self.last_error())
        return y

    def autotune(self, pairs, iters=40, cache_path=None, **kw):
        """Tune the slab-pass launch shape for these shapes / precision."""
        probs = (Problem * len(pairs))(*[self.problem(a, b, **kw) for a, b in pairs])
        out = (C.c_double * 5)()
        st = lib().hot_autotune(self.h, probs, len(pairs), iters,
                                cache_path.encode() if cache_path else None, out)
        if st != HOT_OK:
            raise HotError(st, self.last_error())
        return {"item_elems": int(out[0]), "unroll": int(out[1]),
                "us_per_iter": out[2] * 1e6, "default_us_per_iter": out[3] * 1e6,
                "vec_per_lane": int(out[4])}

    def autotune_load(self, cache_path):
        return lib().hot_autotune_load(self.h, cache_path.encode()) == HOT_OK

    def _problems(self, pairs, kw):
        """pairs: (mu1, mu2) or (mu1, mu2, per-pair keyword dict)."""
        out = []
        for pr in pairs:
            extra = pr[2] if len(pr) > 2 else {}
            out.append(self.problem(pr[0], pr[1], **{**kw, **extra}))
        return out

    def batch_submit(self, pairs, stream=None, **kw):
        """pairs: list of (mu1, mu2) CUDA tensors, optionally with a third
        element holding per-pair keywords (e.g. coord_row / coord_col).
        Returns a Batch handle."""
        plist = self._problems(pairs, kw)
        probs = (Problem * len(pairs))(*plist)
        h = C.c_void_p()
        st = lib().hot_batch_submit(self.h, probs, len(pairs), _stream_ptr(stream), C.byref(h))
        if st != HOT_OK:
            raise HotError(st, self.last_error())
        return Batch(self, h, len(pairs), (pairs, [p._keep for p in plist]), probs)

    def batch_solve(self, pairs, **kw):
        return self.batch_submit(pairs, **kw).wait()


class Batch:
    def __init__(self, ctx, h, count, keep_alive, probs):
        self.ctx, self.h, self.count = ctx, h, count
        self._keep = (keep_alive, probs)

    def wait(self):
        res = (Result * self.count)()
        st = lib().hot_batch_wait(self.h, res)
        self.h = None
        if st != HOT_OK:
            raise HotError(st, self.ctx.last_error())
        return [r.as_dict() for r in res]


class Solution:
    """Device-resident final iterate of one solve."""

    def __init__(self, ctx, h, m, n, keep_alive):
        self.ctx, self.h, self.m, self.n = ctx, h, m, n
        self._keep = keep_alive

    def free(self):
        if self.h:
            lib().hot_solution_free(self.h)
            self.h = None

    def __del__(self):  # pragma: no cover
        try:
            self.free()
        except Exception:
            pass

    def export(self, stream=None):
        """Return (xbar, ybar, zbar, s) as float64 CUDA tensors in paper order."""
        import torch
        m, n = self.m, self.n
        N, M3 = m * m * n + m * n * n, 3 * m * n - 1
        dev = torch.device("cuda", self.ctx.device)
        xb = torch.empty(N, dtype=torch.float64, device=dev)
        zb = torch.empty(N, dtype=torch.float64, device=dev)
        s = torch.empty(N, dtype=torch.float64, device=dev)
        yb = torch.empty(M3, dtype=torch.float64, device=dev)
        st = lib().hot_solution_export(self.ctx.h, self.h, _stream_ptr(stream),
                                       C.c_void_p(xb.data_ptr()), C.c_void_p(yb.data_ptr()),
                                       C.c_void_p(zb.data_ptr()), C.c_void_p(s.data_ptr()))
        if st != HOT_OK:
            raise HotError(st, self.ctx.last_error())
        return xb, yb, zb, s

    def anchor(self, stream=None):
        """(s0 as a float64 CUDA tensor in paper order, info dict): the
        Halpern anchor of the final epoch and the control values."""
        import torch
        m, n = self.m, self.n
        s0 = torch.empty(m * m * n + m * n * n, dtype=torch.float64,
                         device=torch.device("cuda", self.ctx.device))
        info = (C.c_double * 4)()
        st = lib().hot_solution_anchor(self.ctx.h, self.h, _stream_ptr(stream),
                                       C.c_void_p(s0.data_ptr()), info)
        if st != HOT_OK:
            raise HotError(st, self.ctx.last_error())
        return s0, {"k": int(info[0]), "lam": info[1], "sigma": info[2],
                    "anchor": int(info[3])}

    def recover_plan(self, stream=None, capacity=None):
        """Algorithm 1 + marginal repair.  Returns (src, dst, mass, marg_err[4])."""
        import torch
        cap = capacity or plan_capacity(self.m, self.n)
        dev = torch.device("cuda", self.ctx.device)
        src = torch.empty(cap, dtype=torch.int32, device=dev)
        dst = torch.empty(cap, dtype=torch.int32, device=dev)
        mass = torch.empty(cap, dtype=torch.float64, device=dev)
        nnz = C.c_int64()
        err = (C.c_double * 4)()
        st = lib().hot_recover_plan(self.ctx.h, self.h, _stream_ptr(stream),
                                    C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
                                    C.c_void_p(mass.data_ptr()), cap, C.byref(nnz), err)
        if st != HOT_OK:
            raise HotError(st, self.ctx.last_error())
        k = nnz.value
        return src[:k], dst[:k], mass[:k], list(err)


class Server:
    """Continuous-batching service on one context (hot_server_*)."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int = 0, max_slots: int = 8,
                 shared: bool = False):
        self.ctx = ctx
        cfg = ServerConfig(hbm_budget_bytes, max_slots, HOT_SERVER_SHARED if shared else 0)
        h = C.c_void_p()
        st = lib().hot_server_create(ctx.h, C.byref(cfg), C.byref(h))
        if st != HOT_OK:
            raise HotError(st, ctx.last_error())
        self.h = h
        self._alive = {}

    def submit(self, mu1, mu2, tag: int, **kw):
        prob = self.ctx.problem(mu1, mu2, **kw)
        st = lib().hot_server_submit(self.h, C.byref(prob), tag)
        if st != HOT_OK:
            raise HotError(st, "submit rejected")
        # the server reads the histograms (and positions) when it admits the
        # request, possibly much later: keep every buffer alive until then
        self._alive[tag] = prob._keep

    def poll(self, max_results: int = 256):
        res = (Result * max_results)()
        tags = (C.c_uint64 * max_results)()
        lat = (C.c_double * max_results)()
        k = lib().hot_server_poll(self.h, res, tags, lat, max_results)
        out = []
        for q in range(k):
            d = res[q].as_dict()
            d["tag"], d["latency"] = int(tags[q]), float(lat[q])
            self._alive.pop(d["tag"], None)
            out.append(d)
        return out

    def cancel(self):
        st = lib().hot_server_cancel(self.h)
        if st != HOT_OK:
            raise HotError(st, "cancel failed")

    def drain(self, timeout: float = 600.0):
        return lib().hot_server_drain(self.h, timeout)

    def stats(self):
        out = (C.c_double * 9)()
        lib().hot_server_stats(self.h, out)
        keys = ["completed", "submitted", "queued", "resident", "bytes_resident",
                "max_resident", "p50", "p99", "max_shared"]
        return dict(zip(keys, list(out)))

    def close(self):
        if getattr(self, "h", None):
            lib().hot_server_destroy(self.h)
            self.h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass
