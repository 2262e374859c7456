"""ctypes binding of the C oracle (test infrastructure only).

Each function mirrors one routine of ``hot_oracle.c``; see that file for the
passage of the paper each one follows.  Arrays are float64 numpy arrays with
the paper's vectorisation (Sec. 2.1): x = [f1; f2] with f1_{i,k,j} at
(j*m+k)*m+i and f2_{k,j,l} at m*m*n + (l*n+j)*m+k.
"""
import ctypes as C
import os

import numpy as np

from .build import ensure_built

_libs = {}

D = C.POINTER(C.c_double)
I32 = C.POINTER(C.c_int32)


class Params(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32),
                ("check_every", C.c_int32), ("sigma", C.c_double),
                ("restart", C.c_int32), ("fixed_iters", C.c_int32),
                ("admm_rho", C.c_double), ("abs_kkt", C.c_int32),
                ("coord_row", D), ("coord_col", D), ("sigma_update", C.c_int32),
                ("trace", D), ("trace_cap", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("primal_obj", C.c_double), ("dual_obj", C.c_double),
                ("kkt", C.c_double), ("res_dual", C.c_double),
                ("res_comp", C.c_double), ("res_primal", C.c_double),
                ("sigma", C.c_double), ("fp_res", C.c_double), ("kkt_abs", C.c_double),
                ("feaserr", C.c_double),
                ("iters", C.c_int32), ("restarts", C.c_int32),
                ("converged", C.c_int32), ("ntrace", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def lib(openmp=False):
    """The serial oracle, or its OpenMP build (same source, identical results;
    for multi-core timing)."""
    if openmp not in _libs:
        # HOT_ORACLE_LIB: a build of the same source to load instead (the
        # sanitizer test's AddressSanitizer build)
        path = os.environ.get("HOT_ORACLE_LIB") if not openmp else None
        L = C.CDLL(path or ensure_built(openmp))
        L.or_dims.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.or_cost.argtypes = [C.c_int32, C.c_int32, D]
        L.or_cost_xy.argtypes = [C.c_int32, C.c_int32, D, D, D]
        L.or_bvec.argtypes = [C.c_int32, C.c_int32, D, D, D]
        L.or_A.argtypes = [C.c_int32, C.c_int32, D, D]
        L.or_AT.argtypes = [C.c_int32, C.c_int32, D, D]
        L.or_solve_aat.argtypes = [C.c_int32, C.c_int32, D, D]
        L.or_kkt.argtypes = [C.c_int32, C.c_int32, D, D, D, D, D, C.POINTER(Result)]
        L.or_kkt_xy.argtypes = [C.c_int32, C.c_int32, D, D, D, D, D, D, D, C.POINTER(Result)]
        L.or_hot.argtypes = [C.c_int32, C.c_int32, D, D, C.POINTER(Params), D, D, D, D,
                             C.POINTER(Result)]
        L.or_hot.restype = C.c_int32
        L.or_recover.argtypes = [C.c_int32, C.c_int32, D, C.c_int64, I32, I32, D]
        L.or_recover.restype = C.c_int64
        L.or_repair.argtypes = [C.c_int32, C.c_int32, D, D, C.c_int64, C.c_int64, I32, I32, D]
        L.or_repair.restype = C.c_int64
        L.or_marginals.argtypes = [C.c_int32, C.c_int32, C.c_int64, I32, I32, D, D, D]
        L.or_simplex.argtypes = [C.c_int32, C.c_int32, D, D, D, D, D]
        L.or_simplex.restype = C.c_int32
        L.or_w2_1d.argtypes = [C.c_int32, D, D]
        L.or_w2_1d.restype = C.c_double
        _libs[openmp] = L
    return _libs[openmp]


def _d(a):
    return a.ctypes.data_as(D)


def _i(a):
    return a.ctypes.data_as(I32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def dims(m, n):
    N, M3 = C.c_int64(), C.c_int64()
    lib().or_dims(m, n, C.byref(N), C.byref(M3))
    return N.value, M3.value


def cost(m, n, coord_row=None, coord_col=None):
    """c of the reduced model; coord_row/coord_col: grid-line positions
    (length m / n), None for the uniform grid 0..m-1 / 0..n-1."""
    N, _ = dims(m, n)
    c = np.empty(N)
    if coord_row is None and coord_col is None:
        lib().or_cost(m, n, _d(c))
    else:
        u, v = _coords(m, n, coord_row, coord_col)
        lib().or_cost_xy(m, n, _dn(u), _dn(v), _d(c))
    return c


def _coords(m, n, coord_row, coord_col):
    u = None if coord_row is None else _f64(coord_row)
    v = None if coord_col is None else _f64(coord_col)
    if u is not None and u.shape != (m,):
        raise ValueError("coord_row must have length m")
    if v is not None and v.shape != (n,):
        raise ValueError("coord_col must have length n")
    return u, v


def _dn(a):
    return None if a is None else _d(a)


def bvec(mu1, mu2):
    mu1, mu2 = _f64(mu1), _f64(mu2)
    m, n = mu1.shape
    _, M3 = dims(m, n)
    b = np.empty(M3)
    lib().or_bvec(m, n, _d(mu1), _d(mu2), _d(b))
    return b


def A(m, n, x):
    x = _f64(x)
    _, M3 = dims(m, n)
    out = np.empty(M3)
    lib().or_A(m, n, _d(x), _d(out))
    return out


def AT(m, n, y):
    y = _f64(y)
    N, _ = dims(m, n)
    out = np.empty(N)
    lib().or_AT(m, n, _d(y), _d(out))
    return out


def solve_aat(m, n, R):
    R = _f64(R)
    y = np.empty_like(R)
    lib().or_solve_aat(m, n, _d(R), _d(y))
    return y


def kkt(mu1, mu2, x, y, z, coord_row=None, coord_col=None):
    mu1, mu2, x, y, z = map(_f64, (mu1, mu2, x, y, z))
    m, n = mu1.shape
    u, v = _coords(m, n, coord_row, coord_col)
    r = Result()
    lib().or_kkt_xy(m, n, _dn(u), _dn(v), _d(mu1), _d(mu2), _d(x), _d(y), _d(z), C.byref(r))
    return r.as_dict()


def hot(mu1, mu2, tol=1e-6, max_iter=100000, check_every=10, sigma=0.0,
        restart=True, fixed_iters=0, admm_rho=0.0, abs_kkt=False, coord_row=None,
        coord_col=None, sigma_update=False, threads=False, trace=0):
    """Run Algorithm 2; returns (xbar, ybar, zbar, s_state, result dict).
    threads: the OpenMP build (multi-core timing; identical results).
    trace > 0: the result dict also holds "trace", one row (it, k, r,
    restarted) per check, at most `trace` rows."""
    mu1, mu2 = _f64(mu1), _f64(mu2)
    m, n = mu1.shape
    N, M3 = dims(m, n)
    xb, zb, s = np.empty(N), np.empty(N), np.empty(N)
    yb = np.empty(M3)
    u, v = _coords(m, n, coord_row, coord_col)
    tr = np.zeros((max(int(trace), 1), 4))
    p = Params(tol, max_iter, check_every, sigma, 1 if restart else 0, fixed_iters, admm_rho,
               1 if abs_kkt else 0, _dn(u), _dn(v), 1 if sigma_update else 0,
               _d(tr) if trace > 0 else None, int(trace))
    r = Result()
    lib(threads).or_hot(m, n, _d(mu1), _d(mu2), C.byref(p), _d(xb), _d(yb), _d(zb), _d(s),
                        C.byref(r))
    out = r.as_dict()
    if trace > 0:
        out["trace"] = tr[:r.ntrace].copy()
    return xb, yb, zb, s, out


def recover(m, n, x, cap=None):
    """Algorithm 1 on max(x, 0); returns (src, dst, mass) arrays."""
    x = _f64(x)
    if cap is None:
        cap = m * n * (m + n)
    src = np.empty(cap, np.int32)
    dst = np.empty(cap, np.int32)
    mass = np.empty(cap)
    nnz = lib().or_recover(m, n, _d(x), cap, _i(src), _i(dst), _d(mass))
    if nnz > cap:
        return recover(m, n, x, cap=int(nnz))
    return src[:nnz].copy(), dst[:nnz].copy(), mass[:nnz].copy()


def repair(mu1, mu2, src, dst, mass):
    mu1, mu2 = _f64(mu1), _f64(mu2)
    m, n = mu1.shape
    M = m * n
    nnz = len(mass)
    cap = nnz + 2 * M
    s = np.empty(cap, np.int32); s[:nnz] = src
    d = np.empty(cap, np.int32); d[:nnz] = dst
    w = np.empty(cap); w[:nnz] = mass
    out = lib().or_repair(m, n, _d(mu1.ravel()), _d(mu2.ravel()), nnz, cap, _i(s), _i(d), _d(w))
    assert out <= cap
    return s[:out].copy(), d[:out].copy(), w[:out].copy()


def marginals(m, n, src, dst, mass):
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    mass = _f64(mass)
    row, col = np.empty(m * n), np.empty(m * n)
    lib().or_marginals(m, n, len(mass), _i(src), _i(dst), _d(mass), _d(row), _d(col))
    return row, col


def simplex(Amat, b, c):
    """min c^T x s.t. Amat x = b, x >= 0 (dense Bland two-phase)."""
    Amat, b, c = _f64(Amat), _f64(b), _f64(c)
    rows, cols = Amat.shape
    x = np.empty(cols)
    obj = C.c_double()
    st = lib().or_simplex(rows, cols, _d(Amat), _d(b), _d(c), _d(x), C.byref(obj))
    return st, x, obj.value


def w2_1d(a, b):
    a, b = _f64(a), _f64(b)
    return lib().or_w2_1d(len(a), _d(a), _d(b))
