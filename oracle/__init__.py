"""Plain FP64 CPU oracle for deflated restarted GMRES(m) (ctypes binding).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU solver never imports this
package and this package never imports the solver; both take inputs from
``paper_1906_04051_amd.workloads`` only.

Every numerical routine lives in ``oracle.c``, ``dgmres.c`` and ``bgmres.c``
(plain C, FP64, ``-ffp-contract=off``).  This module only marshals numpy arrays.

Parity pins: see ``tests/test_oracle.py``.  Functions without an independent
pin: none (the dense adjoint in ``dense_adjoint`` is itself the pin of the
adjoint path).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SRC_D = os.path.join(_HERE, "dgmres.c")
_SRC_B = os.path.join(_HERE, "bgmres.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

STATUS = {0: "OK", 1: "MAXITER", 2: "BREAKDOWN", -1: "EINVAL", -2: "ESINGULAR", -3: "ENONFINITE",
          -6: "ENOMEM"}


def build() -> str:
    """Compile liboracle.so (gcc, -O2, no FP contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           _SRC, _SRC_D, _SRC_B, "-o", _LIB + ".tmp", "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    override = os.environ.get("ORACLE_LIB")   # another build of the same sources (sanitizers)
    if override:
        lib = C.CDLL(override)
    else:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
    i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
    i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
    f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    vp = C.c_void_p
    lib.oracle_spmv.argtypes = [C.c_int64, i32p, i32p, f64p, f64p, f64p]
    lib.oracle_spmv.restype = None
    lib.oracle_dot.argtypes = [C.c_int64, f64p, f64p]
    lib.oracle_dot.restype = C.c_double
    lib.oracle_lu_factor.argtypes = [C.c_int32, f64p, i32p]
    lib.oracle_lu_factor.restype = C.c_int
    lib.oracle_lu_solve.argtypes = [C.c_int32, f64p, i32p, f64p]
    lib.oracle_lu_solve.restype = None
    lib.oracle_apply_projector.argtypes = [C.c_int64, i32p, i32p, f64p, C.c_int32, i32p, i32p, vp, f64p, f64p]
    lib.oracle_apply_projector.restype = C.c_int
    lib.oracle_gmres.argtypes = [C.c_int64, i32p, i32p, f64p, f64p, vp,
                                 C.c_int32, i32p, i32p, vp,
                                 C.c_int32, C.c_int64, C.c_double, C.c_double,
                                 f64p, i64p, f64p, vp, vp, vp]
    lib.oracle_gmres.restype = C.c_int
    lib.oracle_csr_transpose.argtypes = [C.c_int64, i32p, i32p, f64p, i32p, i32p, f64p]
    lib.oracle_csr_transpose.restype = None
    lib.oracle_grad_vals.argtypes = [C.c_int64, i32p, i32p, f64p, f64p, f64p]
    lib.oracle_grad_vals.restype = None
    lib.oracle_dgmres.argtypes = [C.c_int64, i32p, i32p, f64p, f64p, vp, C.c_int32, C.c_int64,
                                  C.c_double, C.c_int32, f64p, i64p, f64p, vp, vp, vp]
    lib.oracle_dgmres.restype = C.c_int
    lib.oracle_bgmres.argtypes = [C.c_int64, i32p, i32p, f64p, C.c_int32, vp, vp, vp, C.c_int32, f64p, vp,
                                  C.c_int32, C.c_int64, C.c_double, f64p, i64p, f64p, vp]
    lib.oracle_bgmres.restype = C.c_int
    lib.oracle_power_iteration.argtypes = [C.c_int32, f64p, f64p]
    lib.oracle_power_iteration.restype = C.c_double
    lib.oracle_inverse_iteration.argtypes = [C.c_int32, f64p, f64p]
    lib.oracle_inverse_iteration.restype = C.c_int
    lib.oracle_apply_minv.argtypes = [C.c_int64, C.c_int32, f64p, f64p, C.c_double, f64p, f64p]
    lib.oracle_apply_minv.restype = C.c_int
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def spmv(rowptr, colind, vals, x):
    lib = _load()
    n = len(rowptr) - 1
    y = np.empty(n, np.float64)
    lib.oracle_spmv(n, _i32(rowptr), _i32(colind), _f64(vals), _f64(x), y)
    return y


def dot(a, b):
    return _load().oracle_dot(len(a), _f64(a), _f64(b))


def lu_factor(E):
    E = _f64(E).copy()
    r = E.shape[0]
    piv = np.zeros(r, np.int32)
    st = _load().oracle_lu_factor(r, E, piv)
    return st, E, piv


def lu_solve(LU, piv, t):
    x = _f64(t).copy()
    _load().oracle_lu_solve(LU.shape[0], _f64(LU), _i32(piv), x)
    return x


def apply_projector(sysm, y):
    """w = P y with P = I - A Z E^{-1} Z^T for System `sysm`."""
    lib = _load()
    w = np.empty(sysm.n, np.float64)
    zv = _f64(sysm.z_vals)
    st = lib.oracle_apply_projector(sysm.n, _i32(sysm.rowptr), _i32(sysm.colind), _f64(sysm.vals),
                                    sysm.r, _i32(sysm.z_rowptr), _i32(sysm.z_colind), _ptr(zv),
                                    _f64(y), w)
    if st != 0:
        raise RuntimeError("oracle_apply_projector: " + STATUS.get(st, str(st)))
    return w


class Result(dict):
    __getattr__ = dict.__getitem__


def gmres(sysm, m: int, rtol: float, max_iters: int, x0=None, b=None, r0_norm_override: float = 0.0,
          history: bool = False, first_cycle: bool = False, vals=None) -> Result:
    """Deflated GMRES(m) on System `sysm` (A, Z from it; b defaults to sysm.b)."""
    lib = _load()
    n = sysm.n
    b = _f64(sysm.b if b is None else b)
    vals = _f64(sysm.vals if vals is None else vals)
    x0a = None if x0 is None else _f64(x0)
    x = np.zeros(n, np.float64)
    info_i = np.zeros(3, np.int64)
    info_d = np.zeros(3, np.float64)
    hist = np.zeros(max(max_iters, 1), np.float64) if history else None
    V0 = np.zeros((m + 1, n), np.float64) if first_cycle else None
    H0 = np.zeros((m + 1, m), np.float64) if first_cycle else None
    zv = _f64(sysm.z_vals)
    st = lib.oracle_gmres(n, _i32(sysm.rowptr), _i32(sysm.colind), vals, b, _ptr(x0a),
                          sysm.r, _i32(sysm.z_rowptr), _i32(sysm.z_colind), _ptr(zv),
                          m, max_iters, rtol, r0_norm_override,
                          x, info_i, info_d, _ptr(hist), _ptr(V0), _ptr(H0))
    res = Result(x=x, iters=int(info_i[0]), cycles=int(info_i[1]), status=int(st),
                 status_name=STATUS.get(int(st), str(st)), rho0=float(info_d[0]),
                 rel_res_deflated=float(info_d[1]), rel_res_true=float(info_d[2]))
    if history:
        res["history"] = hist[:res.iters].copy()
    if first_cycle:
        res["V0"] = V0
        res["H0"] = H0
    return res


def dgmres(sysm, m: int, rtol: float, max_iters: int, rmax: int = 20, x0=None, b=None,
           history: bool = False, export: bool = False) -> Result:
    """GMRES(m) right-preconditioned by the paper's adaptive spectral deflation
    (Sec. 3.3; readings in dgmres.c).  Uses A and b of System `sysm` (its Z is
    ignored).  rmax = 0 gives plain GMRES(m)."""
    lib = _load()
    n = sysm.n
    b = _f64(sysm.b if b is None else b)
    x0a = None if x0 is None else _f64(x0)
    x = np.zeros(n, np.float64)
    info_i = np.zeros(4, np.int64)
    info_d = np.zeros(4, np.float64)
    hist = np.zeros(max(max_iters, 1), np.float64) if history else None
    U = np.zeros((max(rmax, 1), n), np.float64) if export else None
    T = np.zeros((max(rmax, 1), max(rmax, 1)), np.float64) if export else None
    st = lib.oracle_dgmres(n, _i32(sysm.rowptr), _i32(sysm.colind), _f64(sysm.vals), b, _ptr(x0a),
                           m, max_iters, rtol, rmax, x, info_i, info_d, _ptr(hist), _ptr(U), _ptr(T))
    res = Result(x=x, iters=int(info_i[0]), cycles=int(info_i[1]), status=int(st),
                 status_name=STATUS.get(int(st), str(st)), r=int(info_i[3]), rho0=float(info_d[0]),
                 rel_res=float(info_d[1]), rel_res_true=float(info_d[2]), mu=float(info_d[3]))
    if history:
        res["history"] = hist[:res.iters].copy()
    if export:
        rr = res.r
        res["U"] = U[:rr].copy()
        res["T"] = T.ravel()[:rr * rr].reshape(rr, rr).copy()
    return res


def bgmres(rowptr, colind, vals, B, m: int, rtol: float, max_steps: int, X0=None,
           history: bool = False, z=None) -> Result:
    """Block GMRES(m) for A X = B with the k columns of B (n x k) as right-hand
    sides (definition and readings in bgmres.c).  Iterations are block steps.
    z: None, or (r, z_rowptr, z_colind, z_vals) of a deflation basis Z (n x r,
    CSR): every column deflated as in the single-vector method."""
    lib = _load()
    B = np.ascontiguousarray(B, dtype=np.float64)
    n, k = B.shape
    X = np.zeros((n, k), np.float64)
    X0a = None if X0 is None else np.ascontiguousarray(X0, dtype=np.float64)
    info_i = np.zeros(4, np.int64)
    info_d = np.zeros(4, np.float64)
    hist = np.zeros(max(max_steps, 1), np.float64) if history else None
    if z is None or int(z[0]) == 0:
        zr, zrp, zci, zvv = 0, None, None, None
    else:
        zr, zrp, zci, zvv = int(z[0]), _i32(z[1]), _i32(z[2]), _f64(z[3])
    st = lib.oracle_bgmres(n, _i32(rowptr), _i32(colind), _f64(vals), zr, _ptr(zrp), _ptr(zci), _ptr(zvv),
                           k, B, _ptr(X0a), m, max_steps, rtol, X, info_i, info_d, _ptr(hist))
    res = Result(x=X, iters=int(info_i[0]), cycles=int(info_i[1]), status=int(st),
                 status_name=STATUS.get(int(st), str(st)), rho0_max=float(info_d[0]),
                 rel_res_est=float(info_d[1]), rel_res_true=float(info_d[2]))
    if history:
        res["history"] = hist[:res.iters].copy()
    return res


def apply_minv(U, T, mu, v):
    """M^{-1} v = v + U (|mu| T^{-1} - I) U^T v for U given as r x n rows."""
    U = _f64(U)
    r, n = U.shape
    out = np.zeros(n, np.float64)
    st = _load().oracle_apply_minv(n, r, U, _f64(T), float(mu), _f64(v), out)
    if st != 0:
        raise RuntimeError("oracle_apply_minv: " + STATUS.get(st, str(st)))
    return out


def power_iteration(M):
    """(|mu|, z): the oracle's fixed-count power iteration on a small matrix."""
    M = _f64(M)
    z = np.zeros(M.shape[0], np.float64)
    mu = _load().oracle_power_iteration(M.shape[0], M, z)
    return mu, z


def inverse_iteration(M):
    """(status, z): the oracle's fixed-count inverse iteration on a small matrix."""
    M = _f64(M)
    z = np.zeros(M.shape[0], np.float64)
    st = _load().oracle_inverse_iteration(M.shape[0], M, z)
    return st, z


def csr_transpose(rowptr, colind, vals):
    lib = _load()
    n = len(rowptr) - 1
    nnz = int(rowptr[-1])
    trp = np.zeros(n + 1, np.int32)
    tci = np.zeros(nnz, np.int32)
    tv = np.zeros(nnz, np.float64)
    lib.oracle_csr_transpose(n, _i32(rowptr), _i32(colind), _f64(vals), trp, tci, tv)
    return trp, tci, tv


def grad_vals(rowptr, colind, lam, x):
    lib = _load()
    n = len(rowptr) - 1
    g = np.zeros(int(rowptr[-1]), np.float64)
    lib.oracle_grad_vals(n, _i32(rowptr), _i32(colind), _f64(lam), _f64(x), g)
    return g


def adjoint(sysm, x, grad_x, m: int, rtol: float, max_iters: int, vals=None):
    """Adjoint of x = A^{-1} b: solve A^T lam = grad_x with the same deflated
    GMRES(m) on the transposed matrix (same Z), then
    dL/db = lam and dL/dA_ij = -lam_i x_j on A's pattern."""
    import copy
    vals = sysm.vals if vals is None else vals
    trp, tci, tv = csr_transpose(sysm.rowptr, sysm.colind, vals)
    st = copy.copy(sysm)
    st.rowptr, st.colind, st.vals = trp, tci, tv
    res = gmres(st, m, rtol, max_iters, b=grad_x)
    lam = res.x
    g = grad_vals(sysm.rowptr, sysm.colind, lam, x)
    res["grad_b"] = lam
    res["grad_vals"] = g
    return res
