"""Python binding of libgmres_mi355x.so (argument marshalling only).

Every step of the solve runs in the library's HIP kernels; this module only
passes torch CUDA tensors' device pointers and the stream to the C interface
declared in include/gmres.h.  There is no fallback: if the library is not
built, importing the binding's entry points raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgmres_mi355x.so")

GMRES_FP64, GMRES_MIXED_F32, GMRES_MIXED_F16 = 0, 1, 2
PRECISIONS = {"fp64": GMRES_FP64, "mixed_f32": GMRES_MIXED_F32, "mixed_f16": GMRES_MIXED_F16}
STATUS = {0: "OK", 1: "MAXITER", 2: "BREAKDOWN", 3: "STAGNATED", -1: "EINVAL", -2: "ESINGULAR",
          -3: "ENONFINITE", -4: "EDEVICE", -5: "EWORKSPACE"}
GMRES_EWORKSPACE = -5

# Every symbol include/gmres.h declares.
EXPORTS = ["gmres_default_opts", "gmres_workspace_bytes", "gmres_workspace_required", "gmres_setup",
           "gmres_solve", "gmres_solve_batched", "gmres_batched_attach", "gmres_block_workspace_bytes",
           "gmres_solve_block",
           "gmres_solve_block_noalloc",
           "gmres_adjoint", "gmres_update_values", "gmres_spmv", "gmres_history",
           "gmres_autotune", "gmres_set_timing", "gmres_kernel_times", "gmres_set_stream",
           "gmres_destroy", "gmres_last_error"]


class GmresOpts(C.Structure):
    _fields_ = [("m", C.c_int32), ("max_iters", C.c_int64), ("rtol", C.c_double),
                ("r0_norm_override", C.c_double), ("precision", C.c_int32),
                ("inner_rtol", C.c_double), ("max_refine", C.c_int32),
                ("inner_max_iters", C.c_int64), ("use_graph", C.c_int32),
                ("record_history", C.c_int32), ("spmv_lanes", C.c_int32),
                ("num_blocks", C.c_int32), ("batch_wg", C.c_int32), ("batch_lanes", C.c_int32),
                ("ortho", C.c_int32), ("adapt_rmax", C.c_int32)]


class GmresInfo(C.Structure):
    _fields_ = [("iters", C.c_int64), ("cycles", C.c_int32), ("refinements", C.c_int32),
                ("status", C.c_int32), ("defl_r", C.c_int32), ("rho0", C.c_double),
                ("rel_res", C.c_double), ("rel_res_true", C.c_double), ("solve_ms", C.c_double),
                ("mu", C.c_double)]

    def to_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["status_name"] = STATUS.get(self.status, str(self.status))
        return d


class GmresError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library():
    """Loads the built library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    # GMRES_LIB: another build of the same sources (the host-sanitizer or the
    # bounds-checking build); the release build otherwise.
    path = os.environ.get("GMRES_LIB") or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1906_04051_amd.build`")
    lib = C.CDLL(path)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    lib.gmres_default_opts.argtypes = [C.POINTER(GmresOpts)]
    lib.gmres_default_opts.restype = None
    sz = C.c_size_t
    lib.gmres_workspace_bytes.argtypes = [i32, C.POINTER(i64), C.POINTER(i64), i64, i64,
                                          C.POINTER(GmresOpts), i32]
    lib.gmres_workspace_bytes.restype = sz
    lib.gmres_workspace_required.argtypes = []
    lib.gmres_workspace_required.restype = sz
    lib.gmres_setup.argtypes = [C.POINTER(vp), i32, C.POINTER(i64), C.POINTER(i64), vp, vp, vp, i64,
                                vp, vp, vp, i64, C.POINTER(GmresOpts), i32, vp, sz, vp]
    lib.gmres_block_workspace_bytes.argtypes = [vp, i32]
    lib.gmres_block_workspace_bytes.restype = sz
    lib.gmres_solve.argtypes = [vp, vp, vp, vp, C.POINTER(GmresInfo)]
    lib.gmres_solve_batched.argtypes = [vp, vp, vp, vp, C.POINTER(GmresInfo)]
    lib.gmres_batched_attach.argtypes = [vp, i32, vp, i64]
    lib.gmres_adjoint.argtypes = [vp, vp, vp, vp, vp, C.POINTER(GmresInfo)]
    lib.gmres_solve_block.argtypes = [vp, i32, i32, vp, vp, vp, vp, sz, C.POINTER(GmresInfo)]
    lib.gmres_solve_block_noalloc.argtypes = [vp, i32, i32, vp, vp, vp, C.POINTER(GmresInfo)]
    lib.gmres_update_values.argtypes = [vp, vp]
    lib.gmres_spmv.argtypes = [vp, vp, vp]
    lib.gmres_history.argtypes = [vp, C.POINTER(dbl), i64]
    lib.gmres_history.restype = i64
    lib.gmres_autotune.argtypes = [vp, C.POINTER(i32)]
    lib.gmres_set_timing.argtypes = [vp, i32]
    lib.gmres_kernel_times.argtypes = [vp, C.POINTER(dbl)]
    lib.gmres_set_stream.argtypes = [vp, vp]
    lib.gmres_destroy.argtypes = [vp]
    lib.gmres_destroy.restype = None
    lib.gmres_last_error.argtypes = []
    lib.gmres_last_error.restype = C.c_char_p
    for name in ("gmres_setup", "gmres_solve", "gmres_solve_batched", "gmres_batched_attach", "gmres_solve_block",
                 "gmres_solve_block_noalloc", "gmres_adjoint",
                 "gmres_update_values", "gmres_spmv", "gmres_autotune", "gmres_set_timing",
                 "gmres_kernel_times", "gmres_set_stream"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _check(st: int, allow_positive: bool = True) -> int:
    if st < 0 or (st > 0 and not allow_positive):
        msg = load_library().gmres_last_error().decode(errors="replace")
        raise GmresError(st, msg)
    return st


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def default_opts(**kw) -> GmresOpts:
    o = GmresOpts()
    load_library().gmres_default_opts(C.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


class Plan:
    """A solver plan over torch CUDA tensors (int32 CSR, float64 values).

    rowptr/colind/vals: CSR of A (block-diagonal for batches, global indices);
    z_rowptr/z_colind/z_vals: CSR of Z (may be None when r = 0);
    sys_row_off / sys_zcol_off: numpy int64 block offsets (default: one system).
    Options are the fields of gmres_opts (m, max_iters, rtol, precision, ...).
    """

    def __init__(self, rowptr, colind, vals, z_rowptr=None, z_colind=None, z_vals=None,
                 r: int = 0, sys_row_off=None, sys_zcol_off=None, need_adjoint: bool = False,
                 stream=None, **opts):
        import torch
        lib = load_library()
        self._lib = lib
        n = rowptr.numel() - 1
        self.n = n
        self.nnz = colind.numel()
        if sys_row_off is None:
            sys_row_off = np.array([0, n], np.int64)
        if sys_zcol_off is None:
            sys_zcol_off = np.array([0, r], np.int64)
        self.row_off = np.ascontiguousarray(sys_row_off, np.int64)
        self.zcol_off = np.ascontiguousarray(sys_zcol_off, np.int64)
        self.nsys = len(self.row_off) - 1
        for t, dt in ((rowptr, torch.int32), (colind, torch.int32), (vals, torch.float64)):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise TypeError("rowptr/colind must be contiguous int32 CUDA tensors, vals float64")
        self.opts = default_opts(**opts)
        self._keep = (rowptr, colind, vals, z_rowptr, z_colind, z_vals)
        self._vals_version = 0
        znnz = 0 if z_colind is None else z_colind.numel()
        roff = self.row_off.ctypes.data_as(C.POINTER(C.c_int64))
        zoff = self.zcol_off.ctypes.data_as(C.POINTER(C.c_int64))
        adj = int(bool(need_adjoint))
        # The plan's device memory: one torch-owned workspace, sized from host
        # data; when the data-dependent parts exceed their bound, setup reports
        # the exact size and runs again with it.
        nbytes = lib.gmres_workspace_bytes(self.nsys, roff, zoff, self.nnz, znnz, C.byref(self.opts), adj)
        if nbytes == 0:
            raise GmresError(-1, "invalid plan sizes or options")
        h = C.c_void_p()
        for attempt in range(2):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=vals.device)
            st = lib.gmres_setup(C.byref(h), self.nsys, roff, zoff, _ptr(rowptr), _ptr(colind), _ptr(vals),
                                 self.nnz, _ptr(z_rowptr), _ptr(z_colind), _ptr(z_vals), znnz,
                                 C.byref(self.opts), adj, _ptr(self.workspace), nbytes,
                                 _stream_handle(stream))
            if st != GMRES_EWORKSPACE or attempt == 1:
                break
            need = lib.gmres_workspace_required()
            if need <= nbytes:
                break
            nbytes = need
        _check(st, allow_positive=False)
        self.workspace_bytes = nbytes
        self._block_ws = None
        self._subs = {}   # attached continuation plans by system (kept alive here)
        self._h = h
        self._device = vals.device

    def close(self):
        if getattr(self, "_h", None):
            self._lib.gmres_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        _check(self._lib.gmres_set_stream(self._h, _stream_handle(stream)))

    def _vec(self, t, name):
        import torch
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != self.n:
            raise TypeError(f"{name} must be a contiguous float64 CUDA tensor of {self.n} entries")
        return t

    def solve(self, b, x0=None, out=None):
        """Returns (x, info dict)."""
        import torch
        self._vec(b, "b")
        if x0 is not None:
            self._vec(x0, "x0")
        x = out if out is not None else torch.empty_like(b)
        info = GmresInfo()
        st = self._lib.gmres_solve(self._h, _ptr(b), _ptr(x0), _ptr(x), C.byref(info))
        _check(st)
        return x, info.to_dict()

    def solve_batched(self, b, x0=None, out=None):
        """Returns (x, list of per-system info dicts)."""
        import torch
        self._vec(b, "b")
        x = out if out is not None else torch.empty_like(b)
        infos = (GmresInfo * self.nsys)()
        st = self._lib.gmres_solve_batched(self._h, _ptr(b), _ptr(x0), _ptr(x), infos)
        _check(st)
        return x, [i.to_dict() for i in infos]

    def solve_block(self, B, m_block: int, X0=None, out=None):
        """Block GMRES(m_block) for the k columns of B (n x k, row-major,
        float64, on the plan's device).  Returns (X, info dict); iters are
        block steps."""
        import torch
        for t, name in ((B, "B"), (X0, "X0")):
            if t is None:
                continue
            if (t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.dim() != 2
                    or t.shape[0] != self.n):
                raise TypeError(f"{name} must be a contiguous float64 CUDA tensor of shape (n, k)")
        k = int(B.shape[1])
        if X0 is not None and tuple(X0.shape) != tuple(B.shape):
            raise ValueError("X0 must have the shape of B")
        X = out if out is not None else torch.empty_like(B)
        need = self._lib.gmres_block_workspace_bytes(self._h, int(m_block))
        if self._block_ws is None or self._block_ws.numel() < need:
            self._block_ws = torch.empty(max(need, 1), dtype=torch.uint8, device=B.device)
        info = GmresInfo()
        st = self._lib.gmres_solve_block(self._h, k, int(m_block), _ptr(B), _ptr(X0), _ptr(X),
                                         _ptr(self._block_ws), self._block_ws.numel(), C.byref(info))
        _check(st)
        return X, info.to_dict()

    def adjoint(self, x, grad_x):
        """Returns (grad_b, grad_vals, info dict)."""
        import torch
        gb = torch.empty_like(grad_x)
        gv = torch.empty(self.nnz, dtype=torch.float64, device=grad_x.device)
        info = GmresInfo()
        st = self._lib.gmres_adjoint(self._h, _ptr(x), _ptr(grad_x), _ptr(gb), _ptr(gv), C.byref(info))
        _check(st)
        return gb, gv, info.to_dict()

    def update_values(self, vals):
        self._keep = (self._keep[0], self._keep[1], vals) + self._keep[3:]
        self._vals_version += 1
        _check(self._lib.gmres_update_values(self._h, _ptr(vals)), allow_positive=False)
        self._subs = {}   # the library detached every continuation plan

    def attach(self, s: int, sub, steps: int):
        """Continuation plan for system s of this batched plan (None detaches):
        the system leaves the batched launch at the first restart after `steps`
        inner steps and goes on on `sub` (gmres_batched_attach)."""
        h = None if sub is None else sub._h
        _check(self._lib.gmres_batched_attach(self._h, int(s), h, int(steps) if sub is not None else 0),
               allow_positive=False)
        if sub is None:
            self._subs.pop(int(s), None)
        else:
            self._subs[int(s)] = sub

    def spmv(self, x):
        import torch
        y = torch.empty_like(x)
        _check(self._lib.gmres_spmv(self._h, _ptr(x), _ptr(y)))
        return y

    def history(self, cap: int = 1 << 24) -> np.ndarray:
        buf = np.zeros(cap, np.float64)
        k = self._lib.gmres_history(self._h, buf.ctypes.data_as(C.POINTER(C.c_double)), cap)
        if k < 0:
            raise RuntimeError("no history recorded (record_history=1 needed)")
        return buf[:k].copy()

    def autotune(self) -> dict:
        ch = (C.c_int32 * 4)()
        _check(self._lib.gmres_autotune(self._h, ch))
        return dict(spmv_lanes=ch[0], num_blocks=ch[1], batch_wg=ch[2], batch_lanes=ch[3])

    def set_timing(self, period):
        """Per-kernel timing of later solves: 0/False off, True/1 every restart
        cycle, k > 1 one cycle in k (the others replay the cycle graph)."""
        _check(self._lib.gmres_set_timing(self._h, int(period)))

    def kernel_times(self) -> dict:
        out = (C.c_double * 24)()
        _check(self._lib.gmres_kernel_times(self._h, out))
        names = ["spmv", "pass1", "pass2", "pass3", "pass1_lag", "block_dots", "block_gemm", "block_spmm"]
        return {nm: dict(launches=out[3 * k], ms=out[3 * k + 1], bytes=out[3 * k + 2])
                for k, nm in enumerate(names)}


def upload(sysm, device="cuda"):
    """numpy System (or Batch) arrays -> dict of CUDA tensors."""
    import torch

    def t(a, dt):
        return torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)
    return dict(rowptr=t(sysm.rowptr, torch.int32), colind=t(sysm.colind, torch.int32),
                vals=t(sysm.vals, torch.float64), b=t(sysm.b, torch.float64),
                z_rowptr=t(sysm.z_rowptr, torch.int32), z_colind=t(sysm.z_colind, torch.int32),
                z_vals=t(sysm.z_vals, torch.float64))


def plan_for(sysm, device="cuda", need_adjoint=False, **opts):
    """Plan for a workloads.System (single system) or workloads.Batch."""
    d = upload(sysm, device)
    if hasattr(sysm, "row_off"):
        plan = Plan(d["rowptr"], d["colind"], d["vals"], d["z_rowptr"], d["z_colind"], d["z_vals"],
                    sys_row_off=sysm.row_off, sys_zcol_off=sysm.zcol_off, need_adjoint=need_adjoint,
                    **opts)
    else:
        plan = Plan(d["rowptr"], d["colind"], d["vals"], d["z_rowptr"], d["z_colind"], d["z_vals"],
                    r=sysm.r, need_adjoint=need_adjoint, **opts)
    return plan, d


def attach_continuations(plan: Plan, batch, min_rows: int, work: float, device="cuda", **opts):
    """Builds single-system plans for the systems of `batch` (a
    workloads.Batch planned as `plan`) with at least min_rows rows and
    attaches them with a step limit of `work` row-steps, rounded up to whole
    cycles: steps_s = m * ceil(work / (rows_s * m)).  opts: the batch's plan
    options (m, rtol, max_iters, ...).  Returns {system: plan}."""
    m = int(plan.opts.m)
    subs = {}
    rows = np.diff(batch.row_off)
    for s in np.nonzero(rows >= min_rows)[0]:
        s = int(s)
        sub, _ = plan_for(batch.systems[s], device=device, **opts)
        steps = m * max(1, int(np.ceil(work / (float(rows[s]) * m))))
        plan.attach(s, sub, steps)
        subs[s] = sub
    return subs


class DeflatedGMRES:
    """torch.autograd.Function: x = A(vals)^{-1} b through the plan's solver,
    with the adjoint solve in backward (dL/db = lambda, dL/dvals = -lambda_i x_j)."""

    @staticmethod
    def apply(vals, b, plan: Plan):
        return _fn().apply(vals, b, plan)


_FN = None


def _fn():
    global _FN
    if _FN is not None:
        return _FN
    import torch

    class _DeflatedGMRES(torch.autograd.Function):
        @staticmethod
        def forward(ctx, vals, b, plan):
            v = vals.detach().contiguous()
            plan.update_values(v)
            x, info = plan.solve(b.detach().contiguous())
            ctx.plan = plan
            ctx.info = info
            ctx.version = plan._vals_version
            ctx.save_for_backward(x, v)
            return x

        @staticmethod
        def backward(ctx, gx):
            x, v = ctx.saved_tensors
            # The adjoint runs on the plan's current A^T: another forward (or
            # update_values) on the same plan since this forward replaced the
            # values, so put this forward's values back first.
            if ctx.plan._vals_version != ctx.version:
                ctx.plan.update_values(v)
            gb, gv, _ = ctx.plan.adjoint(x, gx.contiguous())
            return gv, gb, None

    _FN = _DeflatedGMRES
    return _FN
