"""Drives the library's host code through the C ABI without a GPU: option
and offset validation, the workspace layout in sizing mode for every plan
kind, the EWORKSPACE protocol of gmres_setup and the NULL-plan error paths.
Run by tests/test_sanitizers.py in a child process on a build whose host
code carries AddressSanitizer and UBSan (GMRES_LIB names it); exits non-zero
on the first wrong answer, and the sanitizers abort on the first error.
"""
import ctypes as C
import sys

import numpy as np

from paper_1906_04051_amd import gmres as G

EINVAL, EWORKSPACE = -1, -5


def i64p(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def opts(**kw):
    return G.default_opts(**kw)


def ws_bytes(lib, roff, zoff, nnz, znnz, o, adj=0):
    roff = np.asarray(roff, np.int64)
    zoff = None if zoff is None else np.asarray(zoff, np.int64)
    return lib.gmres_workspace_bytes(len(roff) - 1, i64p(roff), None if zoff is None else i64p(zoff),
                                     nnz, znnz, C.byref(o), adj)


def check(cond, what):
    if not cond:
        print("FAILED:", what, flush=True)
        sys.exit(1)


def main():
    lib = G.load_library()
    n, nnz = 10_000, 90_000
    valid = []
    for prec in (0, 1, 2):
        for ortho in (0, 1, 2):
            if ortho == 2 and prec != 0:
                continue
            for R in (0, 16, 256):
                for m in (1, 30, 96):
                    o = opts(m=m, precision=prec, ortho=ortho)
                    b = ws_bytes(lib, [0, n], [0, R], nnz, 4 * R + n, o)
                    check(b > 0, f"sizing prec {prec} ortho {ortho} R {R} m {m}")
                    valid.append(((prec, ortho, R, m), b))
    by = dict(valid)
    check(by[(0, 1, 16, 96)] > by[(0, 1, 16, 30)] > by[(0, 1, 16, 1)], "bytes grow with m")
    check(by[(0, 1, 256, 30)] > by[(0, 1, 0, 30)], "bytes grow with r")
    # Adjoint, adaptive deflation, batches of uneven systems.
    check(ws_bytes(lib, [0, n], [0, 8], nnz, n, opts(), adj=1) > by[(0, 1, 16, 30)] * 0 + 1, "adjoint")
    check(ws_bytes(lib, [0, n], None, nnz, 0, opts(adapt_rmax=20)) > 0, "adaptive")
    rng = np.random.default_rng(7)
    for nsys in (1, 2, 17, 512):
        sizes = rng.integers(1, 3000, nsys)
        roff = np.concatenate([[0], np.cumsum(sizes)])
        rs = np.minimum(rng.integers(0, 9, nsys), sizes)
        zoff = np.concatenate([[0], np.cumsum(rs)])
        check(ws_bytes(lib, roff, zoff, 9 * int(roff[-1]), int(roff[-1]), opts(m=40)) > 0, f"batch {nsys}")
    # Invalid arguments: size 0.
    bad = [
        ([0, n], [0, 4], opts(m=0)), ([0, n], [0, 4], opts(m=97)), ([0, n], [0, 4], opts(precision=3)),
        ([0, n], [0, 4], opts(ortho=3)), ([0, n], [0, 4], opts(ortho=2, precision=1)),
        ([0, n], [0, 4], opts(adapt_rmax=23)), ([0, n], [0, 4], opts(adapt_rmax=4)),
        ([0, n], [0, 4], opts(precision=2, inner_rtol=1.0)), ([0, n], [0, 4], opts(num_blocks=4096)),
        ([0, n], [0, 4], opts(spmv_lanes=3)), ([1, n], [0, 4], opts()), ([0, n], [1, 4], opts()),
        ([0, 5, 5], [0, 1, 1], opts()), ([0, n], [0, 257], opts()), ([0, 4], [0, 5], opts()),
        ([0, 1 << 31], [0, 4], opts()), ([0, n], [0, 4], opts(rtol=-1.0)),
    ]
    for roff, zoff, o in bad:
        check(ws_bytes(lib, roff, zoff, nnz, 100, o) == 0, f"rejects {roff} {zoff}")
    check(ws_bytes(lib, [0, n], [0, 4], -1, 100, opts()) == 0, "negative nnz")
    check(lib.gmres_workspace_bytes(0, None, None, nnz, 0, C.byref(opts()), 0) == 0, "nsys 0")
    check(lib.gmres_workspace_bytes(1, i64p(np.array([0, n], np.int64)), None, nnz, 0, None, 0) == 0,
          "NULL opts")
    # gmres_setup: without a workspace EWORKSPACE and the exact size; a
    # misaligned one EINVAL.  Neither dereferences the (dummy) array pointers.
    roff = np.array([0, n], np.int64)
    zoff = np.array([0, 16], np.int64)
    o = opts(m=30)
    need = ws_bytes(lib, roff, zoff, nnz, n, o)
    dummy = C.c_void_p(0x10000)
    h = C.c_void_p()
    st = lib.gmres_setup(C.byref(h), 1, i64p(roff), i64p(zoff), dummy, dummy, dummy, nnz, dummy, dummy,
                         dummy, n, C.byref(o), 0, None, 0, None)
    check(st == EWORKSPACE and not h.value, f"no workspace: {st}")
    check(lib.gmres_workspace_required() == need, "required == sizing")
    check(b"workspace" in lib.gmres_last_error(), "message")
    st = lib.gmres_setup(C.byref(h), 1, i64p(roff), i64p(zoff), dummy, dummy, dummy, nnz, dummy, dummy,
                         dummy, n, C.byref(o), 0, C.c_void_p(0x10008), need, None)
    check(st == EINVAL and not h.value, f"misaligned: {st}")
    st = lib.gmres_setup(C.byref(h), 1, i64p(roff), i64p(zoff), None, dummy, dummy, nnz, dummy, dummy,
                         dummy, n, C.byref(o), 0, None, 0, None)
    check(st == EINVAL, "NULL rowptr")
    check(lib.gmres_setup(None, 1, i64p(roff), i64p(zoff), dummy, dummy, dummy, nnz, dummy, dummy, dummy,
                          n, C.byref(o), 0, None, 0, None) == EINVAL, "NULL out")
    # NULL plans.
    info = G.GmresInfo()
    check(lib.gmres_solve(None, dummy, None, dummy, C.byref(info)) == EINVAL, "solve NULL")
    check(lib.gmres_solve_batched(None, dummy, None, dummy, None) == EINVAL, "batched NULL")
    check(lib.gmres_adjoint(None, dummy, dummy, dummy, dummy, None) == EINVAL, "adjoint NULL")
    check(lib.gmres_update_values(None, dummy) == EINVAL, "update NULL")
    check(lib.gmres_spmv(None, dummy, dummy) == EINVAL, "spmv NULL")
    check(lib.gmres_autotune(None, None) == EINVAL, "autotune NULL")
    check(lib.gmres_set_timing(None, 1) == EINVAL, "timing NULL")
    check(lib.gmres_block_workspace_bytes(None, 8) == 0, "block bytes NULL")
    check(lib.gmres_solve_block(None, 4, 8, dummy, None, dummy, None, 0, None) == EINVAL, "block NULL")
    check(lib.gmres_solve_block_noalloc(None, 4, 8, dummy, None, dummy, None) == EINVAL, "noalloc NULL")
    lib.gmres_destroy(None)
    print("host ABI driver: all checks passed", flush=True)


if __name__ == "__main__":
    main()
