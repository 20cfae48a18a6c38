"""Host-side checks of the C interface (no GPU needed): the library loads and
exports every function include/gmres.h declares; struct layouts of the binding
match the header's field order."""
import ctypes
import os
import re

import pytest

from paper_1906_04051_amd import gmres as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    hdr = open(os.path.join(ROOT, "include", "gmres.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(gmres_[a-z_]+)\s*\(", hdr)))


def test_header_declares_binding_exports():
    assert _declared() == sorted(G.EXPORTS)


@pytest.mark.parametrize("variant", ["release", "bounds-checking"])
def test_library_exports_every_declared_symbol(variant):
    from paper_1906_04051_amd import build as B
    path = G.LIB_PATH if variant == "release" else B.LIB_DEBUG
    if not os.path.exists(path):
        pytest.fail(f"{os.path.basename(path)} is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    for name in _declared():
        assert hasattr(lib, name), name


def test_struct_fields_follow_header_order():
    hdr = re.sub(r"/\*.*?\*/", "", open(os.path.join(ROOT, "include", "gmres.h")).read(), flags=re.S)
    for cname, pyst in (("gmres_opts", G.GmresOpts), ("gmres_info", G.GmresInfo)):
        body = re.search(r"typedef struct \{([^{}]*)\}\s*" + cname + ";", hdr).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        names = re.findall(r"(\w+)\s*(?:,|;)", body)
        assert names == [f for f, _ in pyst._fields_], (cname, names)


def test_default_opts_roundtrip():
    o = G.default_opts(m=50, rtol=1e-10, precision="mixed_f16")
    assert o.m == 50 and o.rtol == 1e-10 and o.precision == 2 and o.use_graph == 1
    with pytest.raises(TypeError):
        G.default_opts(bogus=1)


def _ws_bytes(n, nnz, r, zn, adj=0, **opts):
    import numpy as np
    lib = G.load_library()
    roff = np.array([0, n], np.int64)
    zoff = np.array([0, r], np.int64)
    o = G.default_opts(**opts)
    return lib.gmres_workspace_bytes(1, roff.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                     zoff.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), nnz, zn,
                                     ctypes.byref(o), adj)


def test_workspace_bytes_from_sizes():
    """The workspace size is a host computation (no GPU): it covers at least
    the basis, A's copy and Z's copy, grows with m, the adjoint and reduced
    precision, and is 0 for invalid arguments."""
    n, nnz, r = 1_050_625, 9_443_329, 64
    b50 = _ws_bytes(n, nnz, r, n, m=50)
    assert b50 >= 51 * n * 8 + 12 * nnz + 12 * n
    assert b50 % 256 == 0
    assert _ws_bytes(n, nnz, r, n, m=80) > b50
    assert _ws_bytes(n, nnz, r, n, adj=1, m=50) > b50 + 12 * nnz      # A^T copy
    assert _ws_bytes(n, nnz, r, n, m=50, precision="mixed_f16") > b50 + 4 * nnz
    assert _ws_bytes(n, nnz, r, n, m=0) == 0
    assert _ws_bytes(n, nnz, 300, n, m=30) == 0                        # r > 256
    assert _ws_bytes(n, 2**31, r, n, m=30) == 0                        # beyond int32 CSR
    # Same arguments, same answer.
    assert _ws_bytes(n, nnz, r, n, m=50) == b50
