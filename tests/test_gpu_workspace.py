"""Caller-owned device memory and general deflation bases on the GPU.

The library allocates no device memory: the plan lives in one workspace the
caller owns (a torch uint8 tensor here).  These tests call the C interface
directly where the binding would hide the protocol (a workspace that is too
small gives EWORKSPACE and the exact size), and check that deflation bases
with several entries per row -- which take the general code paths: the
multi-entry rows of Z and A Z, the separate Z^T pass when a row block reaches
more than 64 deflation columns, a compact A Z larger than its bound from
sizes -- solve the same trajectories as the oracle.
"""
import copy
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_1906_04051_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1906_04051_amd import gmres as G
    G.load_library()     # raises if the HIP library is missing: no fallback
    yield


def G():
    from paper_1906_04051_amd import gmres
    return gmres


def say(*a):
    print(*a, flush=True)


def assert_close(x, ref, tol, what=""):
    """Normwise and elementwise: ||x - ref|| <= tol ||ref|| and
    max|x - ref| <= tol max|ref|."""
    nr = float(np.linalg.norm(x - ref) / np.linalg.norm(ref))
    mx = float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))
    say(f"{what}: normwise {nr:.3e} elementwise {mx:.3e}")
    assert nr <= tol and mx <= tol, (what, nr, mx)


def _setup_raw(s, d, ws, nbytes, opts):
    lib = G().load_library()
    h = C.c_void_p()
    roff = np.array([0, s.n], np.int64)
    zoff = np.array([0, s.r], np.int64)
    st = lib.gmres_setup(C.byref(h), 1, roff.ctypes.data_as(C.POINTER(C.c_int64)),
                         zoff.ctypes.data_as(C.POINTER(C.c_int64)), G()._ptr(d["rowptr"]),
                         G()._ptr(d["colind"]), G()._ptr(d["vals"]), s.nnz, G()._ptr(d["z_rowptr"]),
                         G()._ptr(d["z_colind"]), G()._ptr(d["z_vals"]), len(s.z_colind), C.byref(opts), 0,
                         None if ws is None else G()._ptr(ws), nbytes, None)
    return st, h


def test_workspace_too_small_then_exact():
    lib = G().load_library()
    s = W.make_config(1, mesh=24)
    d = G().upload(s)
    opts = G().default_opts(m=20, rtol=0.0, max_iters=60)
    roff = np.array([0, s.n], np.int64)
    zoff = np.array([0, s.r], np.int64)
    est = lib.gmres_workspace_bytes(1, roff.ctypes.data_as(C.POINTER(C.c_int64)),
                                    zoff.ctypes.data_as(C.POINTER(C.c_int64)), s.nnz, len(s.z_colind),
                                    C.byref(opts), 0)
    say("estimate", est)
    assert est > 0
    # No workspace, then one of 4 KiB: EWORKSPACE with the size from sizes.
    for ws, nb in ((None, 0), (torch.empty(4096, dtype=torch.uint8, device="cuda"), 4096)):
        st, h = _setup_raw(s, d, ws, nb, opts)
        assert st == G().GMRES_EWORKSPACE and not h.value
        assert lib.gmres_workspace_required() == est
    # Misaligned workspace.
    big = torch.empty(est + 512, dtype=torch.uint8, device="cuda")
    st, h = _setup_raw(s, d, big[8:], est, opts)
    assert st == -1 and not h.value
    # The estimate is enough; the plan solves the oracle's trajectory.
    ws = torch.empty(est, dtype=torch.uint8, device="cuda")
    st, h = _setup_raw(s, d, ws, est, opts)
    assert st == 0 and h.value
    x = torch.empty_like(d["b"])
    info = G().GmresInfo()
    assert lib.gmres_solve(h, G()._ptr(d["b"]), None, G()._ptr(x), C.byref(info)) in (0, 1)
    lib.gmres_destroy(h)
    ref = oracle.gmres(s, 20, 0.0, 60)
    assert_close(x.cpu().numpy(), ref.x, 1e-8, "estimate-sized workspace")


def _heavy_z(s, R, every, per_row, seed):
    """Deflation basis with `per_row` entries in every `every`-th row (random
    columns of R) and none elsewhere: multi-entry rows of Z and of A Z; with
    R > 64 the row blocks of the SpMV reach more than 64 columns (separate
    Z^T pass)."""
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for i in range(0, s.n, every):
        c = np.sort(rng.choice(R, size=per_row, replace=False))
        rows += [i] * per_row
        cols += list(c)
        vals += list(rng.uniform(0.5, 1.5, per_row))
    t = copy.copy(s)
    t.r = R
    zrp = np.zeros(s.n + 1, np.int32)
    np.add.at(zrp, np.array(rows) + 1, 1)
    t.z_rowptr = np.cumsum(zrp).astype(np.int32)
    t.z_colind = np.array(cols, np.int32)
    t.z_vals = np.array(vals, np.float64)
    return t


def _check_solves(s, m, K, ortho, what):
    plan, d = G().plan_for(s, m=m, rtol=0.0, max_iters=K, ortho=ortho)
    x, info = plan.solve(d["b"])
    ref = oracle.gmres(s, m, 0.0, K)
    assert info["iters"] == ref.iters == K
    assert_close(x.cpu().numpy(), ref.x, 1e-8, f"fixed count, {what}")
    # To tolerance: same iteration count within one step, true residual, and
    # Z^T (b - A x) = 0 (the coarse correction).
    p2, d2 = G().plan_for(s, m=m, rtol=1e-8, max_iters=5000, ortho=ortho)
    x2, info2 = p2.solve(d2["b"])
    ref2 = oracle.gmres(s, m, 1e-8, 5000)
    say(f"{what}: iterations {info2['iters']} (oracle {ref2.iters})")
    assert abs(info2["iters"] - ref2.iters) <= 1 and info2["status_name"] == "OK"
    xg = x2.cpu().numpy()
    assert_close(xg, ref2.x, 1e-8, f"to tolerance, {what}")
    r = s.b - oracle.spmv(s.rowptr, s.colind, s.vals, xg)
    assert np.linalg.norm(r) <= 1e-8 * ref2.rho0 * (1 + 1e-6)
    Zd = W.dense_z(s)
    assert np.max(np.abs(Zd.T @ r)) <= 1e-10 * np.linalg.norm(s.b)
    return plan


@pytest.mark.parametrize("R,ortho", [(96, 1), (96, 0), (48, 1)])
def test_general_z_multi_entry_rows(R, ortho):
    s = _heavy_z(W.make_config(1, mesh=40), R=R, every=16, per_row=16, seed=R)
    _check_solves(s, 30, 90, ortho, f"R={R} ortho={ortho}")


def _dense_column_system():
    """Q1 system (25 x 25 nodes) plus a dense column c of A, and a deflation
    basis of 8 x 8 subdomain indicators whose row c holds all 64 columns; one
    node of 63 subdomains is left out so that z_nnz = n."""
    base = W.make_config(1, mesh=24)
    n, c = base.n, base.n // 2 + 7
    A = W.dense(base)
    rng = np.random.default_rng(11)
    A[:, c] += np.where(A[:, c] == 0, 1e-3 * rng.uniform(0.5, 1.0, n), 0.0)
    r, _, zc, _ = W.indicator_z(1, 24, 8)
    Z = np.zeros((n, r))
    Z[np.arange(n), zc] = 1.0
    Z[c, :] = np.where(Z[c, :] == 0, 0.25, 1.0)
    left_out = 0
    for col in range(r):
        if left_out == r - 1:
            break
        rows = [i for i in np.nonzero(zc == col)[0] if i != c]
        Z[rows[0], :] = 0.0
        left_out += 1
    return W.from_dense(A, base.b, Z=Z)


def test_workspace_bound_exceeded_then_exact():
    """Every row of A Z holds all 64 deflation columns (the dense column of A
    meets the dense row of Z), far beyond the bound nnz(A) * ceil(z_nnz / n)
    from sizes: setup with the estimate reports EWORKSPACE and the exact
    size, which is then enough (and 256 bytes less is not)."""
    s = _dense_column_system()
    n = s.n
    assert len(s.z_colind) == n
    lib = G().load_library()
    roff = np.array([0, n], np.int64)
    zoff = np.array([0, s.r], np.int64)
    opts = G().default_opts(m=30, rtol=0.0, max_iters=90)
    est = lib.gmres_workspace_bytes(1, roff.ctypes.data_as(C.POINTER(C.c_int64)),
                                    zoff.ctypes.data_as(C.POINTER(C.c_int64)), s.nnz, n, C.byref(opts), 0)
    d = G().upload(s)
    ws = torch.empty(est, dtype=torch.uint8, device="cuda")
    st, h = _setup_raw(s, d, ws, est, opts)
    need = lib.gmres_workspace_required()
    say(f"estimate {est}, exact {need}")
    assert st == G().GMRES_EWORKSPACE and not h.value and need > est
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    st, h = _setup_raw(s, d, ws, need - 256, opts)
    assert st == G().GMRES_EWORKSPACE and lib.gmres_workspace_required() == need
    st, h = _setup_raw(s, d, ws, need, opts)
    assert st == 0 and h.value
    lib.gmres_destroy(h)
    plan = _check_solves(s, 30, 90, 1, "dense column")
    assert plan.workspace_bytes == need


def test_invariant_subspace_z():
    rng = np.random.default_rng(6)
    n, r = 300, 12
    lam = np.concatenate([np.linspace(1e-3, 1e-2, r), np.linspace(1.0, 6.0, n - r)])
    S = rng.standard_normal((n, n)) / np.sqrt(n) + 3 * np.eye(n)
    A = S @ np.diag(lam) @ np.linalg.inv(S)
    Z = S[:, :r]                                  # A Z = Z diag(lam[:r]): an exact invariant subspace
    s = W.from_dense(A, rng.standard_normal(n), Z=Z)
    plan, d = G().plan_for(s, m=40, rtol=0.0, max_iters=80)
    x, info = plan.solve(d["b"])
    ref = oracle.gmres(s, 40, 0.0, 80)
    assert_close(x.cpu().numpy(), ref.x, 1e-8, "invariant subspace, fixed count")
    # The slow eigenvalues are deflated: the solve converges in far fewer
    # steps than without Z, to the dense solution.
    p2, d2 = G().plan_for(s, m=40, rtol=1e-10, max_iters=2000)
    x2, info2 = p2.solve(d2["b"])
    ref2 = oracle.gmres(s, 40, 1e-10, 2000)
    assert abs(info2["iters"] - ref2.iters) <= 1
    xd = np.linalg.solve(A, s.b)
    assert_close(x2.cpu().numpy(), xd, 1e-8, "invariant subspace vs dense solve")
    s0 = copy.copy(s)
    s0.r = 0
    s0.z_rowptr = np.zeros(n + 1, np.int32)
    s0.z_colind = np.zeros(0, np.int32)
    s0.z_vals = np.zeros(0)
    p3, d3 = G().plan_for(s0, m=40, rtol=1e-10, max_iters=2000)
    _, info3 = p3.solve(d3["b"])
    say(f"iterations with Z: {info2['iters']}, without: {info3['iters']}")
    assert info2["iters"] < info3["iters"]


def test_sliced_ell_budget_falls_back_to_csr():
    # One long row per 64-row slice: the sliced-ELL copy would pad every slice
    # to the long row (far beyond nnz + nnz/4), so the plan keeps CSR kernels.
    n, L = 64 * 40, 300
    rng = np.random.default_rng(3)
    rows, cols, vals = [], [], []
    for i in range(n):
        cs = {i}
        if i % 64 == 0:
            cs |= set(rng.choice(n, size=L, replace=False).tolist())
        cs = sorted(cs)
        for c in cs:
            rows.append(i)
            cols.append(c)
            vals.append(4.0 * L if c == i else rng.uniform(-1, 1))
    rp = np.zeros(n + 1, np.int32)
    np.add.at(rp, np.array(rows) + 1, 1)
    s = W.System(n=n, rowptr=np.cumsum(rp).astype(np.int32), colind=np.array(cols, np.int32),
                 vals=np.array(vals), b=rng.uniform(-1, 1, n), r=0,
                 z_rowptr=np.zeros(n + 1, np.int32), z_colind=np.zeros(0, np.int32), z_vals=np.zeros(0))
    plan, d = G().plan_for(s, m=20, rtol=1e-10, max_iters=400)
    with pytest.raises(G().GmresError):
        G().plan_for(s, m=20, spmv_lanes=-64)      # no sliced-ELL copy to force
    x, info = plan.solve(d["b"])
    ref = oracle.gmres(s, 20, 1e-10, 400)
    assert abs(info["iters"] - ref.iters) <= 1
    assert_close(x.cpu().numpy(), ref.x, 1e-8, "CSR fallback")
    y = plan.spmv(d["b"]).cpu().numpy()
    yr = oracle.spmv(s.rowptr, s.colind, s.vals, s.b)
    assert np.max(np.abs(y - yr)) <= 1e-12 * np.max(np.abs(yr))


def test_unsorted_or_duplicate_columns_rejected():
    s = W.make_config(1, mesh=8)
    k0 = s.rowptr[20]
    uns = copy.copy(s)
    uns.colind = s.colind.copy()
    uns.colind[k0], uns.colind[k0 + 1] = s.colind[k0 + 1], s.colind[k0]
    dup = copy.copy(s)
    dup.colind = s.colind.copy()
    dup.colind[k0 + 1] = s.colind[k0]
    zun = copy.copy(s)
    zun.z_rowptr = np.arange(0, 2 * s.n + 1, 2, dtype=np.int32)
    zun.z_colind = np.tile(np.array([1, 0], np.int32), s.n)
    zun.z_vals = np.ones(2 * s.n)
    for bad in (uns, dup, zun):
        with pytest.raises(G().GmresError) as e:
            G().plan_for(bad, m=5)
        assert e.value.status == -1
