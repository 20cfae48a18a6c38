"""gmres_solve_block_noalloc: the block solve with its scratch in the
library's static device array, for callers that cannot allocate.  Checked
against gmres_solve_block (scratch in a caller workspace) on the same plan
and inputs, on two calls in a row where the second is smaller (fewer rows,
fewer right-hand sides, shorter cycles): both run the same kernels, so the
results must agree to the FP64 gate (they are in fact bitwise equal)."""
import copy
import ctypes as C

import numpy as np
import pytest

from paper_1906_04051_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")
    from paper_1906_04051_amd import gmres as G
    G.load_library()
    yield


def _plain(mesh):
    s = copy.copy(W.make_config(1, mesh=mesh))
    s.r = 0
    s.z_rowptr = np.zeros(s.n + 1, np.int32)
    s.z_colind = np.zeros(0, np.int32)
    s.z_vals = np.zeros(0)
    return s


def _relF(a, b):
    d = a - b
    return max(float(np.linalg.norm(d) / np.linalg.norm(b)), float(np.abs(d).max() / np.abs(b).max()))


def test_noalloc_block_matches_workspace_block_twice():
    from paper_1906_04051_amd import gmres as G
    lib = G.load_library()
    for mesh, k, mb, seed in ((64, 8, 4, 1), (32, 3, 3, 2)):       # second call: smaller input
        s = _plain(mesh)
        plan, d = G.plan_for(s, m=30, rtol=1e-8, max_iters=3000)
        B = torch.from_numpy(np.random.default_rng(seed).standard_normal((s.n, k))).cuda()
        X_ws, info_ws = plan.solve_block(B, mb)
        X_st = torch.full_like(B, np.nan)
        info = G.GmresInfo()
        print(f"noalloc: n={s.n} k={k} m_block={mb}", flush=True)
        st = lib.gmres_solve_block_noalloc(plan._h, k, mb, G._ptr(B), None, G._ptr(X_st), C.byref(info))
        G._check(st)
        torch.cuda.synchronize()
        a, b = X_st.cpu().numpy(), X_ws.cpu().numpy()
        e = _relF(a, b)
        print(f"  steps {info.iters} (workspace {info_ws['iters']}), rel diff {e:.3e}, "
              f"bitwise {np.array_equal(a, b)}", flush=True)
        assert info.status == 0 and info_ws["status_name"] == "OK"
        assert info.iters == info_ws["iters"]
        assert e <= 1e-8
        assert abs(info.rel_res_true - info_ws["rel_res_true"]) <= 1e-12
        plan.close()


def test_noalloc_rejects_more_than_the_static_scratch():
    from paper_1906_04051_amd import gmres as G
    lib = G.load_library()
    s = _plain(320)                                     # 103,041 rows
    plan, d = G.plan_for(s, m=30, rtol=1e-8, max_iters=10)
    need = lib.gmres_block_workspace_bytes(plan._h, 4)
    assert need > (64 << 20)
    B = torch.ones((s.n, 2), dtype=torch.float64, device="cuda")
    X = torch.empty_like(B)
    info = G.GmresInfo()
    st = lib.gmres_solve_block_noalloc(plan._h, 2, 4, G._ptr(B), None, G._ptr(X), C.byref(info))
    assert st == -1
    assert b"static scratch" in lib.gmres_last_error()
    plan.close()
