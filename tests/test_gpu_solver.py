"""GPU parity of the HIP deflated GMRES(m) path against the FP64 CPU oracle.

Every test calls the library through its C interface (ctypes binding) on
seeded synthetic FEM systems and compares with the oracle on the same inputs.
Gates (the target accuracy of the FP64 path is ||x - x_ref|| / ||x_ref|| <= 1e-8):
  * SpMV: exact on integer-valued data; elementwise |y - y_ref| <= c eps (|A||x|)
    on FEM data (rows cancel, so a relative test per entry would be wrong);
  * trajectory parity: fixed-count runs (rtol = 0, the paper's protocol of
    Sec. 4) over the same Krylov spaces -> ||x - x_ora|| / ||x_ora|| <= 1e-8;
  * to-tolerance parity: iteration counts within one step, same 1e-8 gate,
    true residual (recomputed in FP64 on the host) <= rtol.
"""
import copy

import numpy as np
import pytest

import oracle
from paper_1906_04051_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps


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


def host_residual(s, x, b=None):
    b = s.b if b is None else b
    return b - oracle.spmv(s.rowptr, s.colind, s.vals, x)


def rel(a, b):
    """Larger of the normwise ||a - b|| / ||b|| and the elementwise
    max|a - b| / max|b| relative differences (a gate on it bounds both)."""
    d = np.asarray(a) - np.asarray(b)
    nb = max(float(np.linalg.norm(b)), 1e-300)
    mb = max(float(np.max(np.abs(b))), 1e-300) if np.size(b) else 1.0
    return max(float(np.linalg.norm(d)) / nb, float(np.max(np.abs(d), initial=0.0)) / mb)


def no_defl(s):
    s = copy.copy(s)
    s.r = 0
    s.z_rowptr = np.zeros(s.n + 1, np.int32)
    s.z_colind = np.zeros(0, np.int32)
    s.z_vals = np.zeros(0)
    return s


# ---------------------------------------------------------------- SpMV

@pytest.mark.parametrize("maxlen", [10, 30, 40, 130])
def test_spmv_integer_exact_all_lane_counts(maxlen):
    """Random row lengths (empty rows included): the sliced-ELL copy sorts the
    rows of each 256-row block by length, and the kernel instance follows the
    longest row (<= 12, <= 32, any)."""
    rng = np.random.default_rng(11 + maxlen)
    n = 3001
    dens = rng.random((n,)) * maxlen
    rows, cols, vals = [], [], []
    for i in range(n):
        k = int(dens[i]) + (1 if i % 7 else 0)
        c = np.unique(rng.integers(0, n, size=k))
        rows += [i] * len(c)
        cols += list(c)
        vals += list(rng.integers(-8, 9, size=len(c)).astype(float))
    rowptr = np.zeros(n + 1, np.int32)
    np.add.at(rowptr, np.array(rows) + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    s = W.System(n=n, rowptr=rowptr, colind=np.array(cols, np.int32), vals=np.array(vals),
                 b=np.zeros(n), r=0, z_rowptr=np.zeros(n + 1, np.int32),
                 z_colind=np.zeros(0, np.int32), z_vals=np.zeros(0))
    x = rng.integers(-4, 5, size=n).astype(np.float64)
    ref = oracle.spmv(s.rowptr, s.colind, s.vals, x)
    for L in (1, 2, 4, 8, 16, 32, 64, -64, -128, -256):
        say("spmv integer maxlen", maxlen, "L =", L)
        plan, d = G().plan_for(s, m=4, spmv_lanes=L)
        y = plan.spmv(torch.from_numpy(x).cuda()).cpu().numpy()
        assert np.array_equal(y, ref), L
        plan.close()


def test_spmv_far_columns_without_sliced_ell():
    """Column offsets |col - row| > 32767 do not fit the 16-bit sliced-ELL
    copy: the plan falls back to the CSR kernels (exact on integer data) and an
    explicit request for the sliced-ELL kernel is rejected."""
    n = 70001
    rows = np.concatenate([np.arange(n), np.arange(1, n), [0, n - 1]])
    cols = np.concatenate([np.arange(n), np.arange(n - 1), [n - 1, 0]])
    vals = np.concatenate([np.full(n, 4.0), np.full(n - 1, -1.0), [2.0, -3.0]])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(n + 1, np.int32)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    s = W.System(n=n, rowptr=rowptr, colind=cols.astype(np.int32), vals=vals.astype(np.float64),
                 b=np.zeros(n), r=0, z_rowptr=np.zeros(n + 1, np.int32),
                 z_colind=np.zeros(0, np.int32), z_vals=np.zeros(0))
    x = np.random.default_rng(13).integers(-4, 5, size=n).astype(np.float64)
    ref = oracle.spmv(s.rowptr, s.colind, s.vals, x)
    plan, d = G().plan_for(s, m=4)
    assert np.array_equal(plan.spmv(torch.from_numpy(x).cuda()).cpu().numpy(), ref)
    plan.close()
    with pytest.raises(G().GmresError) as e:
        G().plan_for(s, m=4, spmv_lanes=-64)
    assert e.value.status == -1


@pytest.mark.parametrize("cfg,mesh", [(1, 64), (2, 96), (3, 24)])
def test_spmv_fem_elementwise_bound(cfg, mesh):
    s = W.make_config(cfg, mesh=mesh)
    rng = np.random.default_rng(12)
    x = rng.standard_normal(s.n)
    ref = oracle.spmv(s.rowptr, s.colind, s.vals, x)
    absax = oracle.spmv(s.rowptr, s.colind, np.abs(s.vals), np.abs(x))
    cmax = int(np.diff(s.rowptr).max())
    plan, d = G().plan_for(s, m=4)
    y = plan.spmv(torch.from_numpy(x).cuda()).cpu().numpy()
    assert np.all(np.abs(y - ref) <= cmax * EPS * absax + 1e-300)


# ------------------------------------------------------ single system FP64

def _gpu_solve(s, b=None, x0=None, **opts):
    plan, d = G().plan_for(s, **opts)
    bb = d["b"] if b is None else torch.from_numpy(np.ascontiguousarray(b)).cuda()
    x0t = None if x0 is None else torch.from_numpy(np.ascontiguousarray(x0)).cuda()
    x, info = plan.solve(bb, x0t)
    out = x.cpu().numpy()
    return out, info, plan


@pytest.mark.parametrize("ortho", [0, 1, 2])
def test_config1_trajectory_parity(ortho):
    s = W.make_config(1)
    ref_tol = oracle.gmres(s, 30, 1e-8, 2000)
    K = ref_tol.iters
    ref = oracle.gmres(s, 30, 0.0, K)
    say("config 1 fixed-count K =", K, "ortho", ortho)
    x, info, _ = _gpu_solve(s, m=30, rtol=0.0, max_iters=K, ortho=ortho)
    assert info["iters"] == K and info["status_name"] == "MAXITER"
    assert rel(x, ref.x) <= 1e-8
    assert abs(info["rel_res"] - ref.rel_res_deflated) <= 1e-6 * ref.rel_res_deflated + 1e-14


@pytest.mark.parametrize("use_graph,ortho", [(1, 1), (0, 1), (1, 0), (1, 2), (0, 2)])
def test_config1_to_tolerance(use_graph, ortho):
    s = W.make_config(1)
    ref = oracle.gmres(s, 30, 1e-8, 2000)
    x, info, _ = _gpu_solve(s, m=30, rtol=1e-8, max_iters=2000, use_graph=use_graph, ortho=ortho)
    say("config 1 iters gpu/oracle", info["iters"], ref.iters)
    assert info["status_name"] == "OK"
    assert abs(info["iters"] - ref.iters) <= 1
    assert rel(x, ref.x) <= 1e-8
    r = host_residual(s, x)
    assert np.linalg.norm(r) <= 1e-8 * ref.rho0 * (1 + 1e-9)
    assert abs(info["rel_res_true"] - np.linalg.norm(r) / ref.rho0) <= 1e-12


@pytest.mark.parametrize("ortho", [0, 1, 2])
def test_residual_history_matches_oracle(ortho):
    s = W.make_config(1, mesh=32)
    ref = oracle.gmres(s, 30, 1e-8, 2000, history=True)
    plan, d = G().plan_for(s, m=30, rtol=1e-8, max_iters=2000, record_history=1, ortho=ortho)
    x, info = plan.solve(d["b"])
    h = plan.history()
    k = min(len(h), len(ref.history))
    assert k >= ref.iters - 1
    relerr = np.abs(h[:k] - ref.history[:k]) / ref.history[:k]
    assert relerr.max() <= 1e-6


@pytest.mark.parametrize("ortho", [0, 1, 2])
@pytest.mark.parametrize("mesh,s_sub,m", [(5, 2, 7), (13, 3, 20), (37, 4, 30), (91, 8, 50), (150, 5, 80)])
def test_ragged_sizes_and_restart_lengths(mesh, s_sub, m, ortho):
    # n = (mesh+1)^2 is never a multiple of the 256-thread workgroup.
    sysm = W.convection_diffusion_lognormal(mesh, beta=(30.0, 5.0), sigma=1.0, s=s_sub,
                                            seed_seq=W.config_seed(100 + mesh))
    ref_tol = oracle.gmres(sysm, m, 1e-9, 5000)
    K = min(ref_tol.iters, 3 * m + 5)
    ref = oracle.gmres(sysm, m, 0.0, K)
    say("ragged mesh", mesh, "n", sysm.n, "m", m, "K", K, "ortho", ortho)
    x, info, _ = _gpu_solve(sysm, m=m, rtol=0.0, max_iters=K, ortho=ortho)
    assert info["iters"] == K
    assert rel(x, ref.x) <= 1e-8
    x2, info2, _ = _gpu_solve(sysm, m=m, rtol=1e-9, max_iters=5000, ortho=ortho)
    assert abs(info2["iters"] - ref_tol.iters) <= 1
    assert rel(x2, ref_tol.x) <= 1e-8


def test_no_deflation_and_nonzero_x0():
    s = no_defl(W.make_config(1, mesh=40))
    rng = np.random.default_rng(13)
    x0 = rng.standard_normal(s.n)
    ref = oracle.gmres(s, 25, 0.0, 90, x0=x0)
    x, info, _ = _gpu_solve(s, x0=x0, m=25, rtol=0.0, max_iters=90)
    assert rel(x, ref.x) <= 1e-8
    assert abs(info["rho0"] - ref.rho0) <= 1e-12 * ref.rho0


def test_resume_from_checkpoint():
    s = W.make_config(1, mesh=48)
    full = oracle.gmres(s, 20, 0.0, 120)
    x1, i1, _ = _gpu_solve(s, m=20, rtol=0.0, max_iters=40)
    x2, i2, _ = _gpu_solve(s, x0=x1, m=20, rtol=0.0, max_iters=80, r0_norm_override=i1["rho0"])
    assert rel(x2, full.x) <= 1e-8


@pytest.mark.parametrize("ortho", [0, 1, 2])
def test_degenerate_cases(ortho):
    n = 300
    b = np.linspace(1.0, 2.0, n)
    # A = I: one step.
    x, info, _ = _gpu_solve(W.from_dense(np.eye(n), b), m=10, rtol=1e-12, max_iters=50, ortho=ortho)
    assert info["iters"] == 1 and np.allclose(x, b, rtol=1e-14)
    # Four distinct eigenvalues: four steps.
    d = np.repeat([1.0, 2.0, 5.0, -3.0], n // 4)
    x, info, _ = _gpu_solve(W.from_dense(np.diag(d), b), m=20, rtol=1e-13, max_iters=100, ortho=ortho)
    assert info["iters"] == 4 and np.allclose(x, b / d, rtol=1e-12)
    # rho0 = 0 (b = A x0 exactly): immediate return with x = x0.
    s = W.make_config(1, mesh=16)
    s0 = copy.copy(s)
    s0.b = np.zeros(s.n)
    x, info, _ = _gpu_solve(s0, m=10, rtol=1e-8, max_iters=100, ortho=ortho)
    assert info["iters"] == 0 and info["status_name"] == "OK" and not np.any(x)
    x0 = np.random.default_rng(1).standard_normal(n)
    x, info, _ = _gpu_solve(W.from_dense(np.eye(n), x0), x0=x0, m=10, rtol=1e-8, max_iters=100, ortho=ortho)
    assert info["iters"] == 0 and info["status_name"] == "OK"
    assert np.array_equal(x, x0)
    # Z = I: the coarse solve alone gives the answer after zero steps.
    rng = np.random.default_rng(5)
    nz = 40
    A = rng.standard_normal((nz, nz)) / np.sqrt(nz) + 4 * np.eye(nz)
    bz = rng.standard_normal(nz)
    x, info, _ = _gpu_solve(W.from_dense(A, bz, Z=np.eye(nz)), m=5, rtol=1e-12, max_iters=50, ortho=ortho)
    assert info["iters"] == 0 and rel(x, np.linalg.solve(A, bz)) <= 1e-12
    # Cyclic shift with m < N: stagnation, MAXITER.
    nc = 64
    Ac = np.roll(np.eye(nc), 1, axis=0)
    bc = np.zeros(nc)
    bc[0] = 1.0
    x, info, _ = _gpu_solve(W.from_dense(Ac, bc), m=8, rtol=1e-8, max_iters=64, ortho=ortho)
    assert info["status_name"] == "MAXITER" and info["iters"] == 64


def test_error_statuses():
    Gm = G()
    s = W.make_config(1, mesh=8)
    bad = copy.copy(s)
    bad.b = s.b.copy()
    bad.b[5] = np.nan
    with pytest.raises(Gm.GmresError) as e:
        _gpu_solve(bad, m=5)
    assert e.value.status == -3
    dup = copy.copy(s)
    dup.r = 2
    dup.z_rowptr = np.arange(0, 2 * s.n + 1, 2, dtype=np.int32)
    dup.z_colind = np.tile(np.array([0, 1], np.int32), s.n)
    dup.z_vals = np.ones(2 * s.n)
    with pytest.raises(Gm.GmresError) as e:
        Gm.plan_for(dup, m=5)
    assert e.value.status == -2
    mal = copy.copy(s)
    mal.colind = s.colind.copy()
    mal.colind[3] = s.n + 7
    with pytest.raises(Gm.GmresError) as e:
        Gm.plan_for(mal, m=5)
    assert e.value.status == -1
    with pytest.raises(Gm.GmresError):
        Gm.plan_for(s, m=0)
    nanA = copy.copy(s)
    nanA.vals = s.vals.copy()
    nanA.vals[0] = np.inf
    with pytest.raises(Gm.GmresError) as e:
        Gm.plan_for(nanA, m=5)
    assert e.value.status == -3
    # The single-reduction CGS2 (ortho = 2) is an FP64 single-system variant.
    with pytest.raises(Gm.GmresError) as e:
        Gm.plan_for(s, m=5, ortho=2, precision="mixed_f16")
    assert e.value.status == -1
    with pytest.raises(Gm.GmresError) as e:
        Gm.plan_for(s, m=5, ortho=3)
    assert e.value.status == -1


def test_deterministic_reruns():
    s = W.make_config(2, mesh=64)
    plan, d = G().plan_for(s, m=50, rtol=1e-8, max_iters=3000)
    x1, i1 = plan.solve(d["b"])
    x1 = x1.cpu().numpy()
    x2, i2 = plan.solve(d["b"])
    assert i1["iters"] == i2["iters"]
    assert np.array_equal(x1, x2.cpu().numpy())


def test_update_values_matches_fresh_plan():
    s = W.make_config(5, mesh=32)
    plan, d = G().plan_for(s, m=50, rtol=1e-10, max_iters=5000)
    K = s.meta["K_vals"]
    v2 = s.vals + 0.3 * K
    plan.update_values(torch.from_numpy(v2).cuda())
    x, info = plan.solve(d["b"])
    s2 = copy.copy(s)
    s2.vals = v2
    ref = oracle.gmres(s2, 50, 1e-10, 5000)
    assert abs(info["iters"] - ref.iters) <= 1
    assert rel(x.cpu().numpy(), ref.x) <= 1e-8


# --------------------------------------------------------- mixed precision

def _forward_error_bound(s, x1, x2, rho0, rtol):
    """||x1 - x2|| <= ||A^{-1}|| (||r1|| + ||r2||): both satisfy the FP64 residual
    test, so their difference is bounded by the smallest singular value."""
    A = W.dense(s)
    smin = np.linalg.svd(A, compute_uv=False)[-1]
    r1 = np.linalg.norm(host_residual(s, x1))
    r2 = np.linalg.norm(host_residual(s, x2))
    return (r1 + r2) / smin


@pytest.mark.parametrize("ortho", [0, 1])
@pytest.mark.parametrize("prec", ["mixed_f32", "mixed_f16"])
@pytest.mark.parametrize("cfg,mesh", [(1, 32), (2, 48), (5, 32)])
def test_mixed_precision_reaches_fp64_accuracy(prec, cfg, mesh, ortho):
    s = W.make_config(cfg, mesh=mesh)
    m = W.CONFIGS[cfg]["m"]
    ref = oracle.gmres(s, m, 1e-8, 20000)
    inner = 1e-3 if prec == "mixed_f16" else 1e-5
    x, info, _ = _gpu_solve(s, m=m, rtol=1e-8, max_iters=20000, precision=prec, inner_rtol=inner,
                            ortho=ortho)
    r = host_residual(s, x)
    err = rel(x, ref.x)
    say(prec, "config", cfg, "mesh", mesh, "iters", info["iters"], "refinements",
        info["refinements"], "rel err vs FP64 oracle %.2e" % err)
    assert info["status_name"] == "OK"
    assert np.linalg.norm(r) <= 1e-8 * ref.rho0 * (1 + 1e-6)
    assert np.linalg.norm(x - ref.x) <= _forward_error_bound(s, x, ref.x, ref.rho0, 1e-8) * (1 + 1e-6)


# ----------------------------------------------------------------- batched

def _small_batch(nsys=24, lo=6, hi=40):
    ss = W.config_seed(77)
    s_mesh, s_beta, s_sys = ss.spawn(3)
    meshes = np.random.default_rng(s_mesh).integers(lo, hi + 1, size=nsys)
    betas = np.random.default_rng(s_beta).uniform(0.0, 50.0, size=(nsys, 2))
    subs = s_sys.spawn(nsys)
    systems = [W.convection_diffusion_lognormal(int(meshes[i]), beta=tuple(betas[i]), sigma=1.0,
                                                s=(2 if meshes[i] < 12 else 4), seed_seq=subs[i])
               for i in range(nsys)]
    return W.concat_systems(systems)


@pytest.mark.parametrize("wg,lanes", [(256, 8), (512, 4), (1024, 16)])
def test_batched_matches_per_system_oracle(wg, lanes):
    batch = _small_batch()
    plan, d = G().plan_for(batch, m=30, rtol=1e-8, max_iters=5000, batch_wg=wg, batch_lanes=lanes)
    x, infos = plan.solve_batched(d["b"])
    x = x.cpu().numpy()
    for i, s in enumerate(batch.systems):
        ref = oracle.gmres(s, 30, 1e-8, 5000)
        xi = x[batch.row_off[i]:batch.row_off[i + 1]]
        assert infos[i]["status_name"] == "OK", (i, infos[i])
        assert abs(infos[i]["iters"] - ref.iters) <= 1, (i, infos[i]["iters"], ref.iters)
        assert rel(xi, ref.x) <= 1e-8, i
        assert infos[i]["rel_res_true"] <= 1e-8 * (1 + 1e-6)


def test_batched_fixed_count_trajectory():
    batch = _small_batch(nsys=9)
    K = 45
    plan, d = G().plan_for(batch, m=20, rtol=0.0, max_iters=K)
    x, infos = plan.solve_batched(d["b"])
    x = x.cpu().numpy()
    for i, s in enumerate(batch.systems):
        ref = oracle.gmres(s, 20, 0.0, K)
        assert infos[i]["iters"] == K and infos[i]["status_name"] == "MAXITER"
        assert rel(x[batch.row_off[i]:batch.row_off[i + 1]], ref.x) <= 1e-8


@pytest.mark.parametrize("m,wg", [(40, 512), (64, 256), (7, 512)])
def test_batched_restart_lengths(m, wg):
    """Restart lengths beyond 32 take the kernel instance with 64-column
    sweeps (lanes per row pair up to 8); m = 7 restarts often.  Fixed-count
    trajectories over two cycles and to-tolerance solves against the
    per-system oracle."""
    batch = _small_batch(nsys=7, lo=10, hi=36)
    K = 2 * m + 3
    plan, d = G().plan_for(batch, m=m, rtol=0.0, max_iters=K, batch_wg=wg)
    x, infos = plan.solve_batched(d["b"])
    x = x.cpu().numpy()
    for i, s in enumerate(batch.systems):
        ref = oracle.gmres(s, m, 0.0, K)
        assert infos[i]["iters"] == ref.iters, (i, infos[i]["iters"], ref.iters)
        assert rel(x[batch.row_off[i]:batch.row_off[i + 1]], ref.x) <= 1e-8, i
    plan2, d2 = G().plan_for(batch, m=m, rtol=1e-8, max_iters=20000, batch_wg=wg)
    x2, infos2 = plan2.solve_batched(d2["b"])
    x2 = x2.cpu().numpy()
    for i, s in enumerate(batch.systems):
        ref = oracle.gmres(s, m, 1e-8, 20000)
        assert infos2[i]["status_name"] == "OK", (i, infos2[i])
        assert abs(infos2[i]["iters"] - ref.iters) <= 1, (i, infos2[i]["iters"], ref.iters)
        assert rel(x2[batch.row_off[i]:batch.row_off[i + 1]], ref.x) <= 1e-8, i


def _attach_all(plan, batch, steps, **opts):
    subs = {}
    for s in range(len(batch.systems)):
        sub, _ = G().plan_for(batch.systems[s], **opts)
        plan.attach(s, sub, steps)
        subs[s] = sub
    return subs


def test_batched_continuation_fixed_count():
    """Every system leaves the batched launch after its first cycle and goes
    on on its own single-system plan: at a fixed count over three cycles the
    result is the oracle's GMRES(20) trajectory (restarting from the
    corrected iterate is the same iteration)."""
    batch = _small_batch(nsys=9)
    K = 45
    opts = dict(m=20, rtol=0.0, max_iters=K)
    plan, d = G().plan_for(batch, **opts)
    subs = _attach_all(plan, batch, 20, **opts)
    x, infos = plan.solve_batched(d["b"])
    x = x.cpu().numpy()
    for i, s in enumerate(batch.systems):
        ref = oracle.gmres(s, 20, 0.0, K)
        assert infos[i]["iters"] == K and infos[i]["status_name"] == "MAXITER", (i, infos[i])
        assert infos[i]["cycles"] == ref.cycles, (i, infos[i]["cycles"], ref.cycles)
        assert rel(x[batch.row_off[i]:batch.row_off[i + 1]], ref.x) <= 1e-8, i
    assert len(subs) == 9


def test_batched_continuation_to_tolerance():
    """Continuations after one cycle, up to 16 running at once: solutions,
    iteration counts and true residuals as in the per-system oracle solve;
    a second call reuses the plans; detaching restores the plain launch."""
    batch = _small_batch()
    opts = dict(m=30, rtol=1e-8, max_iters=5000)
    plan, d = G().plan_for(batch, **opts)
    _attach_all(plan, batch, 30, **opts)
    refs = [oracle.gmres(s, 30, 1e-8, 5000) for s in batch.systems]
    assert sum(r.iters > 30 for r in refs) >= 17   # more continuations than run at once
    for call in range(2):
        x, infos = plan.solve_batched(d["b"])
        x = x.cpu().numpy()
        for i, ref in enumerate(refs):
            xi = x[batch.row_off[i]:batch.row_off[i + 1]]
            assert infos[i]["status_name"] == "OK", (call, i, infos[i])
            assert abs(infos[i]["iters"] - ref.iters) <= 1, (call, i, infos[i]["iters"], ref.iters)
            assert rel(xi, ref.x) <= 1e-8, (call, i)
            assert infos[i]["rel_res_true"] <= 1e-8 * (1 + 1e-6)
    for s in range(len(batch.systems)):
        plan.attach(s, None, 0)
    x2, infos2 = plan.solve_batched(d["b"])
    for i, ref in enumerate(refs):
        assert abs(infos2[i]["iters"] - ref.iters) <= 1, i


def test_batched_attach_errors_and_update_detaches():
    Gm = G()
    batch = _small_batch(nsys=5)
    opts = dict(m=30, rtol=1e-8, max_iters=5000)
    plan, d = Gm.plan_for(batch, **opts)
    sizes = np.diff(batch.row_off)
    other = int(np.nonzero(sizes != sizes[0])[0][0])
    wrong, _ = Gm.plan_for(batch.systems[other], **opts)
    with pytest.raises(Gm.GmresError):
        plan.attach(0, wrong, 30)               # another system's size
    right, _ = Gm.plan_for(batch.systems[0], **opts)
    with pytest.raises(Gm.GmresError):
        plan.attach(0, right, 0)                # steps < 1
    with pytest.raises(Gm.GmresError):
        plan.attach(len(batch.systems), right, 30)
    m20, _ = Gm.plan_for(batch.systems[0], m=20, rtol=1e-8, max_iters=5000)
    with pytest.raises(Gm.GmresError):
        plan.attach(0, m20, 30)                 # another restart length
    with pytest.raises(Gm.GmresError):
        right.attach(0, right, 30)              # not a batched plan
    plan.attach(0, right, 30)
    twin = int(np.nonzero(sizes == sizes[0])[0][1]) if (sizes == sizes[0]).sum() > 1 else None
    if twin is not None:
        with pytest.raises(Gm.GmresError):
            plan.attach(twin, right, 30)        # one plan, two systems
    plan.update_values(d["vals"])
    assert plan._subs == {}
    x, infos = plan.solve_batched(d["b"])
    ref = oracle.gmres(batch.systems[0], 30, 1e-8, 5000)
    assert abs(infos[0]["iters"] - ref.iters) <= 1


def test_single_system_batch_equals_solve():
    s = W.make_config(1, mesh=40)
    b = W.concat_systems([s])
    pb, db = G().plan_for(b, m=30, rtol=1e-8, max_iters=2000)
    xb, ib = pb.solve_batched(db["b"])
    ps, ds = G().plan_for(s, m=30, rtol=1e-8, max_iters=2000)
    xs, is_ = ps.solve(ds["b"])
    assert abs(ib[0]["iters"] - is_["iters"]) <= 1
    assert rel(xb.cpu().numpy(), xs.cpu().numpy()) <= 1e-8


# ------------------------------------------------------------------ adjoint

def test_adjoint_against_dense_oracle():
    s = W.make_config(5, mesh=32)
    plan, d = G().plan_for(s, need_adjoint=True, m=50, rtol=1e-12, max_iters=5000)
    x, info = plan.solve(d["b"])
    xt = torch.from_numpy(s.meta["x_target"]).cuda()
    gx = (x - xt).contiguous()
    gb, gv, ainfo = plan.adjoint(x, gx)
    A = W.dense(s)
    xn = x.cpu().numpy()
    lam = np.linalg.solve(A.T, gx.cpu().numpy())
    rows = np.repeat(np.arange(s.n), np.diff(s.rowptr))
    gv_ref = -lam[rows] * xn[s.colind]
    assert rel(gb.cpu().numpy(), lam) <= 1e-9
    assert rel(gv.cpu().numpy(), gv_ref) <= 1e-9
    ora = oracle.adjoint(s, xn, gx.cpu().numpy(), 50, 1e-12, 5000)
    assert rel(gb.cpu().numpy(), ora.grad_b) <= 1e-9


def test_autograd_kappa_gradient_finite_difference():
    Gm = G()
    s = W.make_config(5, mesh=32)
    plan, d = Gm.plan_for(s, need_adjoint=True, m=50, rtol=1e-13, max_iters=10000)
    K = torch.from_numpy(s.meta["K_vals"]).cuda()
    Cv = torch.from_numpy(s.meta["C_vals"] + s.meta["D_vals"]).cuda()
    xt = torch.from_numpy(s.meta["x_target"]).cuda()
    b = d["b"]

    def loss(kappa):
        vals = kappa * K + Cv
        x = Gm.DeflatedGMRES.apply(vals, b, plan)
        return 0.5 * torch.sum((x - xt) ** 2)

    kappa = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    L = loss(kappa)
    L.backward()
    g = float(kappa.grad)
    h = 1e-6
    with torch.no_grad():
        fd = (float(loss(torch.tensor(1.0 + h, dtype=torch.float64, device="cuda")))
              - float(loss(torch.tensor(1.0 - h, dtype=torch.float64, device="cuda")))) / (2 * h)
    say("dL/dkappa adjoint %.10e fd %.10e" % (g, fd))
    assert abs(g - fd) <= 1e-5 * abs(g)


def _fd_directions(s, k, seed):
    """k seeded unit directions jointly over (b, the stored entries of the
    non-Dirichlet rows of A, kappa): arrays (db, dv, dk)."""
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(s.n), np.diff(s.rowptr))
    drows = np.nonzero(s.meta["D_vals"] != 0)[0]
    dirichlet_row = np.zeros(s.n, bool)
    dirichlet_row[rows[drows]] = True
    free = ~dirichlet_row[rows]
    out = []
    for _ in range(k):
        db = rng.standard_normal(s.n)
        db[dirichlet_row] = 0.0
        dv = np.where(free, rng.standard_normal(s.nnz), 0.0)
        dk = rng.standard_normal()
        nrm = np.sqrt(np.dot(db, db) + np.dot(dv, dv) + dk * dk)
        out.append((db / nrm, dv / nrm, dk / nrm))
    return out


def test_adjoint_32_directions_central_differences():
    """dL along 32 seeded unit directions over (b, non-Dirichlet values of A,
    kappa) from one adjoint solve, against central differences (h = 1e-6) of
    L = 1/2 ||x - x_target||^2 with FP64 solves started from the unperturbed
    solution (so the solver error scales with h); gate 1e-5 of ||g||."""
    s = W.make_config(5, mesh=32)
    plan, d = G().plan_for(s, need_adjoint=True, m=50, rtol=1e-13, max_iters=20000)
    x, info = plan.solve(d["b"])
    assert info["status_name"] == "OK"
    xt = s.meta["x_target"]
    xn = x.cpu().numpy()
    gx = torch.from_numpy(xn - xt).cuda()
    gb, gv, ainfo = plan.adjoint(x, gx)
    gb, gv = gb.cpu().numpy(), gv.cpu().numpy()
    Kv = s.meta["K_vals"]
    gk = float(np.dot(gv, Kv))
    gnorm = np.sqrt(np.dot(gb, gb) + np.dot(gv, gv) + gk * gk)
    # Warm-started FD solves: the initial residual is O(h), so rtol = 1e-7 puts
    # the solver error at O(1e-7 h) (above the FP64 floor) and the FD error
    # does not grow as h shrinks.
    fdp, fdd = G().plan_for(s, m=50, rtol=1e-7, max_iters=20000)
    x0 = torch.from_numpy(xn).cuda()
    h = 1e-6
    worst = 0.0
    for i, (db, dv, dk) in enumerate(_fd_directions(s, 32, 20190610 + 5)):
        adj = float(np.dot(gb, db) + np.dot(gv, dv) + gk * dk)
        L = []
        for sg in (1.0, -1.0):
            fdp.update_values(torch.from_numpy(s.vals + sg * h * (dv + dk * Kv)).cuda())
            xs, si = fdp.solve(torch.from_numpy(s.b + sg * h * db).cuda(), x0)
            assert si["status_name"] == "OK"
            xs = xs.cpu().numpy()
            L.append(0.5 * np.dot(xs - xt, xs - xt))
        fd = (L[0] - L[1]) / (2 * h)
        err = abs(adj - fd) / gnorm
        worst = max(worst, err)
        if i < 4 or err > 1e-6:
            say(f"direction {i}: adjoint {adj:.10e} central difference {fd:.10e} (|diff|/||g|| {err:.1e})")
    say(f"32 directions: largest |adjoint - FD| / ||g|| = {worst:.2e}")
    assert worst <= 1e-5


def test_mixed_refinement_escalation_and_stagnation():
    """Inner solves capped at two steps cannot halve the FP64 residual, so the
    refinement raises the inner precision: FP16 basis (first refinement),
    FP32 basis (second: the first did not contract), then an FP64 solve to the
    final tolerance (third).  With max_refine = 2 the same stall ends in
    STAGNATED with the refined iterate.  The FP64-accurate result is compared
    with the oracle's solution through the forward-error bound."""
    s = W.make_config(2, mesh=48)
    m = 50
    ref = oracle.gmres(s, m, 1e-8, 20000)
    assert ref.status_name == "OK"
    x, info, plan = _gpu_solve(s, m=m, rtol=1e-8, max_iters=20000, precision="mixed_f16",
                               inner_rtol=1e-3, inner_max_iters=2, max_refine=10, record_history=1)
    say("escalation: refinements", info["refinements"], "iterations", info["iters"],
        "status", info["status_name"], "rel_res_true %.2e" % info["rel_res_true"])
    assert info["status_name"] == "OK" and info["refinements"] == 3
    assert info["iters"] > 4                      # 2 + 2 reduced-precision steps, then the FP64 solve
    r = host_residual(s, x)
    assert np.linalg.norm(r) <= 1e-8 * ref.rho0 * (1 + 1e-6)
    assert np.linalg.norm(x - ref.x) <= _forward_error_bound(s, x, ref.x, ref.rho0, 1e-8) * (1 + 1e-6)
    # The history holds every inner step of all three solves, in order.
    h = plan.history()
    assert h.size == info["iters"]
    assert np.all(np.isfinite(h)) and h[-1] <= 1e-8 * ref.rho0 * 1.01
    # Stagnation: two refinements allowed, both stall.
    xs, infs, _ = _gpu_solve(s, m=m, rtol=1e-8, max_iters=20000, precision="mixed_f16",
                             inner_rtol=1e-3, inner_max_iters=2, max_refine=2)
    say("stagnation: refinements", infs["refinements"], "status", infs["status_name"],
        "rel_res_true %.2e" % infs["rel_res_true"])
    assert infs["status_name"] == "STAGNATED" and infs["refinements"] == 2 and infs["iters"] == 4
    rs = host_residual(s, xs)
    assert abs(np.linalg.norm(rs) / ref.rho0 - infs["rel_res_true"]) <= 1e-10
    assert infs["rel_res_true"] > 1e-8
