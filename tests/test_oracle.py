"""Pins of the FP64 CPU oracle against facts fixed by the paper and by the
mathematics (never against the oracle itself).

Each test names the passage or identity it checks:
  * CSR product            -- dense brute force, exact on integer data;
  * Arnoldi (Sec. 3.2)     -- orthonormal V_k, A V_k = V_{k+1} Hbar_k (eq. hessenberg);
  * Givens / eq. res       -- |gamma_{k+1}| equals the recomputed residual;
  * GMRES minimality       -- brute-force least squares over an explicit Krylov basis;
  * termination in <= N steps, A = I, k distinct eigenvalues, cyclic shift;
  * deflation              -- P^2 = P, P A Z = 0, Z^T P = 0, Z = I, invariant subspaces;
  * coarse LU              -- numpy.linalg.solve, backward error;
  * whole solve            -- dense direct solve of the config-1 system;
  * restart / resume       -- resuming from x equals the uninterrupted run;
  * adjoint                -- dense FP64 adjoint and central differences.
"""
import copy

import numpy as np
import pytest

import oracle
from paper_1906_04051_amd import workloads as W

EPS = np.finfo(np.float64).eps


def _no_defl(s):
    s = copy.copy(s)
    s.r = 0
    s.z_rowptr = np.zeros(s.n + 1, np.int32)
    s.z_colind = np.zeros(0, np.int32)
    s.z_vals = np.zeros(0)
    return s


def _dense_P(A, Z):
    if Z.shape[1] == 0:
        return np.eye(A.shape[0])
    E = Z.T @ A @ Z
    return np.eye(A.shape[0]) - A @ Z @ np.linalg.solve(E, Z.T)


def _random_nonsym(n, rng, shift=4.0):
    A = rng.standard_normal((n, n)) / np.sqrt(n) + shift * np.eye(n)
    return A


# ----------------------------------------------------------------- SpMV

def test_spmv_integer_exact():
    rng = np.random.default_rng(1)
    n = 57
    A = rng.integers(-9, 10, size=(n, n)) * (rng.random((n, n)) < 0.2)
    x = rng.integers(-5, 6, size=n).astype(np.float64)
    s = W.from_dense(A.astype(np.float64), np.zeros(n))
    y = oracle.spmv(s.rowptr, s.colind, s.vals, x)
    assert np.array_equal(y, A.astype(np.float64) @ x)


def test_spmv_empty_rows():
    rowptr = np.array([0, 0, 2, 2], np.int32)
    colind = np.array([0, 2], np.int32)
    vals = np.array([3.0, -1.0])
    y = oracle.spmv(rowptr, colind, vals, np.array([1.0, 2.0, 5.0]))
    assert np.array_equal(y, [0.0, -2.0, 0.0])


# ----------------------------------------------------------- generator

@pytest.mark.parametrize("n", [4, 8, 64])
def test_q1_pattern_count(n):
    s = W.convection_diffusion_manufactured(n)
    assert s.nnz == (3 * n + 1) ** 2


@pytest.mark.parametrize("n", [2, 4, 16])
def test_q2_pattern_count(n):
    s = W.bratu_jacobian_q2(n, lam=5.0, beta=(50.0, 50.0), s=2, seed_seq=W.config_seed(3))
    assert s.nnz == (8 * n + 1) ** 2


def test_q1_laplacian_stencil_closed_form():
    # Bilinear stiffness of -Lap on a square mesh: centre 8/3, neighbours -1/3.
    a = W.assemble(1, 8)
    S = a["K"].S
    for iy in range(1, 8):
        for ix in range(1, 8):
            expect = np.full((3, 3), -1.0 / 3.0)
            expect[1, 1] = 8.0 / 3.0
            assert np.allclose(S[iy, ix], expect, atol=1e-14)


def test_interior_row_sums_vanish():
    kappa = np.exp(np.random.default_rng(0).standard_normal((16, 16)))
    a = W.assemble(1, 16, kappa_elem=kappa, beta=(30.0, -7.0))
    for st in (a["K"], a["C"]):
        sums = st.S.sum(axis=(2, 3))
        assert np.abs(sums[1:-1, 1:-1]).max() < 1e-12 * np.abs(st.S).max()
    a2 = W.assemble(2, 6, beta=(3.0, 5.0))
    for st in (a2["K"], a2["C"]):
        sums = st.S.sum(axis=(2, 3))
        assert np.abs(sums[1:-1, 1:-1]).max() < 1e-12 * max(1.0, np.abs(st.S).max())


def test_manufactured_solution_second_order():
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    errs = []
    for n in (16, 32, 64):
        s = W.convection_diffusion_manufactured(n)
        A = sp.csr_matrix((s.vals, s.colind, s.rowptr), shape=(s.n, s.n))
        x = sla.spsolve(A.tocsc(), s.b)
        errs.append(np.abs(x - s.meta["u_exact"]).max())
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(3.6 < q < 4.4 for q in ratios), ratios


def test_indicator_z_partition():
    r, zr, zc, zv = W.indicator_z(1, 64, 4)
    assert r == 16 and np.array_equal(np.diff(zr), np.ones(65 * 65, np.int32))
    counts = np.bincount(zc, minlength=16)
    # 65 nodes per side split 16/16/16/17 (interface nodes go to the upper block).
    per = np.array([16, 16, 16, 17])
    assert np.array_equal(np.sort(counts), np.sort(np.outer(per, per).reshape(-1)))


# ---------------------------------------------------------------- LU(E)

def test_lu_against_numpy():
    rng = np.random.default_rng(2)
    for r in (1, 5, 64):
        E = rng.standard_normal((r, r))
        st, LU, piv = oracle.lu_factor(E)
        assert st == 0
        t = rng.standard_normal(r)
        s = oracle.lu_solve(LU, piv, t)
        assert np.allclose(s, np.linalg.solve(E, t), rtol=1e-10, atol=1e-12)
        # Backward error of the factorisation: Pi E = L U.
        L = np.tril(LU, -1) + np.eye(r)
        U = np.triu(LU)
        PE = E.copy()
        for k in range(r):
            PE[[k, piv[k]]] = PE[[piv[k], k]]
        assert np.abs(PE - L @ U).max() <= 50 * r * EPS * np.abs(E).max()


def test_lu_pivots_on_zero_and_tiny_leading_entries():
    """Partial pivoting (the textbook LU the coarse solve names): a zero or
    tiny leading pivot must be swapped away, not divided by."""
    perm = np.eye(5)[[2, 0, 4, 1, 3]] * np.arange(1.0, 6.0)[:, None]
    for E in (np.array([[0.0, 1.0], [1.0, 0.0]]), perm):
        st, LU, piv = oracle.lu_factor(E)
        assert st == 0
        t = np.arange(1.0, E.shape[0] + 1)
        assert np.allclose(oracle.lu_solve(LU, piv, t), np.linalg.solve(E, t), rtol=1e-14, atol=0)
    rng = np.random.default_rng(5)
    E = rng.standard_normal((64, 64))
    np.fill_diagonal(E, 1e-14)
    st, LU, piv = oracle.lu_factor(E)
    assert st == 0
    t = rng.standard_normal(64)
    x, xr = oracle.lu_solve(LU, piv, t), np.linalg.solve(E, t)
    assert np.linalg.norm(x - xr) <= 1e-10 * np.linalg.norm(xr)


def test_lu_singular():
    E = np.array([[1.0, 2.0], [2.0, 4.0]])
    st, _, _ = oracle.lu_factor(E)
    assert oracle.STATUS[st] == "ESINGULAR"


# ------------------------------------------------------ GMRES invariants

def _small_cd(n=16, s=4):
    sysm = W.convection_diffusion_lognormal(n, beta=(40.0, 10.0), sigma=1.0, s=s, seed_seq=W.config_seed(99))
    return sysm


@pytest.mark.parametrize("defl", [True, False])
def test_arnoldi_relation_and_orthonormality(defl):
    s = _small_cd()
    if not defl:
        s = _no_defl(s)
    m = 20
    res = oracle.gmres(s, m, 0.0, m, first_cycle=True)
    assert res.iters == m
    V = res.V0.T                       # n x (m+1)
    H = res.H0                         # (m+1) x m, before rotations
    A = W.dense(s)
    Z = W.dense_z(s)
    PA = _dense_P(A, Z) @ A
    orth = np.abs(V.T @ V - np.eye(m + 1)).max()
    assert orth < 1e-12
    rel = np.linalg.norm(PA @ V[:, :m] - V @ H) / np.linalg.norm(PA)
    assert rel < 1e-13
    assert np.allclose(np.tril(H, -2), 0.0)     # upper Hessenberg


@pytest.mark.parametrize("defl", [True, False])
def test_gamma_is_recomputed_residual_and_minimal(defl):
    """|gamma_{k+1}| (eq. res) equals ||b - A x_k|| of the returned x_k, and is
    the minimum of ||P(b - A x)|| over x0 + K_k(PA, P r0) (brute force)."""
    s = _small_cd()
    if not defl:
        s = _no_defl(s)
    A = W.dense(s)
    Z = W.dense_z(s)
    P = _dense_P(A, Z)
    K = 12
    full = oracle.gmres(s, 40, 0.0, K, history=True)
    p0 = P @ s.b
    basis = [p0]
    for _ in range(K - 1):
        basis.append(P @ A @ basis[-1])
    for k in range(1, K + 1):
        res = oracle.gmres(s, 40, 0.0, k)
        true_res = np.linalg.norm(s.b - A @ res.x)
        assert abs(true_res - full.history[k - 1]) <= 1e-9 * full.history[0]
        Q, _ = np.linalg.qr(np.stack(basis[:k], axis=1))
        y, *_ = np.linalg.lstsq(P @ A @ Q, p0, rcond=None)
        best = np.linalg.norm(p0 - P @ A @ Q @ y)
        assert abs(best - full.history[k - 1]) <= 1e-9 * full.history[0]
    # Monotone residual (minimal-residual property over nested spaces).
    assert np.all(np.diff(full.history) <= 1e-12 * full.history[0])


def test_full_gmres_terminates_in_n_steps():
    rng = np.random.default_rng(3)
    n = 12
    A = _random_nonsym(n, rng, shift=1.0)
    b = rng.standard_normal(n)
    s = W.from_dense(A, b)
    res = oracle.gmres(s, n, 1e-13, 10 * n)
    assert res.status_name == "OK"
    assert res.iters <= n
    xd = np.linalg.solve(A, b)
    assert np.linalg.norm(res.x - xd) <= 1e-10 * np.linalg.norm(xd)


def test_identity_one_step():
    n = 10
    b = np.arange(1.0, n + 1)
    s = W.from_dense(np.eye(n), b)
    res = oracle.gmres(s, 5, 1e-12, 100)
    assert res.iters == 1 and res.status_name == "OK"
    assert np.allclose(res.x, b, rtol=1e-15)


def test_k_distinct_eigenvalues_k_steps():
    n = 20
    d = np.repeat([1.0, 2.0, 5.0, -3.0], 5)
    b = np.linspace(1.0, 2.0, n)
    s = W.from_dense(np.diag(d), b)
    res = oracle.gmres(s, 20, 1e-13, 100)
    assert res.iters == 4
    assert np.allclose(res.x, b / d, rtol=1e-12)


def _closing_direction_system():
    """diag(1, 1, 1, 1, 1 + 1e-10) with b = (1, 1, 1, 1, 1e-12): every entry of
    v1 = b / ||b|| and of the first step's products is exact except the last,
    so the first Arnoldi step leaves h_21 = 1e-10 * 5e-13 = 5e-23, far below
    eps * ||A v1|| = eps: the Krylov space has (numerically) closed."""
    d = np.array([1.0, 1.0, 1.0, 1.0, 1.0 + 1e-10])
    b = np.array([1.0, 1.0, 1.0, 1.0, 1e-12])
    return d, b, W.from_dense(np.diag(d), b)


def test_lucky_breakdown_ends_the_cycle():
    """Reading c8 (lucky breakdown): h_{j+1,j} <= eps ||P A v_j|| ends the
    cycle at that step, and the restart picks up what rounding left.  In the
    fixed-count protocol (rtol = 0, two steps) that is two one-step cycles;
    without the test the cycle would go on with the normalised rounding
    residue as its second direction."""
    d, b, s = _closing_direction_system()
    res = oracle.gmres(s, 4, 0.0, 2, first_cycle=True)
    assert 0.0 < res.H0[1, 0] <= EPS * 1.0
    assert res.iters == 2 and res.cycles == 2
    assert np.isfinite(res.x).all()
    assert np.allclose(res.x, b / d, rtol=1e-15, atol=0)


def test_cyclic_shift_stagnates_then_exact():
    n = 8
    A = np.roll(np.eye(n), 1, axis=0)       # A e_i = e_{i+1}
    b = np.zeros(n)
    b[0] = 1.0
    s = W.from_dense(A, b)
    full = oracle.gmres(s, n, 1e-14, n, history=True)
    assert np.allclose(full.history[:n - 1], 1.0, rtol=1e-14)
    assert full.iters == n and full.status_name == "OK"
    assert np.allclose(A @ full.x, b)
    restarted = oracle.gmres(s, 4, 1e-8, 40, history=True)
    assert restarted.status_name == "MAXITER" and restarted.iters == 40
    assert np.allclose(restarted.history, 1.0)


def test_fixed_count_mode_runs_exactly():
    s = _small_cd()
    res = oracle.gmres(s, 7, 0.0, 23)
    assert res.iters == 23 and res.cycles == 4 and res.status_name == "MAXITER"


# ------------------------------------------------------------ deflation

def test_projector_identities():
    s = _small_cd(n=12, s=3)
    A = W.dense(s)
    Z = W.dense_z(s)
    rng = np.random.default_rng(4)
    y = rng.standard_normal(s.n)
    w = oracle.apply_projector(s, y)
    ww = oracle.apply_projector(s, w)
    assert np.linalg.norm(ww - w) <= 1e-12 * np.linalg.norm(w)          # P^2 = P
    assert np.abs(Z.T @ w).max() <= 1e-12 * np.linalg.norm(y)           # Z^T P = 0
    for k in range(s.r):
        pz = oracle.apply_projector(s, A @ Z[:, k])                      # P A Z = 0
        assert np.linalg.norm(pz) <= 1e-12 * np.linalg.norm(A @ Z[:, k])
    assert np.allclose(w, _dense_P(A, Z) @ y, rtol=1e-11, atol=1e-12)


def test_final_residual_has_zero_subdomain_sums():
    s = _small_cd(n=24, s=4)
    res = oracle.gmres(s, 10, 1e-3, 1000)
    r = s.b - W.dense(s) @ res.x
    Z = W.dense_z(s)
    assert np.abs(Z.T @ r).max() <= 1e-11 * np.linalg.norm(s.b) * np.sqrt(s.n)
    assert abs(res.rel_res_true - res.rel_res_deflated) <= 1e-10


def test_z_identity_solves_by_coarse_correction():
    rng = np.random.default_rng(5)
    n = 15
    A = _random_nonsym(n, rng)
    b = rng.standard_normal(n)
    s = W.from_dense(A, b, Z=np.eye(n))
    res = oracle.gmres(s, 5, 1e-12, 50)
    assert res.iters == 0 and res.status_name == "OK"
    assert np.allclose(res.x, np.linalg.solve(A, b), rtol=1e-12)


def test_invariant_subspace_deflation_spectrum():
    rng = np.random.default_rng(6)
    n, r = 10, 3
    lam = np.array([0.01, 0.02, 0.05, 1.0, 1.5, 2.0, 2.5, 3.0, 4.0, 5.0])
    S = rng.standard_normal((n, n)) + 3 * np.eye(n)
    A = S @ np.diag(lam) @ np.linalg.inv(S)
    Z = S[:, :r]                                  # A Z = Z diag(lam[:r])
    s = W.from_dense(A, rng.standard_normal(n), Z=Z)
    PA = np.stack([oracle.apply_projector(s, A[:, k]) for k in range(n)], axis=1)
    ev = np.sort_complex(np.linalg.eigvals(PA))
    expect = np.sort_complex(np.concatenate([np.zeros(r), lam[r:]]).astype(complex))
    assert np.allclose(ev, expect, atol=1e-8)
    # GMRES on P A then needs at most n - r steps.
    res = oracle.gmres(s, n, 1e-12, 100)
    assert res.iters <= n - r and res.status_name == "OK"
    assert np.allclose(res.x, np.linalg.solve(A, s.b), rtol=1e-9)


def test_singular_coarse_matrix_and_nonfinite():
    s = _small_cd(n=8, s=2)
    dup = copy.copy(s)
    # Two identical deflation columns: E = Z^T A Z is singular.
    dup.r = 2
    dup.z_rowptr = np.arange(0, 2 * s.n + 1, 2, dtype=np.int32)
    dup.z_colind = np.tile(np.array([0, 1], np.int32), s.n)
    dup.z_vals = np.ones(2 * s.n)
    assert oracle.gmres(dup, 5, 1e-8, 10).status_name == "ESINGULAR"
    bad = copy.copy(s)
    bad.b = s.b.copy()
    bad.b[3] = np.nan
    assert oracle.gmres(bad, 5, 1e-8, 10).status_name == "ENONFINITE"


# ------------------------------------------------- whole solve, restart

def test_config1_against_dense_direct():
    s = W.make_config(1)
    res = oracle.gmres(s, 30, 1e-8, 2000)
    assert res.status_name == "OK" and res.rel_res_true <= 1e-8
    A = W.dense(s)
    xd = np.linalg.solve(A, s.b)
    # Both x and xd have ||b - A x|| <= 1e-8 rho0 (xd to rounding), so
    # ||x - xd|| <= ||A^{-1}|| * 1e-8 * rho0 (+ rounding of the direct solve).
    sv_min = np.linalg.svd(A, compute_uv=False)[-1]
    bound = (1e-8 * res.rho0 / sv_min) + 1e-12 * np.linalg.norm(xd)
    assert np.linalg.norm(res.x - xd) <= bound
    assert np.linalg.norm(s.b - A @ res.x) <= 1e-8 * res.rho0 * (1 + 1e-6)


def test_resume_equals_uninterrupted():
    s = _small_cd(n=20, s=4)
    m = 8
    full = oracle.gmres(s, m, 0.0, 6 * m)
    first = oracle.gmres(s, m, 0.0, 2 * m)
    rest = oracle.gmres(s, m, 0.0, 4 * m, x0=first.x, r0_norm_override=first.rho0)
    assert np.linalg.norm(rest.x - full.x) <= 1e-10 * np.linalg.norm(full.x)


def test_restart_with_m_at_least_n_is_full_gmres():
    rng = np.random.default_rng(7)
    n = 9
    A = _random_nonsym(n, rng, shift=0.5)
    s = W.from_dense(A, rng.standard_normal(n))
    a = oracle.gmres(s, n, 0.0, n, history=True)
    b = oracle.gmres(s, 3 * n, 0.0, n, history=True)
    assert np.allclose(a.history, b.history, rtol=0, atol=0)


# -------------------------------------------------------------- adjoint

def test_transpose_identity():
    s = _small_cd(n=10)
    trp, tci, tv = oracle.csr_transpose(s.rowptr, s.colind, s.vals)
    rng = np.random.default_rng(8)
    u = rng.standard_normal(s.n)
    v = rng.standard_normal(s.n)
    lhs = oracle.dot(oracle.spmv(trp, tci, tv, u), v)
    rhs = oracle.dot(u, oracle.spmv(s.rowptr, s.colind, s.vals, v))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)
    assert np.array_equal(W.dense(W.System(s.n, trp, tci, tv, s.b, 0, s.z_rowptr, s.z_colind, s.z_vals)),
                          W.dense(s).T)


def test_adjoint_against_dense_and_fd():
    """32 x 32 instance of the differentiable system: L = 1/2 ||x - x_t||^2."""
    s = W.make_config(5, mesh=32)
    A = W.dense(s)
    xt = s.meta["x_target"]
    K = s.meta["K_vals"]
    fwd = oracle.gmres(s, 50, 1e-13, 5000)
    x = fwd.x
    g = x - xt
    adj = oracle.adjoint(s, x, g, 50, 1e-13, 5000)
    lam_d = np.linalg.solve(A.T, g)
    assert np.linalg.norm(adj.grad_b - lam_d) <= 1e-9 * np.linalg.norm(lam_d)
    rows = np.repeat(np.arange(s.n), np.diff(s.rowptr))
    gv_d = -lam_d[rows] * x[s.colind]
    assert np.linalg.norm(adj.grad_vals - gv_d) <= 1e-9 * np.linalg.norm(gv_d)
    dkappa = float(np.dot(adj.grad_vals, K))
    # Central difference in kappa with tight FP64 solves.
    h = 1e-6
    Lp = []
    for sign in (+1, -1):
        v = s.vals + sign * h * K
        xs = oracle.gmres(s, 50, 1e-13, 5000, vals=v).x
        Lp.append(0.5 * np.dot(xs - xt, xs - xt))
    fd = (Lp[0] - Lp[1]) / (2 * h)
    assert abs(fd - dkappa) <= 1e-5 * abs(dkappa)


# ------------------------------------------- adaptive spectral deflation (Sec. 3.3)

def _spd_with_spectrum(lam, rng):
    n = len(lam)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return Q @ np.diag(lam) @ Q.T, Q


def test_minv_maps_invariant_subspace_to_mu():
    """Eq. precond2 with U an exact invariant subspace (A U = U Lambda, T = U^T A U
    = Lambda): A M^{-1} U = |mu| U, and M^{-1} v = v for v orthogonal to U."""
    rng = np.random.default_rng(21)
    lam = np.array([0.01, 0.03, 0.1, 1.0, 2.0, 3.0, 5.0, 8.0, 9.0, 10.0])
    A, Q = _spd_with_spectrum(lam, rng)
    U = Q[:, :3]
    T = U.T @ A @ U
    mu = 10.0
    for q in range(3):
        y = A @ oracle.apply_minv(U.T, T, mu, U[:, q])
        assert np.allclose(y, mu * U[:, q], atol=1e-10)
    v = Q[:, 5] + 0.5 * Q[:, 8]
    assert np.allclose(oracle.apply_minv(U.T, T, mu, v), v, atol=1e-13)
    # The spectrum of A M^{-1}: the three smallest eigenvalues move to |mu|.
    AM = np.stack([A @ oracle.apply_minv(U.T, T, mu, np.eye(10)[:, k]) for k in range(10)], axis=1)
    ev = np.sort(np.linalg.eigvals(AM).real)
    assert np.allclose(ev, np.sort(np.concatenate([lam[3:], [mu] * 3])), atol=1e-9)


def test_power_and_inverse_iteration_against_eig():
    """The fixed-count iterations find the dominant and the smallest eigenpair
    of a matrix whose extreme eigenvalues are real and well separated."""
    rng = np.random.default_rng(22)
    n = 12
    lam = np.array([0.05, 0.9, 1.0, 1.2, 1.5, 1.7, 2.0, 2.2, 2.5, 2.7, 3.0, 9.0])
    S = rng.standard_normal((n, n)) + 4 * np.eye(n)
    M = S @ np.diag(lam) @ np.linalg.inv(S)
    mu, z = oracle.power_iteration(M)
    assert abs(mu - 9.0) <= 1e-6 * 9.0
    e_big = S[:, -1] / np.linalg.norm(S[:, -1])
    assert abs(abs(z @ e_big) - 1.0) <= 1e-8
    st, z = oracle.inverse_iteration(M)
    assert st == 0
    e_small = S[:, 0] / np.linalg.norm(S[:, 0])
    assert abs(abs(z @ e_small) - 1.0) <= 1e-10
    st, _ = oracle.inverse_iteration(np.diag([1.0, 0.0, 2.0]))
    assert st != 0


def test_dgmres_without_deflation_is_gmres():
    """r_max = 0 gives M^{-1} = I: plain GMRES(m), the same trajectory as the
    pinned deflated GMRES with an empty Z."""
    s = _no_defl(_small_cd())
    ref = oracle.gmres(s, 12, 1e-9, 3000, history=True)
    res = oracle.dgmres(s, 12, 1e-9, 3000, rmax=0, history=True)
    assert res.status_name == "OK" and res.iters == ref.iters and res.r == 0
    assert np.allclose(res.history, ref.history, rtol=1e-8, atol=1e-14 * ref.rho0)
    assert np.linalg.norm(res.x - ref.x) <= 1e-9 * np.linalg.norm(ref.x)


def test_dgmres_lucky_breakdown_ends_the_cycle():
    """The same closing direction as test_lucky_breakdown_ends_the_cycle under
    the adaptive preconditioner (U empty at the first cycle; with r_max > 0
    the second cycle runs on A M^{-1} with the first cycle's Ritz vector)."""
    d, b, s = _closing_direction_system()
    for rmax in (0, 2):
        res = oracle.dgmres(s, 4, 0.0, 2, rmax=rmax)
        assert res.iters == 2 and res.cycles == 2
        assert np.isfinite(res.x).all()
        assert np.allclose(res.x, b / d, rtol=1e-15, atol=0)


def test_dgmres_solves_and_keeps_invariants():
    """Adaptive deflation: the returned x meets the tolerance on the true
    residual, U stays orthonormal with r <= r_max, T = U^T A U."""
    s = _small_cd()
    A = W.dense(s)
    for rmax in (3, 20):
        res = oracle.dgmres(s, 10, 1e-10, 5000, rmax=rmax, export=True)
        assert res.status_name == "OK"
        r = np.linalg.norm(s.b - A @ res.x)
        assert r <= 1e-10 * res.rho0 * (1 + 1e-6)
        assert abs(r / res.rho0 - res.rel_res_true) <= 1e-12
        U = res.U.T
        assert 1 <= res.r <= rmax
        assert np.linalg.norm(U.T @ U - np.eye(res.r)) <= 1e-10
        assert np.linalg.norm(res.T - U.T @ A @ U) <= 1e-10 * np.linalg.norm(A, 2)


def test_dgmres_estimate_is_true_residual_after_one_cycle():
    """Right preconditioning keeps |gamma_{k+1}| = ||b - A x_k|| (eq. res)."""
    s = _small_cd()
    res = oracle.dgmres(s, 15, 0.0, 15, rmax=5, history=True)
    assert res.iters == 15
    assert abs(res.history[-1] - res.rel_res_true * res.rho0) <= 1e-9 * res.rho0


def test_dgmres_deflation_reduces_iterations():
    """Deflating the small Ritz directions speeds up GMRES(m) on a
    diffusion-dominated problem (Sec. 3.3, convergence figure)."""
    s = W.make_config(1, mesh=24)
    plain = oracle.dgmres(s, 10, 1e-8, 20000, rmax=0)
    defl = oracle.dgmres(s, 10, 1e-8, 20000, rmax=20)
    assert plain.status_name == "OK" and defl.status_name == "OK"
    assert defl.iters < 0.8 * plain.iters


def test_dgmres_removal_keeps_smallest_directions():
    """With r_max = 2 the removal keeps U orthonormal and T consistent after
    many restarts; the kept directions have Rayleigh quotients near the small
    end of the spectrum."""
    rng = np.random.default_rng(23)
    lam = np.concatenate([[0.001, 0.002], np.linspace(1.0, 2.0, 58)])
    A, Q = _spd_with_spectrum(lam, rng)
    s = W.from_dense(A, rng.standard_normal(60))
    res = oracle.dgmres(s, 6, 1e-12, 4000, rmax=2, export=True)
    assert res.status_name == "OK" and res.r == 2
    U = res.U.T
    assert np.linalg.norm(U.T @ U - np.eye(2)) <= 1e-10
    assert np.linalg.norm(res.T - U.T @ A @ U) <= 1e-10 * 2.0
    assert np.max(np.abs(np.linalg.eigvals(res.T))) < 0.5
