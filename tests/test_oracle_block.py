"""Pins of the block GMRES(m) oracle (several right-hand sides, oracle/bgmres.c)
against facts fixed by the mathematics, never against the oracle itself:
  * minimality   -- after j block steps each column's residual equals the
                    brute-force least-squares minimum over an explicit block
                    Krylov basis [R0, A R0, ..., A^{j-1} R0] (numpy lstsq);
  * inclusion    -- each column's residual is at most that of single-vector
                    GMRES(m) started from the same column (its Krylov space is
                    a subspace of the block space);
  * k = 1        -- the block method is GMRES(m);
  * termination  -- block dimension N reached: the exact solution (dense solve);
  * A = I        -- one block step;
  * closed space -- a block step whose new columns are rounding residue ends
                    its cycle (few distinct eigenvalues);
  * estimate     -- the least-squares residual equals the recomputed one after
                    one cycle;
  * whole solve  -- to tolerance on a FEM system, every column within its
                    rtol, solution against a dense direct solve;
  * dependent columns -- B with a repeated column and a column that is the
                    sum of two others: the minimisation is linear in B, so
                    X keeps the same relations (restarts keep one basis vector
                    per independent residual direction);
  * invalid input -- a zero right-hand side column, k < 1.
"""
import copy

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from paper_1906_04051_amd import workloads as W


def _csr(A):
    A = sp.csr_matrix(A)
    A.sort_indices()
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64)


def _nonsym(n, seed):
    rng = np.random.default_rng(seed)
    A = sp.random(n, n, density=0.3, random_state=seed) + sp.eye(n) * 3.0
    A = A.tolil()
    for i in range(n - 1):
        A[i, i + 1] = rng.uniform(-1, 1)
    return A.tocsr()


@pytest.mark.parametrize("k,j", [(2, 1), (2, 3), (3, 2)])
def test_block_residual_is_brute_force_minimum(k, j):
    n = 30
    A = _nonsym(n, 5 + k + j)
    rng = np.random.default_rng(7)
    B = rng.standard_normal((n, k))
    X0 = rng.standard_normal((n, k))
    rp, ci, v = _csr(A)
    res = oracle.bgmres(rp, ci, v, B, j, 0.0, j, X0=X0)
    assert res.iters == j and res.status_name == "MAXITER"
    Ad = A.toarray()
    R0 = B - Ad @ X0
    blocks = [R0]
    for _ in range(j - 1):
        blocks.append(Ad @ blocks[-1])
    K = np.hstack(blocks)
    for c in range(k):
        y, *_ = np.linalg.lstsq(Ad @ K, R0[:, c], rcond=None)
        best = np.linalg.norm(R0[:, c] - Ad @ K @ y)
        got = np.linalg.norm(B[:, c] - Ad @ res.x[:, c])
        assert abs(got - best) <= 1e-9 * np.linalg.norm(R0[:, c]), (c, got, best)


def test_each_column_no_worse_than_single_vector_gmres():
    s = W.make_config(1, mesh=16)
    s = copy.copy(s)
    s.r = 0
    s.z_rowptr = np.zeros(s.n + 1, np.int32)
    s.z_colind = np.zeros(0, np.int32)
    s.z_vals = np.zeros(0)
    rng = np.random.default_rng(3)
    k, m = 4, 6
    B = rng.standard_normal((s.n, k))
    res = oracle.bgmres(s.rowptr, s.colind, s.vals, B, m, 0.0, m)
    for c in range(k):
        single = oracle.gmres(s, m, 0.0, m, b=B[:, c])
        rb = np.linalg.norm(B[:, c] - oracle.spmv(s.rowptr, s.colind, s.vals, res.x[:, c]))
        rs = np.linalg.norm(B[:, c] - oracle.spmv(s.rowptr, s.colind, s.vals, single.x))
        assert rb <= rs * (1 + 1e-10), (c, rb, rs)


def test_single_column_is_gmres():
    s = W.make_config(1, mesh=16)
    s = copy.copy(s)
    s.r = 0
    s.z_rowptr = np.zeros(s.n + 1, np.int32)
    s.z_colind = np.zeros(0, np.int32)
    s.z_vals = np.zeros(0)
    ref = oracle.gmres(s, 10, 1e-9, 3000)
    res = oracle.bgmres(s.rowptr, s.colind, s.vals, s.b[:, None], 10, 1e-9, 3000)
    assert res.status_name == "OK" and ref.status_name == "OK"
    assert res.iters == ref.iters
    assert np.linalg.norm(res.x[:, 0] - ref.x) <= 1e-10 * np.linalg.norm(ref.x)


def test_block_dimension_n_is_exact():
    n, k = 12, 3
    A = _nonsym(n, 11)
    B = np.random.default_rng(2).standard_normal((n, k))
    rp, ci, v = _csr(A)
    res = oracle.bgmres(rp, ci, v, B, n // k, 0.0, n // k)
    assert res.iters == n // k and res.cycles == 1
    ex = np.linalg.solve(A.toarray(), B)
    assert np.abs(res.x - ex).max() <= 1e-11 * np.abs(ex).max()


def test_identity_one_block_step():
    n, k = 20, 4
    rp, ci, v = _csr(sp.eye(n))
    B = np.random.default_rng(4).standard_normal((n, k))
    res = oracle.bgmres(rp, ci, v, B, 5, 1e-12, 50)
    assert res.status_name == "OK" and res.iters == 1
    assert np.abs(res.x - B).max() <= 1e-14


def test_block_space_stops_growing_ends_the_cycle():
    """Four distinct eigenvalues of multiplicity five and two right-hand
    sides: the block Krylov space has dimension 8 (two directions per
    eigenspace), so the fifth block step's new columns are rounding residue
    (below 1e-10 of their norm before orthogonalisation) and that cycle ends
    there (reading: the block space has stopped growing; the step is kept).
    Fixed count of 8 block steps with m = 8: a 5-step cycle, then a 3-step
    one.  With A = I the first block step already closes the space, and the
    result stays finite and exact."""
    n = 20
    d = np.repeat([1.0, 2.0, 5.0, -3.0], 5)
    rp, ci, v = _csr(sp.diags(d))
    B = np.random.default_rng(7).standard_normal((n, 2))
    res = oracle.bgmres(rp, ci, v, B, 8, 0.0, 8)
    assert res.iters == 8 and res.cycles == 2
    assert np.isfinite(res.x).all()
    assert np.allclose(res.x, B / d[:, None], rtol=1e-12, atol=0)
    rp, ci, v = _csr(sp.eye(10))
    B = np.random.default_rng(8).standard_normal((10, 3))
    res = oracle.bgmres(rp, ci, v, B, 4, 0.0, 3)
    assert res.status_name == "OK" and np.isfinite(res.x).all()
    assert np.abs(res.x - B).max() <= 1e-14 * np.abs(B).max()


def test_estimate_is_true_residual_after_one_cycle():
    n, k, m = 40, 3, 4
    A = _nonsym(n, 13)
    B = np.random.default_rng(5).standard_normal((n, k))
    rp, ci, v = _csr(A)
    res = oracle.bgmres(rp, ci, v, B, m, 0.0, m)
    assert abs(res.rel_res_est - res.rel_res_true) <= 1e-10


def test_fem_solve_to_tolerance_against_dense():
    s = W.make_config(1, mesh=16)
    rng = np.random.default_rng(6)
    k = 5
    B = rng.standard_normal((s.n, k))
    res = oracle.bgmres(s.rowptr, s.colind, s.vals, B, 8, 1e-10, 5000)
    assert res.status_name == "OK"
    A = sp.csr_matrix((s.vals, s.colind, s.rowptr), shape=(s.n, s.n)).toarray()
    for c in range(k):
        r = np.linalg.norm(B[:, c] - A @ res.x[:, c])
        assert r <= 1e-10 * np.linalg.norm(B[:, c]) * (1 + 1e-6)
    ex = np.linalg.solve(A, B)
    cond = np.linalg.cond(A)
    assert np.abs(res.x - ex).max() <= 2e-10 * cond * np.abs(ex).max()


def test_invalid_inputs():
    n = 10
    rp, ci, v = _csr(sp.eye(n) * 2.0)
    B = np.ones((n, 3))
    B[:, 1] = 0.0
    assert oracle.bgmres(rp, ci, v, B, 4, 1e-8, 10).status_name == "EINVAL"
    assert oracle.bgmres(rp, ci, v, np.ones((n, 2)), 0, 1e-8, 10).status_name == "EINVAL"


def test_dependent_right_hand_sides_keep_linearity():
    s = W.make_config(1, mesh=24)
    rng = np.random.default_rng(9)
    B = rng.standard_normal((s.n, 5))
    B[:, 2] = B[:, 0]
    B[:, 4] = B[:, 1] + B[:, 3]
    res = oracle.bgmres(s.rowptr, s.colind, s.vals, B, 6, 1e-10, 4000)
    assert res.status_name == "OK"
    X = res.x
    scale = np.abs(X).max()
    assert np.abs(X[:, 2] - X[:, 0]).max() <= 1e-12 * scale
    assert np.abs(X[:, 4] - X[:, 1] - X[:, 3]).max() <= 1e-8 * scale
    for c in range(5):
        r = B[:, c] - oracle.spmv(s.rowptr, s.colind, s.vals, X[:, c])
        assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(B[:, c]) * (1 + 1e-6)


def _z(s):
    return (s.r, s.z_rowptr, s.z_colind, s.z_vals)


@pytest.mark.parametrize("rtol,K", [(0.0, 37), (1e-9, 3000)])
def test_deflated_single_column_is_deflated_gmres(rtol, K):
    """With a deflation basis and one right-hand side the block method is the
    deflated GMRES(m) of the single-vector oracle (Sec. 3.3): the same
    iterate at a fixed count over several cycles, the same step count and
    solution to tolerance."""
    s = W.make_config(1, mesh=16)
    assert s.r > 0
    ref = oracle.gmres(s, 10, rtol, K)
    res = oracle.bgmres(s.rowptr, s.colind, s.vals, s.b[:, None], 10, rtol, K, z=_z(s))
    assert res.iters == ref.iters, (res.iters, ref.iters)
    assert np.linalg.norm(res.x[:, 0] - ref.x) <= 1e-10 * np.linalg.norm(ref.x)
    if rtol > 0:
        assert res.status_name == "OK" and ref.status_name == "OK"
    # Without the projection the block method is another iteration.
    plain = oracle.bgmres(s.rowptr, s.colind, s.vals, s.b[:, None], 10, rtol, K)
    assert np.linalg.norm(plain.x[:, 0] - ref.x) > 1e-6 * np.linalg.norm(ref.x) or plain.iters != ref.iters


def test_deflation_with_full_basis_is_exact():
    """Z = I: P A = 0, the projected residual vanishes at the start and the
    coarse correction alone gives X = A^{-1} B, after no block step."""
    n, k = 30, 3
    A = _nonsym(n, 21)
    rp, ci, v = _csr(A)
    B = np.random.default_rng(8).standard_normal((n, k))
    z = (n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))
    res = oracle.bgmres(rp, ci, v, B, 4, 1e-12, 40, z=z)
    assert res.status_name == "OK" and res.iters == 0
    ex = np.linalg.solve(A.toarray(), B)
    assert np.abs(res.x - ex).max() <= 1e-12 * np.abs(ex).max()


def test_deflated_block_to_tolerance():
    """Four right-hand sides with the indicator basis: every column's true
    residual meets rtol times its unprojected initial residual, and Z^T r = 0
    to rounding (the coarse correction at exit)."""
    s = W.make_config(1, mesh=16)
    k = 4
    B = np.random.default_rng(9).standard_normal((s.n, k))
    res = oracle.bgmres(s.rowptr, s.colind, s.vals, B, 8, 1e-10, 5000, z=_z(s))
    assert res.status_name == "OK"
    A = sp.csr_matrix((s.vals, s.colind, s.rowptr), shape=(s.n, s.n))
    Z = sp.csr_matrix((s.z_vals, s.z_colind, s.z_rowptr), shape=(s.n, s.r))
    for c in range(k):
        r = B[:, c] - A @ res.x[:, c]
        assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(B[:, c]) * (1 + 1e-6)
        zr = Z.T @ r
        zscale = abs(Z).T @ (abs(A) @ np.abs(res.x[:, c]) + np.abs(B[:, c]))
        assert np.all(np.abs(zr) <= 1e3 * np.finfo(float).eps * zscale)
