"""The paper's benchmark problem: the 3-D Bratu problem on the unit cube with
27-node (tri-quadratic) hexahedra, solved by Newton's method whose linear
systems go to the GPU GMRES(m) (arXiv 1906.04051, Sec. 3.1).

    lap(u) + lam * exp(u) = 0 in [0,1]^3  (eq. bratu-eq), lam = 6.8,
    u = 0 on the x- and y-faces, du/dz = 0 on the z-faces.

Galerkin residuals (eq. weak-form, boundary term absent):
    R_i = - sum_j u_j int grad(phi_j).grad(phi_i) + lam int exp(u_h) phi_i,
Jacobian J_ij = dR_i/du_j = - K_ij + lam int exp(u_h) phi_j phi_i, and the rows
of x- and y-face nodes replaced by u_i = 0 (identity rows, one stored entry);
interior rows keep their couplings to those nodes.  Newton (eq. system):
J(u^k) du^k = -R(u^k), u^{k+1} = u^k + du^k, until ||du^k|| <= tol.

This module is the input side (the matrices and right-hand sides the solver
receives) and the Newton driver; the linear solves run in the HIP library.

Structure used for speed: on a uniform tensor-product mesh the stiffness
matrix is a sum of Kronecker products of the 1-D Q2 stiffness and mass
matrices, so only the exp(u) term needs element quadrature (3 Gauss points
per direction); it is scattered into the CSR values through a precomputed
position map.
"""
from __future__ import annotations

import dataclasses
import sys
import time
from typing import Optional

import numpy as np
import scipy.sparse as sp

from .workloads import System

LAMBDA = 6.8   # Sec. 3.1


def table1_meshes():
    """Elements per side n of the paper's Table 1 sizes: DOF = (2n + 1)^3."""
    return [15, 25, 30, 35, 40, 45, 50, 55, 60]


def pattern_nnz(n: int) -> int:
    """Stored entries of the Jacobian: x/y-interior rows keep the tensor
    stencil (1-D Q2 coupling count 8n + 1 per direction, minus the two
    Dirichlet end rows' 3 couplings in x and y), x/y-face rows one entry."""
    p = 2 * n + 1
    return (8 * n + 1 - 6) ** 2 * (8 * n + 1) + (p ** 3 - (p - 2) ** 2 * p)


def csr_mib(n: int) -> float:
    """CSR storage in MiB: 8-byte values, 4-byte indices, 4-byte row pointers."""
    p = 2 * n + 1
    return (12.0 * pattern_nnz(n) + 4.0 * (p ** 3 + 1)) / 2 ** 20


# ----------------------------------------------------------- 1-D Q2 pieces
_GP = np.array([-np.sqrt(0.6), 0.0, np.sqrt(0.6)])
_GW = np.array([5.0, 8.0, 5.0]) / 9.0


def _q2_1d(t):
    """Q2 shape functions on [0, 1] at points t (nodes 0, 1/2, 1) and their
    derivatives: arrays (3, len(t))."""
    t = np.asarray(t, dtype=np.float64)
    N = np.stack([2 * (t - 0.5) * (t - 1), -4 * t * (t - 1), 2 * t * (t - 0.5)])
    dN = np.stack([4 * t - 3, -8 * t + 4, 4 * t - 1])
    return N, dN


def q2_element_1d(h: float):
    """1-D element stiffness and mass of a Q2 element of length h (3-point
    Gauss, exact for these polynomials)."""
    t = 0.5 * (_GP + 1.0)
    w = 0.5 * _GW
    N, dN = _q2_1d(t)
    K = (dN * w) @ dN.T / h
    M = (N * w) @ N.T * h
    return K, M


def _global_1d(n: int):
    """1-D global Q2 stiffness and mass (p = 2n + 1 nodes), CSR."""
    h = 1.0 / n
    Ke, Me = q2_element_1d(h)
    p = 2 * n + 1
    K = np.zeros((p, p))
    M = np.zeros((p, p))
    for e in range(n):
        idx = [2 * e, 2 * e + 1, 2 * e + 2]
        K[np.ix_(idx, idx)] += Ke
        M[np.ix_(idx, idx)] += Me
    return sp.csr_matrix(K), sp.csr_matrix(M)


@dataclasses.dataclass
class BratuMesh:
    """Pattern, linear part and quadrature map of one mesh (n elements per side)."""
    n: int
    p: int
    N: int
    rowptr: np.ndarray      # int32, Dirichlet rows reduced to the diagonal
    colind: np.ndarray      # int32
    negK: np.ndarray        # values of -K on the pattern (Dirichlet rows 0)
    dirichlet: np.ndarray   # bool [N]
    diag_pos: np.ndarray    # position of each row's diagonal entry
    elem_nodes: np.ndarray  # int64 [E, 27]
    pos: np.ndarray         # int64 [E, 27*27]: CSR position of (a, b), -1 for Dirichlet rows
    phi: np.ndarray         # [27 quad points, 27 shape functions]
    wdet: np.ndarray        # [27] quadrature weights times the element volume


def _log(verbose, *a):
    if verbose:
        print("[bratu3d]", *a, file=sys.stderr, flush=True)


def build_mesh(n: int, verbose: bool = False) -> BratuMesh:
    t0 = time.time()
    p = 2 * n + 1
    N = p ** 3
    K1, M1 = _global_1d(n)
    # Node (ix, iy, iz) -> index ix + p*iy + p^2*iz, so the Kronecker order is z, y, x.
    def kron3(a, b, c):
        return sp.kron(sp.kron(a, b, format="coo"), c, format="coo")

    K = (kron3(M1, M1, K1) + kron3(M1, K1, M1) + kron3(K1, M1, M1)).tocsr()
    K.eliminate_zeros()   # block formats may carry explicit zeros
    K.sort_indices()
    if K.nnz != (8 * n + 1) ** 3:
        raise RuntimeError("unexpected Q2 tensor pattern")
    ix = np.arange(N) % p
    iy = (np.arange(N) // p) % p
    dirichlet = (ix == 0) | (ix == p - 1) | (iy == 0) | (iy == p - 1)
    # Pattern: full tensor stencil in x/y-interior rows, the diagonal alone in
    # x/y-face rows.
    lens = np.diff(K.indptr)
    keep_row = ~dirichlet
    row_of = np.repeat(np.arange(N), lens)
    keep = keep_row[row_of] | (K.indices == row_of)
    colind = K.indices[keep].astype(np.int32)
    newlens = np.bincount(row_of[keep], minlength=N)
    rowptr = np.zeros(N + 1, np.int64)
    np.cumsum(newlens, out=rowptr[1:])
    negK = -K.data[keep]
    rows_kept = row_of[keep]
    negK[dirichlet[rows_kept]] = 0.0
    diag_pos = np.searchsorted(np.asarray(rows_kept, np.int64) * N + colind, np.arange(N, dtype=np.int64) * (N + 1))
    _log(verbose, f"n={n}: pattern {len(colind)} entries ({time.time() - t0:.1f} s)")
    # Elements and quadrature.
    ne = n ** 3
    e = np.arange(ne)
    ex, ey, ez = e % n, (e // n) % n, e // (n * n)
    loc = np.array([(a % 3, (a // 3) % 3, a // 9) for a in range(27)])   # local (x, y, z) offsets
    elem_nodes = ((2 * ex[:, None] + loc[None, :, 0]) + p * (2 * ey[:, None] + loc[None, :, 1])
                  + p * p * (2 * ez[:, None] + loc[None, :, 2])).astype(np.int64)
    t = 0.5 * (_GP + 1.0)
    w1 = 0.5 * _GW
    N1, _ = _q2_1d(t)                               # (3 shapes, 3 points)
    qloc = np.array([(g % 3, (g // 3) % 3, g // 9) for g in range(27)])
    phi = (N1[loc[None, :, 0], qloc[:, None, 0]] * N1[loc[None, :, 1], qloc[:, None, 1]]
           * N1[loc[None, :, 2], qloc[:, None, 2]])   # [g, a]
    h = 1.0 / n
    wdet = w1[qloc[:, 0]] * w1[qloc[:, 1]] * w1[qloc[:, 2]] * h ** 3
    # CSR position of every element pair (a, b) in a non-Dirichlet row.
    keys = rows_kept.astype(np.int64) * N + colind
    rows_e = np.repeat(elem_nodes, 27, axis=1)       # a-major
    cols_e = np.tile(elem_nodes, (1, 27))
    pos = np.searchsorted(keys, (rows_e * N + cols_e).ravel()).reshape(ne, 27 * 27)
    pos[dirichlet[rows_e]] = -1
    _log(verbose, f"n={n}: quadrature map ready ({time.time() - t0:.1f} s)")
    return BratuMesh(n=n, p=p, N=N, rowptr=rowptr.astype(np.int32), colind=colind, negK=negK,
                     dirichlet=dirichlet, diag_pos=diag_pos, elem_nodes=elem_nodes, pos=pos, phi=phi,
                     wdet=wdet)


def _negK_matvec(mesh: BratuMesh, u: np.ndarray) -> np.ndarray:
    """(-K u) restricted to the non-Dirichlet rows' stored couplings."""
    A = sp.csr_matrix((mesh.negK, mesh.colind, mesh.rowptr), shape=(mesh.N, mesh.N))
    return A @ u


def jacobian_residual(mesh: BratuMesh, u: np.ndarray, lam: float = LAMBDA, chunk: int = 20000):
    """Values of J(u) on the mesh pattern and R(u) (eq. weak-form; Dirichlet rows
    J = identity, R_i = u_i)."""
    vals = mesh.negK.copy()
    R = _negK_matvec(mesh, u)
    E = mesh.elem_nodes.shape[0]
    for c0 in range(0, E, chunk):
        en = mesh.elem_nodes[c0:c0 + chunk]
        ug = u[en] @ mesh.phi.T                              # [e, g]
        wg = lam * np.exp(ug) * mesh.wdet[None, :]           # [e, g]
        Me = np.einsum("eg,ga,gb->eab", wg, mesh.phi, mesh.phi).reshape(len(en), -1)
        ps = mesh.pos[c0:c0 + chunk].ravel()
        ok = ps >= 0
        vals += np.bincount(ps[ok], weights=Me.ravel()[ok], minlength=len(vals))
        Fe = wg @ mesh.phi                                    # [e, a]: lam int exp(u) phi_a
        rows = en.ravel()
        R += np.bincount(rows, weights=Fe.ravel(), minlength=mesh.N)
    R[mesh.dirichlet] = u[mesh.dirichlet]
    vals[mesh.diag_pos[mesh.dirichlet]] = 1.0
    return vals, R


def system_at(mesh: BratuMesh, u: np.ndarray, lam: float = LAMBDA) -> System:
    """The Newton system J(u) du = -R(u) as a System without a deflation basis."""
    vals, R = jacobian_residual(mesh, u, lam)
    return System(n=mesh.N, rowptr=mesh.rowptr, colind=mesh.colind, vals=vals, b=-R, r=0,
                  z_rowptr=np.zeros(mesh.N + 1, np.int32), z_colind=np.zeros(0, np.int32),
                  z_vals=np.zeros(0), meta=dict(problem="bratu3d", n=mesh.n, lam=lam))


def newton(mesh: BratuMesh, solve, lam: float = LAMBDA, tol: float = 1e-8, max_newton: int = 12,
           u0: Optional[np.ndarray] = None, verbose: bool = False):
    """Newton's method (eq. system).  solve(vals, b) -> (du, info) solves
    J du = b for the current values on the mesh pattern.  Stops when
    ||du||_2 <= tol * max(1, ||u||_2).  Returns (u, history)."""
    u = np.zeros(mesh.N) if u0 is None else np.array(u0, dtype=np.float64)
    hist = []
    for k in range(max_newton):
        t0 = time.time()
        vals, R = jacobian_residual(mesh, u, lam)
        ta = time.time() - t0
        du, info = solve(vals, -R)
        u = u + du
        nd = float(np.linalg.norm(du))
        hist.append(dict(newton=k, du=nd, res=float(np.linalg.norm(R)), assembly_s=ta, **info))
        _log(verbose, f"newton {k}: ||R|| {hist[-1]['res']:.3e} ||du|| {nd:.3e} "
                      f"gmres iters {info.get('iters')} ({info.get('solve_ms', 0):.0f} ms)")
        if nd <= tol * max(1.0, float(np.linalg.norm(u))):
            break
    return u, hist


def gpu_solver(mesh: BratuMesh, lam: float = LAMBDA, **opts):
    """A Newton linear solver on the GPU library: one plan for the mesh
    pattern, the Jacobian values replaced at every Newton step
    (gmres_update_values), then gmres_solve.  Returns (solve, plan)."""
    import torch

    from . import gmres as G

    sys0 = system_at(mesh, np.zeros(mesh.N), lam)
    plan, d = G.plan_for(sys0, **opts)
    plan.autotune()   # SpMV variant and grids for this pattern, kept for every Newton step

    def solve(vals, b):
        plan.update_values(torch.from_numpy(np.ascontiguousarray(vals)).cuda())
        x, info = plan.solve(torch.from_numpy(np.ascontiguousarray(b)).cuda())
        return x.cpu().numpy(), dict(iters=info["iters"], status=info["status_name"],
                                     rel_res_true=info["rel_res_true"], solve_ms=info["solve_ms"],
                                     defl_r=info["defl_r"])

    return solve, plan
