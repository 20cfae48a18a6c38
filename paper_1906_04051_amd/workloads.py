"""Seeded synthetic FEM systems Ax = b (inputs only).

This module builds the linear systems that the deflated GMRES(m) solver and
the CPU oracle are both run on.  It holds none of the solver's arithmetic:
it assembles matrices, right-hand sides and deflation bases and nothing else,
so both sides can take their inputs from here without sharing any solver code.

Problem family (the paper's benchmark is a Galerkin FEM Jacobian of a Bratu
problem, Sec. 3.1, eqs. bratu-eq .. system; this module builds its 2-D
counterparts):

* Q1 (bilinear) or Q2 (biquadratic Lagrange) elements on a uniform n x n mesh
  of the unit square, nodes numbered lexicographically (x fastest).
* Operator  -div(kappa grad u) + beta . grad u  (Galerkin, no stabilisation),
  optionally  - lambda e^{u_h} u  (the linearised Bratu term).
* Dirichlet nodes get identity rows and b_i = 0; interior rows keep their
  couplings to Dirichlet columns (Sec. 3.1: boundary equations are replaced
  by u_i = 0).  Every row stores the full structural stencil, with explicit
  zeros in the Dirichlet rows, so nnz = (3n+1)^2 for Q1 and (8n+1)^2 for Q2.
* CSR with int32 row pointers and column indices, sorted columns, float64
  values (Sec. 4: CSR storage, double precision).
* Deflation basis Z: indicator functions of an s x s grid of subdomains,
  stored as an N x s^2 CSR matrix with one unit entry per row.

Seeds: numpy SeedSequence(20190610 + config_index).spawn(...) substreams.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

BASE_SEED = 20190610

# 1-D Gauss-Legendre rules on [0, 1].
_G2_PTS = np.array([0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0)])
_G2_WTS = np.array([0.5, 0.5])
_G3_PTS = np.array([0.5 - 0.5 * math.sqrt(0.6), 0.5, 0.5 + 0.5 * math.sqrt(0.6)])
_G3_WTS = np.array([5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0])


@dataclasses.dataclass
class System:
    """One sparse system in CSR form plus its deflation basis and metadata."""

    n: int                       # unknowns
    rowptr: np.ndarray           # int32 [n+1]
    colind: np.ndarray           # int32 [nnz]
    vals: np.ndarray             # float64 [nnz]
    b: np.ndarray                # float64 [n]
    r: int                       # deflation vectors
    z_rowptr: np.ndarray         # int32 [n+1]
    z_colind: np.ndarray         # int32 [z_nnz]
    z_vals: np.ndarray           # float64 [z_nnz]
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])


# ---------------------------------------------------------------------------
# 1-D shape functions on the reference interval [0, 1]
# ---------------------------------------------------------------------------

def _shape_1d(order: int, t: np.ndarray):
    """Values and derivatives of the 1-D Lagrange basis at points t."""
    t = np.asarray(t, dtype=np.float64)
    if order == 1:
        val = np.stack([1.0 - t, t])
        der = np.stack([-np.ones_like(t), np.ones_like(t)])
    elif order == 2:
        val = np.stack([2.0 * (t - 0.5) * (t - 1.0), -4.0 * t * (t - 1.0), 2.0 * t * (t - 0.5)])
        der = np.stack([4.0 * t - 3.0, -8.0 * t + 4.0, 4.0 * t - 1.0])
    else:
        raise ValueError("order must be 1 or 2")
    return val, der  # shape [order+1, len(t)]


def _quad_2d(pts, wts):
    """Tensor Gauss rule: list of (tx, ty, w)."""
    out = []
    for iy, ty in enumerate(pts):
        for ix, tx in enumerate(pts):
            out.append((tx, ty, wts[ix] * wts[iy]))
    return out


# ---------------------------------------------------------------------------
# Structured assembly into a per-node stencil array
# ---------------------------------------------------------------------------

class _Stencil:
    """Per-node coupling coefficients S[iy, ix, dy, dx] for offsets in
    [-w, w]^2, plus the structural-coupling mask of the FEM pattern."""

    def __init__(self, order: int, n: int):
        self.order = order
        self.n = n
        self.p = order * n + 1          # nodes per side
        self.w = order                  # max offset
        k = 2 * self.w + 1
        self.S = np.zeros((self.p, self.p, k, k), dtype=np.float64)

    def add_element_matrix(self, a, b, coef):
        """Add coef[ey, ex] (per element) at row = local node a, col = local
        node b of every element.  a, b are (ax, ay) local tensor indices."""
        o, n, w = self.order, self.n, self.w
        ax, ay = a
        bx, by = b
        # Element (ex, ey) has local node (ax, ay) at global (o*ex + ax, o*ey + ay).
        sl_y = slice(ay, ay + o * n, o)
        sl_x = slice(ax, ax + o * n, o)
        self.S[sl_y, sl_x, by - ay + w, bx - ax + w] += coef

    def pattern_mask_1d(self):
        """mask1[p, d+w]: node p couples to node p+d in 1-D."""
        o, w, P = self.order, self.w, self.p
        m = np.zeros((P, 2 * w + 1), dtype=bool)
        pos = np.arange(P)
        for d in range(-w, w + 1):
            q = pos + d
            inb = (q >= 0) & (q < P)
            if o == 1:
                ok = inb & (abs(d) <= 1)
            else:
                # Q2: vertex (even) nodes couple within +-2, mid (odd) nodes within +-1;
                # the pair must share an element (both in [2e, 2e+2] for some e).
                lo = np.minimum(pos, q)
                hi = np.maximum(pos, q)
                e_lo = np.ceil((hi - 2) / 2.0)
                e_hi = np.floor(lo / 2.0)
                ok = inb & (e_lo <= e_hi) & (e_hi >= 0) & (e_lo <= self.n - 1)
            m[:, d + w] = ok
        return m

    def to_csr(self, dirichlet: np.ndarray):
        """CSR of the full structural pattern.  Dirichlet rows become identity
        rows with explicit zeros in the off-diagonal positions."""
        P, w = self.p, self.w
        S = self.S
        S[dirichlet] = 0.0
        S[dirichlet, w, w] = 1.0
        m1 = self.pattern_mask_1d()
        mask = m1[:, None, :, None] & m1[None, :, None, :]          # [iy, ix, dy, dx]
        counts = mask.reshape(P * P, -1).sum(axis=1)
        rowptr = np.zeros(P * P + 1, dtype=np.int64)
        np.cumsum(counts, out=rowptr[1:])
        if rowptr[-1] >= 2**31:
            raise ValueError("nnz exceeds int32 range")
        iy, ix, dy, dx = np.nonzero(mask)                             # C order == row-major, sorted cols
        colind = ((iy + dy - w) * P + (ix + dx - w)).astype(np.int32)
        vals = S[iy, ix, dy, dx]
        return rowptr.astype(np.int32), colind, np.ascontiguousarray(vals, dtype=np.float64)


def _boundary_mask(P: int) -> np.ndarray:
    d = np.zeros((P, P), dtype=bool)
    d[0, :] = d[-1, :] = d[:, 0] = d[:, -1] = True
    return d


def _node_coords(P: int):
    t = np.linspace(0.0, 1.0, P)
    return np.meshgrid(t, t, indexing="xy")   # X[iy, ix], Y[iy, ix]


def _elem_values(order, n, nodal, tx, ty):
    """u_h at reference point (tx, ty) of every element, from nodal values
    nodal[iy, ix]; returns [n, n] (ey, ex)."""
    val, _ = _shape_1d(order, np.array([tx, ty]))
    out = np.zeros((n, n))
    o = order
    for ay in range(o + 1):
        for ax in range(o + 1):
            out += val[ax, 0] * val[ay, 1] * nodal[ay:ay + o * n:o, ax:ax + o * n:o]
    return out


def assemble(order: int, n: int, kappa_elem=None, beta=(0.0, 0.0), lam: float = 0.0,
             u_nodal: Optional[np.ndarray] = None, f=None, want_parts: bool = False):
    """Galerkin assembly of  -div(kappa grad u) + beta.grad u - lam e^{u_h} u.

    kappa_elem: per-element diffusion [n, n] (ey, ex) or None (= 1).
    lam, u_nodal: Bratu Jacobian term -lam * int e^{u_h} phi_j phi_i (Sec. 3.1,
      J_ij = dR_i/du_j), evaluated at the iterate u_nodal [P, P].
    f: callable f(x, y) for the load int f phi_i (3x3 Gauss), or None.
    Returns a dict of stencils/loads before Dirichlet treatment.
    """
    o = order
    P = o * n + 1
    h = 1.0 / n
    nl = o + 1
    pts, wts = (_G2_PTS, _G2_WTS) if (o == 1 and lam == 0.0) else (_G3_PTS, _G3_WTS)
    quad = _quad_2d(pts, wts)
    if kappa_elem is None:
        kappa_elem = np.ones((n, n))
    kappa_elem = np.asarray(kappa_elem, dtype=np.float64)

    # Reference element matrices (per unit kappa / per unit beta component).
    Kref = np.zeros((nl, nl, nl, nl))      # [ay, ax, by, bx]
    Cx = np.zeros_like(Kref)
    Cy = np.zeros_like(Kref)
    for tx, ty, wq in quad:
        vx, dx = _shape_1d(o, np.array([tx]))
        vy, dy = _shape_1d(o, np.array([ty]))
        phi = vy[:, 0][:, None] * vx[:, 0][None, :]                # [ay, ax]
        gx = vy[:, 0][:, None] * dx[:, 0][None, :]                 # d/dxi
        gy = dy[:, 0][:, None] * vx[:, 0][None, :]
        Kref += wq * (gx[:, :, None, None] * gx[None, None, :, :] + gy[:, :, None, None] * gy[None, None, :, :])
        Cx += wq * h * (phi[:, :, None, None] * gx[None, None, :, :])
        Cy += wq * h * (phi[:, :, None, None] * gy[None, None, :, :])

    stK = _Stencil(o, n)
    stC = _Stencil(o, n)
    stM = _Stencil(o, n) if lam != 0.0 else None
    beta = (float(beta[0]), float(beta[1]))
    for ay in range(nl):
        for ax in range(nl):
            for by in range(nl):
                for bx in range(nl):
                    stK.add_element_matrix((ax, ay), (bx, by), Kref[ay, ax, by, bx] * kappa_elem)
                    c = beta[0] * Cx[ay, ax, by, bx] + beta[1] * Cy[ay, ax, by, bx]
                    if c != 0.0:
                        stC.add_element_matrix((ax, ay), (bx, by), np.full((n, n), c))

    expu_q = None
    if lam != 0.0:
        # e^{u_h} at each quadrature point of every element.
        expu_q = [np.exp(_elem_values(o, n, u_nodal, tx, ty)) for tx, ty, _ in quad]
        for ay in range(nl):
            for ax in range(nl):
                for by in range(nl):
                    for bx in range(nl):
                        acc = np.zeros((n, n))
                        for qi, (tx, ty, wq) in enumerate(quad):
                            vx, _ = _shape_1d(o, np.array([tx]))
                            vy, _ = _shape_1d(o, np.array([ty]))
                            pa = vx[ax, 0] * vy[ay, 0]
                            pb = vx[bx, 0] * vy[by, 0]
                            acc += (wq * h * h * pa * pb) * expu_q[qi]
                        stM.add_element_matrix((ax, ay), (bx, by), acc)

    load = None
    if f is not None:
        load = np.zeros((P, P))
        for tx, ty, wq in _quad_2d(_G3_PTS, _G3_WTS):
            vx, _ = _shape_1d(o, np.array([tx]))
            vy, _ = _shape_1d(o, np.array([ty]))
            ex = np.arange(n)
            X = (ex[None, :] + tx) * h
            Y = (ex[:, None] + ty) * h
            fq = f(X, Y) * (wq * h * h)
            for ay in range(nl):
                for ax in range(nl):
                    load[ay:ay + o * n:o, ax:ax + o * n:o] += vx[ax, 0] * vy[ay, 0] * fq
    bratu_load = None
    if lam != 0.0:
        # int e^{u_h} phi_i (for the Bratu residual).
        bratu_load = np.zeros((P, P))
        for qi, (tx, ty, wq) in enumerate(quad):
            vx, _ = _shape_1d(o, np.array([tx]))
            vy, _ = _shape_1d(o, np.array([ty]))
            for ay in range(nl):
                for ax in range(nl):
                    bratu_load[ay:ay + o * n:o, ax:ax + o * n:o] += (wq * h * h * vx[ax, 0] * vy[ay, 0]) * expu_q[qi]
    return dict(order=o, n=n, P=P, K=stK, C=stC, M=stM, load=load, bratu_load=bratu_load)


def _stencil_apply(st: _Stencil, u: np.ndarray) -> np.ndarray:
    """Row-wise product of the (pre-Dirichlet) stencil with nodal values u[P, P]."""
    P, w = st.p, st.w
    out = np.zeros((P, P))
    up = np.zeros((P + 2 * w, P + 2 * w))
    up[w:w + P, w:w + P] = u
    for dy in range(-w, w + 1):
        for dx in range(-w, w + 1):
            out += st.S[:, :, dy + w, dx + w] * up[w + dy:w + dy + P, w + dx:w + dx + P]
    return out


def indicator_z(order: int, n: int, s: int):
    """Indicator functions of an s x s subdomain grid as an N x s^2 CSR.

    Node (x, y) belongs to subdomain (min(floor(x s), s-1), min(floor(y s), s-1));
    interface nodes go to the upper block, boundary nodes are included, values 1.
    """
    P = order * n + 1
    N = P * P
    if s == 0:
        return 0, np.zeros(N + 1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float64)
    idx = np.arange(P, dtype=np.int64)
    sub = np.minimum((idx * s) // (P - 1), s - 1)
    zc = (sub[:, None] * s + sub[None, :]).reshape(-1).astype(np.int32)   # [iy, ix] -> sy*s + sx
    rowptr = np.arange(N + 1, dtype=np.int32)
    return s * s, rowptr, zc, np.ones(N, np.float64)


def _make_system(asm, dirichlet, b_nodal, s, scale_K=1.0, include_M_sign=-1.0, lam=0.0, meta=None):
    st = asm["K"]
    if scale_K != 1.0:
        st.S *= scale_K
    st.S += asm["C"].S
    if asm["M"] is not None:
        st.S += include_M_sign * lam * asm["M"].S
    rowptr, colind, vals = st.to_csr(dirichlet)
    b = np.array(b_nodal, dtype=np.float64).reshape(-1)
    b[dirichlet.reshape(-1)] = 0.0
    r, zr, zc, zv = indicator_z(asm["order"], asm["n"], s)
    return System(n=b.size, rowptr=rowptr, colind=colind, vals=vals, b=b, r=r,
                  z_rowptr=zr, z_colind=zc, z_vals=zv, meta=meta or {})


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def manufactured_rhs(beta):
    """f for u = sin(pi x) sin(pi y) under -Lap u + beta . grad u."""
    b1, b2 = beta
    pi = math.pi

    def f(x, y):
        return (2 * pi * pi * np.sin(pi * x) * np.sin(pi * y)
                + b1 * pi * np.cos(pi * x) * np.sin(pi * y)
                + b2 * pi * np.sin(pi * x) * np.cos(pi * y))
    return f


def convection_diffusion_manufactured(n: int, beta=(10.0, 10.0), s: int = 4) -> System:
    """Q1, kappa = 1, manufactured u = sin(pi x) sin(pi y), homogeneous Dirichlet."""
    asm = assemble(1, n, beta=beta, f=manufactured_rhs(beta))
    P = n + 1
    X, Y = _node_coords(P)
    meta = dict(kind="q1_manufactured", mesh=n, beta=tuple(beta), s=s,
                u_exact=(np.sin(np.pi * X) * np.sin(np.pi * Y)).reshape(-1))
    return _make_system(asm, _boundary_mask(P), asm["load"], s, meta=meta)


def convection_diffusion_lognormal(n: int, beta, sigma: float, s: int, seed_seq) -> System:
    """Q1, per-element log-normal kappa_e = exp(sigma g_e), b ~ U[-1, 1]."""
    sk, sb = seed_seq.spawn(2)
    g = np.random.default_rng(sk).standard_normal((n, n))
    kappa = np.exp(sigma * g)
    asm = assemble(1, n, kappa_elem=kappa, beta=beta)
    P = n + 1
    b = np.random.default_rng(sb).uniform(-1.0, 1.0, size=P * P)
    meta = dict(kind="q1_lognormal", mesh=n, beta=tuple(beta), sigma=sigma, s=s)
    return _make_system(asm, _boundary_mask(P), b, s, meta=meta)


def sine_modes(P: int, rng, amplitude: float = 1.0, modes: int = 8) -> np.ndarray:
    """amplitude * sum_k a_k sin(p_k pi x) sin(q_k pi y), a_k ~ U[-1,1], p_k, q_k ~ U{1..4}."""
    X, Y = _node_coords(P)
    a = rng.uniform(-1.0, 1.0, size=modes)
    p = rng.integers(1, 5, size=modes)
    q = rng.integers(1, 5, size=modes)
    u = np.zeros((P, P))
    for k in range(modes):
        u += a[k] * np.sin(p[k] * np.pi * X) * np.sin(q[k] * np.pi * Y)
    return amplitude * u


def bratu_jacobian_q2(n: int, lam: float, beta, s: int, seed_seq) -> System:
    """Newton system J(u) du = -R(u) of -Lap u + beta.grad u - lam e^u = 0 (Q2).

    R_i = int grad u_h . grad phi_i + int (beta . grad u_h) phi_i - lam int e^{u_h} phi_i,
    J_ij = int grad phi_j . grad phi_i + int (beta . grad phi_j) phi_i - lam int e^{u_h} phi_j phi_i,
    at u = 0.1 * (8 seeded sine modes).  Dirichlet rows: identity, b_i = 0.
    """
    (su,) = seed_seq.spawn(1)
    P = 2 * n + 1
    u = sine_modes(P, np.random.default_rng(su), amplitude=0.1)
    asm = assemble(2, n, beta=beta, lam=lam, u_nodal=u)
    Ku = _stencil_apply(asm["K"], u) + _stencil_apply(asm["C"], u)
    R = Ku - lam * asm["bratu_load"]
    meta = dict(kind="q2_bratu_jacobian", mesh=n, beta=tuple(beta), lam=lam, s=s)
    return _make_system(asm, _boundary_mask(P), -R, s, lam=lam, meta=meta)


# Config registry: the five benchmark systems of the build.
CONFIGS = {
    1: dict(name="q1_cd_64_manufactured", m=30, rtol=1e-8, max_iters=2000, s=4),
    2: dict(name="q1_cd_1024_lognormal", m=50, rtol=1e-8, max_iters=200000, s=8),
    3: dict(name="q2_bratu_512_jacobian", m=80, rtol=1e-10, max_iters=200000, s=16),
    4: dict(name="q1_cd_batched_512", m=30, rtol=1e-8, max_iters=200000, s=4),
    5: dict(name="q1_cd_2048_differentiable", m=50, rtol=1e-8, max_iters=200000, s=8),
}


def config_seed(k: int) -> np.random.SeedSequence:
    return np.random.SeedSequence(BASE_SEED + k)


def make_config(k: int, mesh: Optional[int] = None) -> System:
    """Build benchmark system k (1, 2, 3 or 5); `mesh` overrides the mesh size
    (same generator at another resolution, for small-scale tests)."""
    ss = config_seed(k)
    if k == 1:
        sysm = convection_diffusion_manufactured(mesh or 64, beta=(10.0, 10.0), s=4)
    elif k == 2:
        sysm = convection_diffusion_lognormal(mesh or 1024, beta=(100.0, 0.0), sigma=1.0, s=8, seed_seq=ss)
    elif k == 3:
        sysm = bratu_jacobian_q2(mesh or 512, lam=5.0, beta=(50.0, 50.0), s=16, seed_seq=ss)
    elif k == 5:
        sysm = differentiable_system(mesh or 2048)
    else:
        raise ValueError("config 4 is a batch: use make_batch()")
    sysm.meta.update(config=k, **{kk: v for kk, v in CONFIGS[k].items() if kk != "s"})
    return sysm


def differentiable_system(n: int, kappa: float = 1.0, s: int = 8):
    """A(kappa) = kappa K + C (Q1, beta = (10, 10)), manufactured load,
    plus the pieces needed to differentiate through kappa: K and C values on
    the same pattern, and a seeded smooth target x_target."""
    beta = (10.0, 10.0)
    asm = assemble(1, n, beta=beta, f=manufactured_rhs(beta))
    P = n + 1
    dmask = _boundary_mask(P)
    # Values of K alone and C alone on the shared pattern (Dirichlet rows: K
    # carries the identity, C carries zeros, so A(kappa) keeps unit Dirichlet
    # rows only at kappa = 1; the pattern split is used for d/dkappa).
    Kst = asm["K"]
    Cst = asm["C"]
    S_K = Kst.S.copy()
    S_C = Cst.S.copy()
    Kst.S = S_K.copy()
    rp, ci, kv = Kst.to_csr(dmask.copy())
    Cst.S = S_C.copy()
    _, _, cv = Cst.to_csr(dmask.copy())
    drows = dmask.reshape(-1)
    row_of = np.repeat(np.arange(P * P), np.diff(rp))
    is_drow = drows[row_of]
    cv = cv.copy()
    cv[is_drow] = 0.0                  # Dirichlet rows: identity carried by K only
    # Keep Dirichlet rows exactly identity for every kappa: A = kappa*K_int + C + D.
    kv_int = kv.copy()
    kv_int[is_drow] = 0.0
    dv = np.zeros_like(kv)
    diag = is_drow & (ci == row_of)
    dv[diag] = 1.0
    vals = kappa * kv_int + cv + dv
    b = asm["load"].reshape(-1).copy()
    b[drows] = 0.0
    r, zr, zc, zv = indicator_z(1, n, s)
    rng = np.random.default_rng(config_seed(5).spawn(1)[0])
    x_target = sine_modes(P, rng, amplitude=1.0).reshape(-1)
    X, Y = _node_coords(P)
    meta = dict(kind="q1_differentiable", mesh=n, beta=beta, s=s, kappa=kappa,
                K_vals=kv_int, C_vals=cv, D_vals=dv, x_target=x_target,
                u_exact=(np.sin(np.pi * X) * np.sin(np.pi * Y)).reshape(-1))
    return System(n=P * P, rowptr=rp, colind=ci, vals=vals, b=b, r=r,
                  z_rowptr=zr, z_colind=zc, z_vals=zv, meta=meta)


@dataclasses.dataclass
class Batch:
    """Block-diagonal concatenation of independent systems."""

    systems: list
    row_off: np.ndarray      # int64 [nsys+1]
    nnz_off: np.ndarray      # int64 [nsys+1]
    zcol_off: np.ndarray     # int64 [nsys+1]
    rowptr: np.ndarray       # int32 [N+1] global nnz offsets
    colind: np.ndarray       # int32 global column indices
    vals: np.ndarray
    b: np.ndarray
    z_rowptr: np.ndarray
    z_colind: np.ndarray     # global deflation-column indices
    z_vals: np.ndarray

    @property
    def nsys(self):
        return len(self.systems)

    @property
    def r_per_sys(self):
        return np.diff(self.zcol_off).astype(np.int32)


def concat_systems(systems) -> Batch:
    ns = len(systems)
    row_off = np.zeros(ns + 1, np.int64)
    nnz_off = np.zeros(ns + 1, np.int64)
    zcol_off = np.zeros(ns + 1, np.int64)
    zn_off = np.zeros(ns + 1, np.int64)
    for i, s in enumerate(systems):
        row_off[i + 1] = row_off[i] + s.n
        nnz_off[i + 1] = nnz_off[i] + s.nnz
        zcol_off[i + 1] = zcol_off[i] + s.r
        zn_off[i + 1] = zn_off[i] + int(s.z_rowptr[-1])
    if nnz_off[-1] >= 2**31 or zn_off[-1] >= 2**31:
        raise ValueError("batch too large for int32 CSR offsets")
    N = int(row_off[-1])
    rowptr = np.empty(N + 1, np.int32)
    z_rowptr = np.empty(N + 1, np.int32)
    rowptr[-1] = nnz_off[-1]
    z_rowptr[-1] = zn_off[-1]
    colind = np.empty(int(nnz_off[-1]), np.int32)
    vals = np.empty(int(nnz_off[-1]), np.float64)
    z_colind = np.empty(int(zn_off[-1]), np.int32)
    z_vals = np.empty(int(zn_off[-1]), np.float64)
    b = np.empty(N, np.float64)
    for i, s in enumerate(systems):
        r0, r1 = row_off[i], row_off[i + 1]
        k0, k1 = nnz_off[i], nnz_off[i + 1]
        rowptr[r0:r1] = s.rowptr[:-1] + k0
        colind[k0:k1] = s.colind + r0
        vals[k0:k1] = s.vals
        b[r0:r1] = s.b
        q0, q1 = zn_off[i], zn_off[i + 1]
        z_rowptr[r0:r1] = s.z_rowptr[:-1] + q0
        z_colind[q0:q1] = s.z_colind + zcol_off[i]
        z_vals[q0:q1] = s.z_vals
    return Batch(systems=systems, row_off=row_off, nnz_off=nnz_off, zcol_off=zcol_off,
                 rowptr=rowptr, colind=colind, vals=vals, b=b,
                 z_rowptr=z_rowptr, z_colind=z_colind, z_vals=z_vals)


def make_batch(nsys: int = 512, mesh_lo: int = 32, mesh_hi: int = 256, s: int = 4) -> Batch:
    """Independent Q1 convection-diffusion systems: n_s ~ U{mesh_lo..mesh_hi},
    log-normal kappa (sigma = 1), beta ~ U[0, 50]^2, b ~ U[-1, 1]."""
    ss = config_seed(4)
    s_mesh, s_beta, s_sys = ss.spawn(3)
    meshes = np.random.default_rng(s_mesh).integers(mesh_lo, mesh_hi + 1, size=nsys)
    betas = np.random.default_rng(s_beta).uniform(0.0, 50.0, size=(nsys, 2))
    subs = s_sys.spawn(nsys)
    systems = []
    for i in range(nsys):
        sy = convection_diffusion_lognormal(int(meshes[i]), beta=tuple(betas[i]), sigma=1.0, s=s, seed_seq=subs[i])
        systems.append(sy)
    batch = concat_systems(systems)
    return batch


def dense(sysm: System) -> np.ndarray:
    """Dense copy of A (small systems only, for tests)."""
    A = np.zeros((sysm.n, sysm.n))
    rows = np.repeat(np.arange(sysm.n), np.diff(sysm.rowptr))
    A[rows, sysm.colind] = sysm.vals
    return A


def dense_z(sysm: System) -> np.ndarray:
    Z = np.zeros((sysm.n, sysm.r))
    rows = np.repeat(np.arange(sysm.n), np.diff(sysm.z_rowptr))
    Z[rows, sysm.z_colind] = sysm.z_vals
    return Z


def from_dense(A: np.ndarray, b: np.ndarray, Z: Optional[np.ndarray] = None, keep_zeros=False) -> System:
    """CSR System from dense arrays (tests)."""
    n = A.shape[0]
    mask = np.ones_like(A, dtype=bool) if keep_zeros else (A != 0)
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n + 1, np.int32)
    rowptr[1:] = np.cumsum(counts)
    rr, cc = np.nonzero(mask)
    if Z is None:
        Z = np.zeros((n, 0))
    zm = Z != 0
    zrp = np.zeros(n + 1, np.int32)
    zrp[1:] = np.cumsum(zm.sum(axis=1))
    zr, zcol = np.nonzero(zm)
    return System(n=n, rowptr=rowptr, colind=cc.astype(np.int32), vals=A[rr, cc].astype(np.float64),
                  b=np.asarray(b, np.float64).copy(), r=Z.shape[1], z_rowptr=zrp,
                  z_colind=zcol.astype(np.int32), z_vals=Z[zr, zcol].astype(np.float64))
