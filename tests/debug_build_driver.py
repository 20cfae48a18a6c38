"""Runs the solver paths on the bounds-checking build of the library
(GMRES_LIB names libgmres_mi355x_debug.so; every device index check that
fails turns the call into GMRES_EDEVICE) and compares each result with the
oracle at the parity gates of the release tests.  Started in a child process
by tests/test_gpu_debug_build.py; prints one line per case and exits
non-zero on the first failure.
"""
import copy
import os
import sys

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import oracle  # noqa: E402
from paper_1906_04051_amd import gmres as G  # noqa: E402
from paper_1906_04051_amd import workloads as W  # noqa: E402


def rel(a, b):
    return max(float(np.linalg.norm(a - b) / np.linalg.norm(b)),
               float(np.abs(a - b).max() / np.abs(b).max()))


def say(*a):
    print(*a, flush=True)


def check(cond, what):
    if not cond:
        say("FAILED:", what)
        sys.exit(1)


def heavy_z(s, R, every, per_row, seed):
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


def main():
    path = G.load_library()._name
    check(path.endswith("libgmres_mi355x_debug.so"), f"loaded {path}")
    say("library", path)
    s = W.make_config(1, mesh=40)
    ref = oracle.gmres(s, 30, 1e-8, 4000)
    for kw in (dict(), dict(ortho=0), dict(ortho=2), dict(spmv_lanes=8), dict(spmv_lanes=-256)):
        plan, d = G.plan_for(s, m=30, rtol=1e-8, max_iters=4000, **kw)
        x, info = plan.solve(d["b"])
        e = rel(x.cpu().numpy(), ref.x)
        say("fp64", kw, info["status_name"], info["iters"], ref.iters, f"{e:.2e}")
        check(info["status_name"] == "OK" and abs(info["iters"] - ref.iters) <= 1 and e <= 1e-8, kw)
    plan, d = G.plan_for(s, m=30, rtol=1e-8, max_iters=4000, precision="mixed_f16")
    x, info = plan.solve(d["b"])
    say("mixed f16", info["status_name"], info["rel_res_true"])
    check(info["status_name"] == "OK" and info["rel_res_true"] <= 1e-8 * (1 + 1e-6), "mixed")
    # General Z: multi-entry rows, more than 64 columns per row block.
    t = heavy_z(s, 80, 3, 3, 5)
    reft = oracle.gmres(t, 20, 0.0, 60)
    plan, d = G.plan_for(t, m=20, rtol=0.0, max_iters=60)
    x, info = plan.solve(d["b"])
    e = rel(x.cpu().numpy(), reft.x)
    say("general Z fixed count", info["iters"], f"{e:.2e}")
    check(info["iters"] == 60 and e <= 1e-8, "general Z")
    # Adjoint.
    sa = W.make_config(1, mesh=24)
    plan, d = G.plan_for(sa, need_adjoint=True, m=30, rtol=1e-12, max_iters=4000)
    x, _ = plan.solve(d["b"])
    gx = torch.from_numpy(np.random.default_rng(3).standard_normal(sa.n)).cuda()
    gb, gv, info = plan.adjoint(x, gx)
    ra = oracle.adjoint(sa, x.cpu().numpy(), gx.cpu().numpy(), 30, 1e-12, 4000)
    e1, e2 = rel(gb.cpu().numpy(), ra["grad_b"]), rel(gv.cpu().numpy(), ra["grad_vals"])
    say("adjoint", info["status_name"], f"{e1:.2e} {e2:.2e}")
    check(info["status_name"] == "OK" and e1 <= 1e-8 and e2 <= 1e-8, "adjoint")
    # Batched.
    ss = W.config_seed(77)
    sub = ss.spawn(6)
    systems = [W.convection_diffusion_lognormal(m_, beta=(10.0, 5.0), sigma=1.0, s=2, seed_seq=sub[i])
               for i, m_ in enumerate((7, 12, 20, 9, 33, 16))]
    batch = W.concat_systems(systems)
    for lanes in (4, 16):
        plan, d = G.plan_for(batch, m=20, rtol=1e-8, max_iters=4000, batch_lanes=lanes)
        xb, infos = plan.solve_batched(d["b"])
        xb = xb.cpu().numpy()
        for i, si in enumerate(systems):
            rb = oracle.gmres(si, 20, 1e-8, 4000)
            e = rel(xb[batch.row_off[i]:batch.row_off[i + 1]], rb.x)
            check(infos[i]["status_name"] == "OK" and e <= 1e-8, f"batched {lanes} {i} {e}")
        say("batched lanes", lanes, "ok")
    # Batched with continuation plans: every system leaves after one cycle.
    plan, d = G.plan_for(batch, m=20, rtol=1e-8, max_iters=4000)
    subs = []
    for i, si in enumerate(systems):
        sp, _ = G.plan_for(si, m=20, rtol=1e-8, max_iters=4000)
        plan.attach(i, sp, 20)
        subs.append(sp)
    xb, infos = plan.solve_batched(d["b"])
    xb = xb.cpu().numpy()
    for i, si in enumerate(systems):
        rb = oracle.gmres(si, 20, 1e-8, 4000)
        e = rel(xb[batch.row_off[i]:batch.row_off[i + 1]], rb.x)
        check(infos[i]["status_name"] == "OK" and e <= 1e-8 and abs(infos[i]["iters"] - rb.iters) <= 1,
              f"batched continuation {i} {e} {infos[i]['iters']} {rb.iters}")
    say("batched continuations ok")
    # Block GMRES, fixed count.
    sb = W.make_config(1, mesh=20)
    sb = copy.copy(sb)
    sb.r = 0
    sb.z_rowptr = np.zeros(sb.n + 1, np.int32)
    sb.z_colind = np.zeros(0, np.int32)
    sb.z_vals = np.zeros(0)
    B = np.random.default_rng(11).standard_normal((sb.n, 4))
    rbk = oracle.bgmres(sb.rowptr, sb.colind, sb.vals, B, 6, 0.0, 12)
    plan, d = G.plan_for(sb, m=8, rtol=0.0, max_iters=12)
    X, info = plan.solve_block(torch.from_numpy(B).cuda(), 6)
    e = rel(X.cpu().numpy(), rbk.x)
    say("block", info["iters"], f"{e:.2e}")
    check(e <= 1e-8, "block")
    # Block GMRES with the indicator deflation basis, fixed count.
    sz = W.make_config(1, mesh=20)
    rbz = oracle.bgmres(sz.rowptr, sz.colind, sz.vals, B, 6, 0.0, 12,
                        z=(sz.r, sz.z_rowptr, sz.z_colind, sz.z_vals))
    plan, d = G.plan_for(sz, m=8, rtol=0.0, max_iters=12)
    X, info = plan.solve_block(torch.from_numpy(B).cuda(), 6)
    e = rel(X.cpu().numpy(), rbz.x)
    say("deflated block", info["iters"], f"{e:.2e}")
    check(e <= 1e-8, "deflated block")
    # Adaptive deflation, fixed count.
    sd = W.make_config(1, mesh=30)
    sd = copy.copy(sd)
    sd.r = 0
    sd.z_rowptr = np.zeros(sd.n + 1, np.int32)
    sd.z_colind = np.zeros(0, np.int32)
    sd.z_vals = np.zeros(0)
    rd = oracle.dgmres(sd, 20, 0.0, 80, rmax=6)
    plan, d = G.plan_for(sd, m=20, rtol=0.0, max_iters=80, adapt_rmax=6)
    x, info = plan.solve(d["b"])
    e = rel(x.cpu().numpy(), rd.x)
    say("adaptive", info["defl_r"], rd.r, f"{e:.2e}")
    check(info["defl_r"] == rd.r and e <= 1e-8, "adaptive")
    say("debug build: all cases passed")


if __name__ == "__main__":
    main()
