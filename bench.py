"""Benchmark: time-to-rtol of deflated GMRES(50) on one MI355X.

Default workload (--config 5): the 2048 x 2048 Q1 convection-diffusion system
of the differentiable-solve configuration (4,198,401 unknowns, 37,761,025
stored entries), diffusion kappa = 1, beta = (10, 10), manufactured load,
64 subdomain-indicator deflation vectors, GMRES(50), rtol 1e-8, zero initial
guess.  Synthetic, seeded inputs, resident in HBM before timing.

One step = the plain FP64 solve followed by the mixed-precision solve (FP32
inner GMRES with an FP16-stored basis inside FP64 iterative refinement) of the
same system, both to a true FP64 relative residual <= 1e-8.  `value` is the
median time-to-rtol of the mixed solve; the FP64 time and the ratio are
reported beside it, and (outside the timed steps) the adjoint solve of the
same plan.  --config 2 / 3 run the other single-system workloads the same
way; --config 4 solves the 512-system batch (solves/s, p50/p99).

Prints one JSON line.  `roofline` covers the dominant Arnoldi kernel (timed
with HIP events on the solver's stream during the timed steps);
`cpu_baseline` times the CPU oracle on a bounded sample of the same solve.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time-to-rtol 1e-8 (s) + SpMV/Arnoldi HBM GB/s; mixed vs FP64 GMRES"
HBM_PEAK_GBS = 8000.0

# HBM traffic of the dominant kernel per workload (FP64 first Gram-Schmidt
# sweep of the two-sweep variant over a restart cycle of GMRES(50)) from
# FETCH_SIZE and WRITE_SIZE counter runs of `bench.py --pmc-sample`, each
# scaled by what the same counter reads for a 512 MiB device copy.  Valid only
# while the kernel sources hash to `sources_sha256`; None until measured.
TRAFFIC = {
    5: {"kind": "pass1_lag",
        "sources_sha256": "c25a2e2286a92d6786a47946ce0578b3f3cc6d7c1974981fab29dd4787a827c1",
        "bytes_per_launch": 1076.4e6},   # 1,008.6 MB read + 67.8 MB written (98 launches)
}
KERNEL_SOURCES = ("paper_1906_04051_amd/csrc/krylov.hip", "paper_1906_04051_amd/csrc/common.hpp",
                  "paper_1906_04051_amd/csrc/internal.hpp")


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_info():
    """CPU model, logical CPUs and OpenMP setting of the host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(cpu_model=model, nproc=os.cpu_count(), omp_num_threads=os.environ.get("OMP_NUM_THREADS"))


def stream_ceilings():
    """What plain streaming library kernels (torch) reach on this GPU, beside
    the 8 TB/s peak: a 1 GiB device copy (bytes read + written) and a 1 GiB
    sum (bytes read), each the best of 10 timed with events."""
    import torch
    n = (1 << 30) // 8
    a = torch.empty(n, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    s = torch.empty((), dtype=torch.float64, device="cuda")

    def best_ms(fn):
        fn()
        best = 1e30
        for _ in range(10):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        return best

    copy_ms = best_ms(lambda: b.copy_(a))
    sum_ms = best_ms(lambda: torch.sum(a, dim=0, out=s))
    del a, b, s
    torch.cuda.empty_cache()
    return (2.0 * (1 << 30) / (copy_ms * 1e-3) / 1e9, (1 << 30) / (sum_ms * 1e-3) / 1e9)


def cpu_baseline(sysm, m, fp64_iters, sample_iters, adapt_rmax=0):
    """Oracle (plain C, FP64, one thread) on the same system: its setup (copy
    of A and Z, A Z, E and its LU, the initial residual) timed alone with a
    zero-step run, then `sample_iters` inner steps; the per-step time is
    scaled to the FP64 solve's iteration count (setup excluded, as on the
    GPU)."""
    import oracle
    run = (lambda k: oracle.dgmres(sysm, m, 0.0, k, rmax=adapt_rmax)) if adapt_rmax > 0 else \
          (lambda k: oracle.gmres(sysm, m, 0.0, k))
    t0 = time.perf_counter()
    run(0)
    setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    res = run(sample_iters)
    dt = time.perf_counter() - t0
    per_iter = max(dt - setup, 1e-9) / max(res.iters, 1)
    return dict(value=per_iter * fp64_iters, unit="s", cores=1, kind="oracle",
                sample=(f"{res.iters} fixed-count deflated GMRES({m}) steps of the same "
                        f"{sysm.n:,}-unknown system ({dt:.1f} s incl. {setup:.1f} s setup); the "
                        f"per-step time scaled to the {fp64_iters} steps the FP64 solve needs "
                        f"to reach the tolerance (extrapolated; setup excluded)"),
                seconds_per_iter=per_iter, sample_seconds=dt, setup_seconds=setup,
                threads=1, **host_info())


def pmc_sample(sysm, d, m, tuned, tuned_mixed=None):
    """Two fixed-count restart cycles of the FP64 solve and two of the FP16-
    basis inner solve (the timed launch configuration) and one 512 MiB device
    copy (512 MiB read + 512 MiB written), for hardware-counter runs."""
    import torch
    from paper_1906_04051_amd import gmres as G
    q = G.Plan(d["rowptr"], d["colind"], d["vals"], d["z_rowptr"], d["z_colind"], d["z_vals"],
               r=sysm.r, precision="fp64", m=m, rtol=0.0, max_iters=2 * m,
               spmv_lanes=tuned["spmv_lanes"], num_blocks=tuned["num_blocks"])
    q.set_timing(True)
    _, info = q.solve(d["b"])
    kt = q.kernel_times()
    q.close()
    per = {"fp64." + k: dict(launches=int(v["launches"]), bytes_per_launch=v["bytes"] / max(v["launches"], 1),
                             avg_us=1000 * v["ms"] / max(v["launches"], 1)) for k, v in kt.items()}
    if tuned_mixed:
        # One refinement whose inner FP16-basis solve runs exactly two cycles.
        qm = G.Plan(d["rowptr"], d["colind"], d["vals"], d["z_rowptr"], d["z_colind"], d["z_vals"],
                    r=sysm.r, precision="mixed_f16", m=m, rtol=1e-30, max_iters=2 * m, inner_rtol=1e-30,
                    inner_max_iters=2 * m, max_refine=1, spmv_lanes=tuned_mixed["spmv_lanes"],
                    num_blocks=tuned_mixed["num_blocks"])
        qm.set_timing(True)
        qm.solve(d["b"])
        for k, v in qm.kernel_times().items():
            per["mixed." + k] = dict(launches=int(v["launches"]), bytes_per_launch=v["bytes"] / max(v["launches"], 1),
                                     avg_us=1000 * v["ms"] / max(v["launches"], 1))
        qm.close()
    src = torch.empty(512 << 20, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"pmc_sample": per, "iters": info["iters"], "copy_bytes_each_way": 512 << 20,
                      "kernel_sources_sha256": kernel_sources_sha256()}), flush=True)


def bratu_newton(args):
    """Newton on the 3-D Bratu problem (lam = 6.8); one JSON line with the GPU
    linear-solve times of every Newton step."""
    import numpy as np
    from paper_1906_04051_amd import bratu3d as B
    n = args.bratu
    t0 = time.perf_counter()
    mesh = B.build_mesh(n, verbose=True)
    log(f"[bench] Bratu mesh n={n}: {mesh.N} unknowns, {len(mesh.colind)} stored entries "
        f"({time.perf_counter() - t0:.1f} s)")
    solve, plan = B.gpu_solver(mesh, m=50, rtol=1e-8, max_iters=200000, adapt_rmax=20)
    u, hist = B.newton(mesh, solve, tol=1e-8, verbose=True)
    solve_s = sum(h["solve_ms"] for h in hist) / 1000.0
    out = {
        "metric": "Newton on 3-D Bratu: GPU linear-solve time (s), GMRES(50) adaptive deflation",
        "value": solve_s, "unit": "s", "n_gpus": 1, "higher_is_better": False, "scaling": "strong",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"bratu3d_q2hex_{n}x{n}x{n}_lam6.8", "unknowns": mesh.N,
                   "nnz": int(len(mesh.colind)), "restart_m": 50, "adapt_rmax": 20,
                   "rtol_linear": 1e-8, "newton_tol": 1e-8},
        "newton_steps": len(hist),
        "gmres_iters": [h["iters"] for h in hist],
        "solve_s": [h["solve_ms"] / 1000.0 for h in hist],
        "assembly_s": [h["assembly_s"] for h in hist],
        "du": [h["du"] for h in hist],
        "status": [h["status"] for h in hist],
        "u_max": float(np.max(u)),
    }
    print(json.dumps(out), flush=True)


def bratu_fixed(args):
    """The paper's timing protocol on its own workload (Sec. 4): the Jacobian of
    the 3-D Bratu problem at u = 0 (first Newton system), GMRES(50) with
    adaptive spectral deflation (r_max 20), exactly 100 restart cycles and no
    termination test.  One JSON line with the solve time, the kernel times and
    the roofline of the dominant kernel class."""
    import numpy as np
    import torch
    from paper_1906_04051_amd import bratu3d as B
    from paper_1906_04051_amd import gmres as G
    n = args.bratu_fixed
    m, cycles, rmax = 50, args.bratu_cycles, 20
    t0 = time.perf_counter()
    mesh = B.build_mesh(n, verbose=True)
    sysm = B.system_at(mesh, np.zeros(mesh.N))
    log(f"[bench] Bratu mesh n={n}: {mesh.N} unknowns, {sysm.nnz} stored entries "
        f"({time.perf_counter() - t0:.1f} s)")
    plan, d = G.plan_for(sysm, m=m, rtol=0.0, max_iters=m * cycles, adapt_rmax=rmax)
    tuned = plan.autotune()
    log(f"[bench] autotune: {tuned}")
    b = d["b"]
    x = torch.empty_like(b)
    timing = 0 if args.no_timing else max(args.timing_period, 1)
    for w in range(args.warmup):
        plan.set_timing(0)
        _, info = plan.solve(b, out=x)
        log(f"[bench] warmup: iters {info['iters']} rel_res_true {info['rel_res_true']:.3e}")
    times, ktot = [], {}
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for step in range(args.steps):
        plan.set_timing(timing)
        t1 = time.perf_counter()
        _, info = plan.solve(b, out=x)
        times.append(time.perf_counter() - t1)
        for kk, v in (plan.kernel_times() if timing else {}).items():
            a = ktot.setdefault(kk, dict(launches=0.0, ms=0.0, bytes=0.0))
            for f in ("launches", "ms", "bytes"):
                a[f] += v[f]
        log(f"[bench] step {step}: {times[-1]:.3f} s iters {info['iters']} "
            f"rel_res_true {info['rel_res_true']:.3e} r {info['defl_r']}")
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    med = float(np.median(times))
    out = {
        "metric": f"GMRES(50) x {cycles} restarts on the 3-D Bratu Jacobian: solve time (s)",
        "value": med, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1000.0 * total / max(args.steps, 1), "higher_is_better": False,
        "scaling": "strong", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"bratu3d_q2hex_{n}x{n}x{n}_lam6.8_jacobian_u0", "unknowns": mesh.N,
                   "nnz": int(sysm.nnz), "restart_m": m, "restarts": cycles, "adapt_rmax": rmax,
                   "spmv_lanes": tuned["spmv_lanes"], "num_blocks": tuned["num_blocks"]},
        "iters": info["iters"], "rel_res_true": info["rel_res_true"], "defl_r": info["defl_r"],
        "us_per_iter": 1e6 * med / max(info["iters"], 1),
    }
    if ktot:
        per = {kk: dict(launches=int(v["launches"]), avg_us=1000 * v["ms"] / v["launches"],
                        GBs=v["bytes"] / (v["ms"] * 1e6), total_ms=v["ms"])
               for kk, v in ktot.items() if v["launches"] > 0}
        out["kernels"] = per
        dom = max(per, key=lambda kk: per[kk]["total_ms"])
        v = ktot[dom]
        achieved = v["bytes"] / (v["ms"] * 1e6)
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                           "traffic_unit": "bytes/launch", "kernel": dom,
                           "launches": int(v["launches"]), "avg_launch_us": 1000 * v["ms"] / v["launches"],
                           "bytes_per_launch_avg": v["bytes"] / v["launches"]}
    if not args.no_cpu_baseline:
        import oracle
        k = args.cpu_sample_iters
        t1 = time.perf_counter()
        res = oracle.dgmres(sysm, m, 0.0, k, rmax=rmax)
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = dict(
            value=dt / max(res.iters, 1) * m * cycles, unit="s", cores=1, kind="oracle",
            sample=(f"{res.iters} fixed-count steps of the same GMRES(50) with adaptive deflation "
                    f"incl. setup ({dt:.1f} s), scaled to {m * cycles} steps"),
            sample_seconds=dt)
    print(json.dumps(out), flush=True)


def block_rhs(args):
    """Several right-hand sides at once: block GMRES(m_block) with k = --block
    columns on the kappa = 1 FEM system (no deflation basis), fixed count
    (the paper's protocol: no termination test).  Reports the block-step rate,
    the same work per right-hand side as single-vector GMRES(50) steps, and
    the roofline of the dominant block kernel (HIP events in its dispatches)."""
    import copy
    import numpy as np
    import torch
    from paper_1906_04051_amd import gmres as G
    from paper_1906_04051_amd import workloads as W
    k, mb, steps_fixed = args.block, args.block_m, args.block_steps
    log(f"[bench] generating the kappa = 1 problem at mesh {args.mesh}")
    sysm = copy.copy(W.make_config(1, mesh=args.mesh))
    if not args.block_defl:
        sysm.r = 0
        sysm.z_rowptr = np.zeros(sysm.n + 1, np.int32)
        sysm.z_colind = np.zeros(0, np.int32)
        sysm.z_vals = np.zeros(0)
    rng = np.random.default_rng(20190610)
    B = rng.standard_normal((sysm.n, k))
    plan, d = G.plan_for(sysm, m=50, rtol=0.0, max_iters=steps_fixed)
    Bt = torch.from_numpy(B).cuda()
    X = torch.empty_like(Bt)
    timing = 0 if args.no_timing else 1
    for _ in range(args.warmup):
        plan.set_timing(0)
        plan.solve_block(Bt, mb, out=X)
    times, ktot = [], {}
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for step in range(args.steps):
        plan.set_timing(timing)
        t1 = time.perf_counter()
        _, info = plan.solve_block(Bt, mb, out=X)
        times.append(time.perf_counter() - t1)
        for kk, v in (plan.kernel_times() if timing else {}).items():
            if kk.startswith("block") and v["launches"] > 0:
                a = ktot.setdefault(kk, dict(launches=0.0, ms=0.0, bytes=0.0))
                for f in ("launches", "ms", "bytes"):
                    a[f] += v[f]
        log(f"[bench] step {step}: {times[-1]:.3f} s block steps {info['iters']} cycles {info['cycles']} "
            f"max rel res {info['rel_res_true']:.3e}")
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    med = float(np.median(times))
    # Single-vector reference on the same operator: plain GMRES(50), fixed count.
    single_steps = 100
    sp_ = G.Plan(d["rowptr"], d["colind"], d["vals"], d["z_rowptr"], d["z_colind"], d["z_vals"], r=0,
                 precision="fp64", m=50, rtol=0.0, max_iters=single_steps)
    sp_.autotune()
    b0 = Bt[:, 0].contiguous()
    x0 = torch.empty_like(b0)
    sp_.solve(b0, out=x0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, sinfo = sp_.solve(b0, out=x0)
    torch.cuda.synchronize()
    single_s = (time.perf_counter() - t1) / max(sinfo["iters"], 1)
    out = {
        "metric": f"block GMRES({mb}) with {k} right-hand sides: time per block step (s)",
        "value": med / max(info["iters"], 1), "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1000.0 * total / max(args.steps, 1),
        "higher_is_better": False, "scaling": "strong", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"q1_convection_diffusion_{args.mesh}x{args.mesh}_kappa1_{k}rhs",
                   "unknowns": sysm.n, "nnz": sysm.nnz, "rhs": k, "block_steps_per_cycle": mb,
                   "block_steps": steps_fixed, "deflation_vectors": int(sysm.r)},
        "solve_s": med, "block_steps": info["iters"], "cycles": info["cycles"],
        "rhs_step_equivalent_us": 1e6 * med / max(info["iters"], 1) / k,
        "single_vector_gmres50_step_us": 1e6 * single_s,
    }
    if ktot:
        per = {kk: dict(launches=int(v["launches"]), avg_us=1000 * v["ms"] / v["launches"],
                        GBs=v["bytes"] / (v["ms"] * 1e6), total_ms=v["ms"]) for kk, v in ktot.items()}
        out["kernels"] = per
        dom = max(per, key=lambda kk: per[kk]["total_ms"])
        v = ktot[dom]
        achieved = v["bytes"] / (v["ms"] * 1e6)
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS, "traffic": None, "traffic_unit": "bytes/launch",
                           "kernel": dom, "launches": int(v["launches"]),
                           "avg_launch_us": 1000 * v["ms"] / v["launches"],
                           "bytes_per_launch_avg": v["bytes"] / v["launches"]}
    if not args.no_cpu_baseline:
        import oracle
        t1 = time.perf_counter()
        res = oracle.bgmres(sysm.rowptr, sysm.colind, sysm.vals, B, mb, 0.0, 1)
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = dict(
            value=dt / max(res.iters, 1), unit="s", cores=1, kind="oracle",
            sample=f"{res.iters} block step of the same solve (k = {k}) incl. the starting block QR "
                   f"({dt:.1f} s); per block step", sample_seconds=dt)
    print(json.dumps(out), flush=True)


def batched_config4(args):
    """Config 4: 512 independent Q1 systems (meshes 32^2 .. 256^2, own seeded
    coefficients, beta and rhs) solved by one call of the batched solver
    (GMRES(30), 16 deflation vectors each, rtol 1e-8).  Systems of at least
    --cont-rows rows get continuation plans: one still running after
    --cont-work row-steps leaves the persistent launch at a restart and goes on
    on the multi-workgroup engine within the same call.  Reports solves/s over
    the whole call and p50/p99 of the per-system solve times."""
    import numpy as np
    import torch
    from paper_1906_04051_amd import gmres as G
    from paper_1906_04051_amd import workloads as W
    t0 = time.perf_counter()
    batch = W.make_batch(512)
    log(f"[bench] batch: {batch.nsys} systems, {batch.rowptr.size - 1} rows, {int(batch.rowptr[-1])} "
        f"stored entries ({time.perf_counter() - t0:.1f} s)")
    plan, d = G.plan_for(batch, m=30, rtol=1e-8, max_iters=200000)
    tuned = plan.autotune()
    log(f"[bench] autotune: {tuned}")
    steps_at = {}
    if args.cont_rows > 0:
        # Continuation plans: a system of at least cont_rows rows that is still
        # running after cont_work row-steps goes on on the multi-workgroup
        # single-system engine (outside the timed region: plan construction).
        t1 = time.perf_counter()
        subs = G.attach_continuations(plan, batch, args.cont_rows, args.cont_work,
                                      m=30, rtol=1e-8, max_iters=200000)
        rows = np.diff(batch.row_off)
        steps_at = {s: 30 * max(1, int(np.ceil(args.cont_work / (float(rows[s]) * 30)))) for s in subs}
        log(f"[bench] {len(subs)} continuation plans ({time.perf_counter() - t1:.1f} s)")
    b = d["b"]
    x = torch.empty_like(b)
    for _ in range(args.warmup):
        _, infos = plan.solve_batched(b, out=x)
    walls, per_sys = [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for step in range(args.steps):
        t1 = time.perf_counter()
        _, infos = plan.solve_batched(b, out=x)
        walls.append(time.perf_counter() - t1)
        per_sys = [i["solve_ms"] / 1000.0 for i in infos]
        bad = [i for i in infos if i["status_name"] != "OK"]
        log(f"[bench] step {step}: {walls[-1]:.3f} s, max rel res "
            f"{max(i['rel_res_true'] for i in infos):.3e}, not converged {len(bad)}")
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    med = float(np.median(walls))
    its = np.array([i["iters"] for i in infos])
    out = {
        "metric": "batched deflated GMRES(30): 512 systems to rtol 1e-8, solves/s",
        "value": batch.nsys / med, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1000.0 * total / max(args.steps, 1),
        "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "q1_convection_diffusion_batch_512_mesh32to256", "systems": batch.nsys,
                   "unknowns_total": int(batch.rowptr.size - 1), "nnz_total": int(batch.rowptr[-1]),
                   "restart_m": 30, "deflation_vectors_each": 16, "rtol": 1e-8,
                   "batch_wg": tuned["batch_wg"], "batch_lanes": tuned["batch_lanes"],
                   "continuation_min_rows": args.cont_rows, "continuation_row_steps": args.cont_work},
        "continued_systems": sum(1 for s, k in steps_at.items() if infos[s]["iters"] > k),
        "call_s": med,
        "solve_s_p50": float(np.percentile(per_sys, 50)), "solve_s_p99": float(np.percentile(per_sys, 99)),
        "solve_s_max": float(np.max(per_sys)),
        "iters_p50": float(np.percentile(its, 50)), "iters_max": int(its.max()),
        "max_rel_res_true": max(i["rel_res_true"] for i in infos),
    }
    if not args.no_cpu_baseline:
        import oracle
        # The oracle on the first systems (largest work is random, so a prefix
        # is a fair sample), scaled to all 512.
        t1 = time.perf_counter()
        k = 0
        while k < batch.nsys and time.perf_counter() - t1 < 15.0:
            oracle.gmres(batch.systems[k], 30, 1e-8, 200000)
            k += 1
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = dict(value=k / dt, unit="solves/s", cores=1, kind="oracle",
                                   sample=f"the first {k} systems of the batch solved to rtol 1e-8 one "
                                          f"after another ({dt:.1f} s)", sample_seconds=dt,
                                   threads=1, **host_info())
        # The same oracle on all host cores: independent systems in parallel
        # (one oracle call per thread at a time; the calls release the GIL).
        import concurrent.futures as cf
        nt = max(1, min(16, os.cpu_count() or 1))
        t1 = time.perf_counter()
        done = 0
        with cf.ThreadPoolExecutor(max_workers=nt) as ex:
            futs = []
            nxt = 0
            while nxt < min(batch.nsys, nt):
                futs.append(ex.submit(oracle.gmres, batch.systems[nxt], 30, 1e-8, 200000))
                nxt += 1
            while futs:
                fin, pend = cf.wait(futs, return_when=cf.FIRST_COMPLETED)
                done += len(fin)
                futs = list(pend)
                for _ in fin:
                    if nxt < batch.nsys and time.perf_counter() - t1 < 15.0:
                        futs.append(ex.submit(oracle.gmres, batch.systems[nxt], 30, 1e-8, 200000))
                        nxt += 1
        dt2 = time.perf_counter() - t1
        out["cpu_baseline_all_cores"] = dict(
            value=done / dt2, unit="solves/s", cores=nt, kind="oracle",
            sample=f"the first {done} systems of the batch solved to rtol 1e-8 on {nt} threads, one "
                   f"system per thread at a time ({dt2:.1f} s)", sample_seconds=dt2, threads=nt,
            **host_info())
    print(json.dumps(out), flush=True)


def single_config(args):
    """Configs 2, 3 and 5: FP64 and mixed-precision solves of one system to
    its tolerance (one step = both), kernel times, roofline, CPU baseline."""
    import numpy as np
    import torch
    from paper_1906_04051_amd import gmres as G
    from paper_1906_04051_amd import workloads as W
    k = args.config
    cfg = W.CONFIGS[k]
    m, rtol = cfg["m"], cfg["rtol"]
    mixed_basis = args.mixed_basis or ("f32" if k == 3 else "f16")
    inner = args.inner_rtol if args.inner_rtol else (1e-3 if mixed_basis == "f16" else 1e-5)
    t0 = time.perf_counter()
    log(f"[bench] generating config {k}" + (f" at mesh {args.mesh}" if args.mesh else ""))
    sysm = W.make_config(k, mesh=args.mesh)
    d = G.upload(sysm)
    log(f"[bench] {sysm.n} unknowns, {sysm.nnz} stored entries ({time.perf_counter() - t0:.1f} s)")
    common = dict(m=m, rtol=rtol, max_iters=200000, ortho=args.ortho)
    plans = {}
    if args.only in ("both", "fp64"):
        plans["fp64"] = G.Plan(d["rowptr"], d["colind"], d["vals"], d["z_rowptr"], d["z_colind"],
                               d["z_vals"], r=sysm.r, precision="fp64", **common)
    if args.only in ("both", "mixed"):
        plans["mixed"] = G.Plan(d["rowptr"], d["colind"], d["vals"], d["z_rowptr"], d["z_colind"],
                                d["z_vals"], r=sysm.r, precision="mixed_" + mixed_basis,
                                need_adjoint=(k == 5 and not args.no_adjoint),
                                inner_rtol=inner, inner_max_iters=100000, max_refine=40, **common)
    tuned = {}
    for name, p in plans.items():
        tuned[name] = p.autotune()
        log(f"[bench] autotune {name}: {tuned[name]}")
    b = d["b"]
    if args.pmc_sample:
        pmc_sample(sysm, d, m, tuned["fp64"], tuned.get("mixed"))
        return
    x = torch.empty_like(b)

    def run(name, timing):
        p = plans[name]
        p.set_timing(timing)
        t1 = time.perf_counter()
        _, info = p.solve(b, out=x)
        dt = time.perf_counter() - t1
        kt = p.kernel_times() if timing else None
        return dt, info, kt

    for _ in range(args.warmup):
        for name in plans:
            dt, info, _ = run(name, False)
            log(f"[bench] warmup {name}: {dt:.3f} s iters {info['iters']} status {info['status_name']} "
                f"rel_res_true {info['rel_res_true']:.3e}")
    timing = 0 if args.no_timing else max(args.timing_period, 1)
    times = {kk: [] for kk in plans}
    infos, ktot = {}, {}
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for step in range(args.steps):
        for name in plans:
            dt, info, kt = run(name, timing)
            times[name].append(dt)
            infos[name] = info
            for kk, v in (kt or {}).items():
                a = ktot.setdefault((name, kk), dict(launches=0.0, ms=0.0, bytes=0.0))
                for fld in ("launches", "ms", "bytes"):
                    a[fld] += v[fld]
            log(f"[bench] step {step} {name}: {dt:.3f} s iters {info['iters']} "
                f"refinements {info['refinements']} status {info['status_name']} "
                f"rel_res_true {info['rel_res_true']:.3e}")
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    med = {kk: float(np.median(v)) for kk, v in times.items()}
    headline = "mixed" if "mixed" in med else "fp64"
    names = {2: f"q1_convection_diffusion_{args.mesh or 1024}x{args.mesh or 1024}_lognormal",
             3: f"q2_bratu_jacobian_{args.mesh or 512}x{args.mesh or 512}",
             5: f"q1_convection_diffusion_{args.mesh or 2048}x{args.mesh or 2048}_kappa1_manufactured"}
    out = {
        "metric": METRIC, "value": med[headline], "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1000.0 * total / max(args.steps, 1),
        "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
        "dtype": (f"f32/{mixed_basis}+f64" if headline == "mixed" else "f64"), "data": "synthetic",
        "config": {"workload": names[k], "unknowns": sysm.n, "nnz": sysm.nnz, "restart_m": m,
                   "deflation_vectors": sysm.r, "rtol": rtol, "step": "+".join(plans),
                   "ortho": args.ortho, "mixed_basis": mixed_basis, "inner_rtol": inner},
    }
    for kk in plans:
        out[f"time_to_rtol_{kk}_s"] = med[kk]
        out[f"iters_{kk}"] = infos[kk]["iters"]
        out[f"rel_res_true_{kk}"] = infos[kk]["rel_res_true"]
        out[f"us_per_iter_{kk}"] = 1e6 * med[kk] / max(infos[kk]["iters"], 1)
    if "mixed" in med and "fp64" in med:
        out["mixed_speedup_vs_fp64"] = med["fp64"] / med["mixed"]
        out["refinements_mixed"] = infos["mixed"]["refinements"]
    if ktot:
        per = {}
        for (name, kk), v in ktot.items():
            if v["launches"] > 0:
                per[f"{name}.{kk}"] = dict(launches=int(v["launches"]), avg_us=1000 * v["ms"] / v["launches"],
                                           GBs=v["bytes"] / (v["ms"] * 1e6), total_ms=v["ms"])
        out["kernels"] = per
        # Dominant kernel: most total time in the FP64 solve (else the mixed one).
        src = "fp64" if "fp64" in plans else "mixed"
        cand = {kk: v for (nm, kk), v in ktot.items() if nm == src and v["launches"] > 0}
        dom = max(cand, key=lambda kk: cand[kk]["ms"])
        v = cand[dom]
        achieved = v["bytes"] / (v["ms"] * 1e6)
        traffic = None
        tr = TRAFFIC.get(k)
        if (tr and tr["bytes_per_launch"] and src == "fp64" and dom == tr["kind"]
                and tr["sources_sha256"] == kernel_sources_sha256() and args.mesh is None):
            traffic = tr["bytes_per_launch"]
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                           "traffic_unit": "bytes/launch",
                           "kernel": f"{src}.{dom}", "launches": int(v["launches"]),
                           "avg_launch_us": 1000 * v["ms"] / v["launches"],
                           "bytes_per_launch_avg": v["bytes"] / v["launches"]}
        # A measured ceiling beside the published peak (outside the timed steps).
        copy_gbs, read_gbs = stream_ceilings()
        out["stream_ceiling"] = {"copy_GBs": copy_gbs, "read_GBs": read_gbs, "unit": "GB/s",
                                 "kind": "torch 1 GiB device copy (read + written bytes) and "
                                         "1 GiB sum (read bytes), best of 10",
                                 "dominant_kernel_frac_of_best": achieved / max(copy_gbs, read_gbs)}
    if k == 5 and "mixed" in plans and not args.no_adjoint:
        # Backward of the differentiable solve (outside the timed steps):
        # L = 1/2 ||x - x_target||^2, adjoint FP64 GMRES on A^T.
        p = plans["mixed"]
        p.set_timing(0)
        xs, _ = p.solve(b, out=x)
        gx = xs - torch.from_numpy(sysm.meta["x_target"]).cuda() if "x_target" in sysm.meta else xs.clone()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        gb, gv, ainfo = p.adjoint(xs, gx)
        torch.cuda.synchronize()
        out["adjoint_s"] = time.perf_counter() - t1
        out["adjoint_iters"] = ainfo["iters"]
        out["adjoint_rel_res_true"] = ainfo["rel_res_true"]
    if not args.no_cpu_baseline:
        fp64_iters = infos["fp64"]["iters"] if "fp64" in infos else infos[headline]["iters"]
        log(f"[bench] cpu baseline: oracle, {args.cpu_sample_iters} steps")
        out["cpu_baseline"] = cpu_baseline(sysm, m, fp64_iters, args.cpu_sample_iters)
    print(json.dumps(out), flush=True)


def adaptive_mode(args):
    """The paper's own preconditioner (adaptive spectral deflation, no fixed
    Z) on the kappa = 1 problem of a 1024^2 mesh, GMRES(30), FP64."""
    import copy
    import numpy as np
    import torch
    from paper_1906_04051_amd import gmres as G
    from paper_1906_04051_amd import workloads as W
    mesh = args.mesh or 1024
    m = W.CONFIGS[1]["m"]
    log(f"[bench] generating the kappa = 1 problem at mesh {mesh}")
    sysm = copy.copy(W.make_config(1, mesh=mesh))
    sysm.r = 0
    sysm.z_rowptr = np.zeros(sysm.n + 1, np.int32)
    sysm.z_colind = np.zeros(0, np.int32)
    sysm.z_vals = np.zeros(0)
    d = G.upload(sysm)
    plan = G.Plan(d["rowptr"], d["colind"], d["vals"], d["z_rowptr"], d["z_colind"], d["z_vals"], r=0,
                  precision="fp64", adapt_rmax=args.adaptive, m=m, rtol=1e-8, max_iters=200000,
                  ortho=args.ortho)
    tuned = plan.autotune()
    b = d["b"]
    x = torch.empty_like(b)
    for _ in range(args.warmup):
        plan.set_timing(0)
        plan.solve(b, out=x)
    timing = 0 if args.no_timing else max(args.timing_period, 1)
    times, ktot = [], {}
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for step in range(args.steps):
        plan.set_timing(timing)
        t1 = time.perf_counter()
        _, info = plan.solve(b, out=x)
        times.append(time.perf_counter() - t1)
        for kk, v in (plan.kernel_times() if timing else {}).items():
            a = ktot.setdefault(kk, dict(launches=0.0, ms=0.0, bytes=0.0))
            for fld in ("launches", "ms", "bytes"):
                a[fld] += v[fld]
        log(f"[bench] step {step}: {times[-1]:.3f} s iters {info['iters']} r {info['defl_r']} "
            f"rel_res_true {info['rel_res_true']:.3e}")
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    med = float(np.median(times))
    out = {
        "metric": "time-to-rtol 1e-8 (s), GMRES(30) with adaptive spectral deflation",
        "value": med, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1000.0 * total / max(args.steps, 1), "higher_is_better": False,
        "scaling": "strong", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"q1_convection_diffusion_{mesh}x{mesh}_kappa1", "unknowns": sysm.n,
                   "nnz": sysm.nnz, "restart_m": m, "deflation": "adaptive spectral (Ritz vectors of H_k)",
                   "adapt_rmax": args.adaptive, "rtol": 1e-8, "spmv_lanes": tuned["spmv_lanes"],
                   "num_blocks": tuned["num_blocks"]},
        "iters": info["iters"], "defl_r": info["defl_r"], "mu": info["mu"],
        "rel_res_true": info["rel_res_true"],
    }
    if ktot:
        per = {kk: dict(launches=int(v["launches"]), avg_us=1000 * v["ms"] / v["launches"],
                        GBs=v["bytes"] / (v["ms"] * 1e6), total_ms=v["ms"])
               for kk, v in ktot.items() if v["launches"] > 0}
        out["kernels"] = per
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sysm, m, info["iters"], args.cpu_sample_iters,
                                           adapt_rmax=args.adaptive)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=5, choices=[2, 3, 4, 5],
                    help="workload: 5 (default) 2048^2 Q1, 4.2 M unknowns; 2 1024^2 Q1 log-normal; "
                         "3 512^2 Q2 Bratu Jacobian; 4 the 512-system batch")
    ap.add_argument("--mesh", type=int, default=None, help="override the config's mesh size")
    ap.add_argument("--cpu-sample-iters", type=int, default=50,
                    help="oracle steps of the CPU baseline (default: one restart cycle of GMRES(50))")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cont-rows", type=int, default=20000,
                    help="config 4: systems of at least this many rows get a continuation plan (0: none)")
    ap.add_argument("--cont-work", type=float, default=128e6,
                    help="config 4: row-steps after which such a system leaves the batched launch")
    ap.add_argument("--no-adjoint", action="store_true", help="config 5: skip the adjoint measurement")
    ap.add_argument("--no-timing", action="store_true", help="no per-kernel HIP events")
    ap.add_argument("--timing-period", type=int, default=8,
                    help="time the kernels of one restart cycle in this many (the others "
                         "replay the captured cycle graph)")
    ap.add_argument("--only", choices=["both", "fp64", "mixed"], default="both")
    ap.add_argument("--mixed-basis", choices=["f16", "f32"], default=None,
                    help="storage of the Krylov basis in the inner FP32 solves (default f16; f32 for config 3)")
    ap.add_argument("--inner-rtol", type=float, default=None,
                    help="tolerance of each inner solve (default 1e-3 for f16, 1e-5 for f32)")
    ap.add_argument("--ortho", type=int, default=1, choices=[0, 1, 2],
                    help="0: CGS2 in three sweeps; 1: CGS2 in two sweeps (lagged normalisation); "
                         "2: CGS2 with one reduction per step (FP64 only: use with --only fp64)")
    ap.add_argument("--adaptive", type=int, default=0, metavar="RMAX",
                    help="instead of the default step: one FP64 solve right-preconditioned by "
                         "adaptive spectral deflation with at most RMAX Ritz vectors (no fixed Z)")
    ap.add_argument("--bratu", type=int, default=0, metavar="NEL",
                    help="instead of the default step: Newton's method on the paper's 3-D Bratu "
                         "problem with NEL^3 27-node hexahedra ((2 NEL + 1)^3 unknowns), linear "
                         "solves by GPU GMRES(50) with adaptive deflation (r_max 20)")
    ap.add_argument("--bratu-fixed", type=int, default=0, metavar="NEL",
                    help="instead of the default step: the paper's protocol on the Bratu Jacobian "
                         "at u = 0 with NEL^3 hexahedra: GMRES(50), adaptive deflation (r_max 20), "
                         "exactly 100 restarts, no termination test")
    ap.add_argument("--bratu-cycles", type=int, default=100,
                    help="restart cycles of --bratu-fixed (the paper's protocol: 100; fewer for "
                         "hardware-counter runs)")
    ap.add_argument("--block", type=int, default=0, metavar="K",
                    help="instead of the default step: block GMRES for K right-hand sides (<= 16) on the "
                         "kappa = 1 system, fixed count, against single-vector GMRES(50)")
    ap.add_argument("--block-m", type=int, default=8, help="block steps per cycle of --block")
    ap.add_argument("--block-defl", action="store_true",
                    help="--block with the configuration's deflation basis (default: without Z)")
    ap.add_argument("--block-steps", type=int, default=48, help="block steps of --block (fixed count)")
    ap.add_argument("--pmc-sample", action="store_true",
                    help="short fixed-count FP64 run (two restart cycles) plus a copy of known "
                         "size, for hardware-counter collection")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(sharding across GPUs is not built)"}))
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    if args.bratu > 0:
        bratu_newton(args)
    elif args.bratu_fixed > 0:
        bratu_fixed(args)
    elif args.block > 0:
        if args.mesh is None:
            args.mesh = 1024
        block_rhs(args)
    elif args.adaptive > 0:
        adaptive_mode(args)
    elif args.config == 4:
        batched_config4(args)
    else:
        single_config(args)


if __name__ == "__main__":
    main()
