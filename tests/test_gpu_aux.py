"""Auxiliary subsystems on the GPU: roctx phase ranges (GMRES_TRACE) and the
autotune cache (GMRES_TUNE_CACHE).

Tracing only brackets host-side phases, so a traced solve must give the same
bits as an untraced one.  The cache must give back exactly the choices the
tuning made, skip the timing on a hit, and tune again when an entry names a
choice the plan cannot run.
"""
import os

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


def test_traced_solves_are_bitwise_equal(monkeypatch):
    s = W.make_config(1, mesh=40)
    out = {}
    for tr in ("0", "1"):
        monkeypatch.setenv("GMRES_TRACE", tr)
        for prec in ("fp64", "mixed_f16"):
            plan, d = G().plan_for(s, m=30, rtol=1e-8, max_iters=4000, precision=prec)
            x, info = plan.solve(d["b"])
            out[(tr, prec)] = (x.cpu().numpy(), info["iters"], info["refinements"])
            say(tr, prec, info["iters"], info["status_name"])
            assert info["status_name"] == "OK"
    for prec in ("fp64", "mixed_f16"):
        a, b = out[("0", prec)], out[("1", prec)]
        assert a[1] == b[1] and a[2] == b[2]
        assert np.array_equal(a[0], b[0]), prec
    ref = oracle.gmres(s, 30, 1e-8, 4000)
    assert np.linalg.norm(out[("1", "fp64")][0] - ref.x) <= 1e-8 * np.linalg.norm(ref.x)


def test_tune_cache_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("GMRES_TUNE_CACHE", str(path))
    s = W.make_config(1, mesh=48)
    p1, d1 = G().plan_for(s, m=30, rtol=1e-8, max_iters=4000)
    c1 = p1.autotune()
    lines = path.read_text().splitlines()
    say("tuned", c1, lines)
    assert len(lines) == 1 and "\t" in lines[0]
    # Same shape: the cached choices, no new line, same solution bits.
    p2, d2 = G().plan_for(s, m=30, rtol=1e-8, max_iters=4000)
    c2 = p2.autotune()
    assert c2 == c1
    assert len(path.read_text().splitlines()) == 1
    x1, i1 = p1.solve(d1["b"])
    x2, i2 = p2.solve(d2["b"])
    assert i1["iters"] == i2["iters"] and torch.equal(x1, x2)
    # Another restart length is another key: tuned and appended.
    p3, _ = G().plan_for(s, m=20, rtol=1e-8, max_iters=4000)
    p3.autotune()
    assert len(path.read_text().splitlines()) == 2
    # An entry the plan cannot run (grid of 0) is ignored: the plan is tuned
    # again and the new line wins from then on.
    key = lines[0].split("\t")[0]
    with open(path, "a") as f:
        f.write(f"{key}\t{c1['spmv_lanes']} 0 {c1['batch_wg']} {c1['batch_lanes']}\n")
    p4, d4 = G().plan_for(s, m=30, rtol=1e-8, max_iters=4000)
    c4 = p4.autotune()
    assert c4["num_blocks"] >= 1
    assert len(path.read_text().splitlines()) == 4
    x4, i4 = p4.solve(d4["b"])
    ref = oracle.gmres(s, 30, 1e-8, 4000)
    assert abs(i4["iters"] - ref.iters) <= 1
    assert np.linalg.norm(x4.cpu().numpy() - ref.x) <= 1e-8 * np.linalg.norm(ref.x)
