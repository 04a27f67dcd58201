"""The serving loop (tt_server_*): continuous batching of single-integral requests.

Every result must be bitwise the one the same problem gets alone
(tt_cross_run): a request's computation depends only on its own problem (its
own sweep counter keys its samples), whatever else shares the launches.
Requests are admitted by memory footprint and slot count, including while
others are running.
"""
import time

import pytest

from gpu_util import gpu_context
from paper_1903_11554_amd.ttcross import TTError, footprint
from paper_1903_11554_amd.workloads import Problem, serving_trace

pytestmark = pytest.mark.gpu


def alone(ctx, p):
    job = ctx.job([p])
    info = job.run()[0]
    job.free()
    return info


def same(a, b):
    keys = ("value", "value_lo", "evals", "sweeps", "reason", "max_rank", "err_flags")
    return all(a[k] == b[k] for k in keys)


def test_server_burst_equals_alone():
    ctx = gpu_context()
    reqs = [p for _, p in serving_trace(duration_s=0.2, seed=5)]
    reqs += [Problem("ising_d", 1, 8, 4, 1e-10), Problem("ising_c", 2, 16, 4, 1e-10)]   # no bonds
    print(f"server burst of {len(reqs)} requests", flush=True)
    srv = ctx.server(max_bytes=2 << 30, max_active=256)
    tickets = [srv.submit(p) for p in reqs]
    got = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    print(f"stats {st}", flush=True)
    assert st["completed"] == len(reqs) and st["max_running"] > 1
    for p, (info, lat) in zip(reqs, got):
        ref = alone(ctx, p)
        assert same(info, ref), (p, info, ref)
        assert lat > 0


def test_server_admits_while_running():
    ctx = gpu_context()
    trace = serving_trace(duration_s=0.3, rate=200.0, seed=7)
    print(f"server stream of {len(trace)} requests", flush=True)
    srv = ctx.server(max_bytes=2 << 30, max_active=256)
    t0 = time.perf_counter()
    tickets = []
    for at, p in trace:
        while time.perf_counter() - t0 < at:
            time.sleep(0.0005)
        tickets.append((p, srv.submit(p)))
    got = [(p, srv.wait(t)) for p, t in tickets]
    st = srv.stats()
    srv.close()
    print(f"stats {st}", flush=True)
    assert st["completed"] == len(trace) and st["admissions"] >= 2
    for p, (info, lat) in got:
        assert same(info, alone(ctx, p)), p


def test_server_admission_by_footprint():
    ctx = gpu_context()
    reqs = [Problem("ising_d", 9, 32, 16, 1e-9, seed=s) for s in range(1, 7)]   # equal footprints
    cap = footprint(reqs[0]) * 2 + 65536                  # room for two at a time, not three
    srv = ctx.server(max_bytes=cap, max_active=64)
    tickets = [srv.submit(p) for p in reqs]
    got = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    print(f"stats {st}", flush=True)
    assert st["max_running"] <= 2 and st["admissions"] >= 3
    for p, (info, _) in zip(reqs, got):
        assert same(info, alone(ctx, p)), p


def test_server_slot_limit_and_rejections():
    ctx = gpu_context()
    srv = ctx.server(max_bytes=256 << 20, max_active=2)
    reqs = [Problem("ising_c", d, 24, 8, 1e-10, seed=d) for d in range(3, 9)]
    tickets = [srv.submit(p) for p in reqs]
    for p, t in zip(reqs, tickets):
        info, _ = srv.wait(t)
        assert same(info, alone(ctx, p))
    assert srv.stats()["max_running"] <= 2
    with pytest.raises(TTError):   # never fits
        srv.submit(Problem("ising_d", 32, 256, 64, 1e-10))
    with pytest.raises(TTError):   # double-double is not served
        srv.submit(Problem("ising_d", 5, 16, 8, 1e-20, precision="dd"))
    with pytest.raises(TTError):   # unknown ticket
        srv.poll(10 ** 9)
    srv.close()
