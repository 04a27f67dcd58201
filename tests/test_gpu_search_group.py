"""Clustered searches: a superblock searched by G workgroups gives what one gives
(in double, double-double and quad-double).

The sweep kernel may spread each superblock's search (Alg. 2 inside Alg. 6) over
G workgroups that combine their block argmaxes after every step.  Every point
is evaluated with the same operations whichever workgroup takes it, and the
combination keeps the single-workgroup tie rule (largest |error|, then lowest
index), so every pivot record, every value of the history, the evaluation counts
and the index sets must be equal bit for bit for G = 1, 2, 3, 8 and the rule's G.
The single-workgroup runs are themselves checked against the oracle by the other
parity tests.
"""
import pytest

from gpu_util import gpu_context
from paper_1903_11554_amd.workloads import Problem, config_batch, config_single_sweep, synthetic_params

pytestmark = pytest.mark.gpu

WORKLOADS = {
    "ising_d5_d10_c4_strict": config_single_sweep(stop="strict"),
    "mixed_batch16": config_batch(count=16, seed=7),
    "ising_d36_streaming": [Problem("ising_d", 36, 6, 6, 1e-10, seed=6)],
    "ising_c41_rank16": [Problem("ising_c", 41, 12, 14, 1e-12, seed=3, max_sweeps=8)],
    "sum2_d12": [Problem("sum2_exp_cos", 12, 32, 8, 1e-12, seed=9, params=synthetic_params(12, 9))],
    "ising_d6_d8_double_double": [Problem("ising_d", d, 16, 16, 1e-20, seed=d, precision="dd") for d in (6, 8)],
    "ising_d5_quad_double": [Problem("ising_d", 5, 5, 8, 1e-40, seed=5, precision="qd")],
}


def run_with_group(probs, group):
    ctx = gpu_context()
    ctx.set_search_group(group)
    try:
        job = ctx.job(probs)
        infos = job.run()
        out = []
        for k in range(len(probs)):
            # the whole value in every number type: its double components and exponent
            hist = job.history_parts(k, 4) if probs[k].precision != "fp64" else job.history_scaled(k)
            out.append(dict(info={key: infos[k][key] for key in ("sweeps", "reason", "evals", "err_flags",
                                                                   "value", "max_rank")},
                            log=job.pivot_log(k), hist=hist, sets=job.index_sets(k)))
        job.free()
        return out
    finally:
        ctx.set_search_group(0)


@pytest.mark.parametrize("name", sorted(WORKLOADS))
def test_search_group_gives_identical_runs(name):
    probs = WORKLOADS[name]
    print(f"{name}: {len(probs)} integrals", flush=True)
    ref = run_with_group(probs, 1)
    for k, r in enumerate(ref):
        assert r["info"]["err_flags"] == 0, (k, r["info"])
    for group in (2, 3, 8, 0):
        got = run_with_group(probs, group)
        for k in range(len(probs)):
            assert got[k]["info"] == ref[k]["info"], (group, k, got[k]["info"], ref[k]["info"])
            assert got[k]["log"] == ref[k]["log"], (group, k)
            assert got[k]["hist"] == ref[k]["hist"], (group, k)
            assert got[k]["sets"] == ref[k]["sets"], (group, k)
        print(f"  group {group}: identical", flush=True)


def test_search_group_range():
    from paper_1903_11554_amd.ttcross import TTError
    ctx = gpu_context()
    for bad in (-1, 9):
        with pytest.raises(TTError):
            ctx.set_search_group(bad)
    ctx.set_search_group(0)
