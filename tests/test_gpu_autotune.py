"""The kernel-variant autotuner (tt_autotune) and its cache file.

A job's kernels come in variants (mode bucket, rank policy) that compute the
same values bit for bit; the tuner times them on the job, keeps the ones whose
results equal the rule's exactly, and records the fastest for later jobs with
the same key.  Checked here: the recorded choice is one that matched, later jobs
of the key take it and give the rule's results bit for bit, the cache file
round-trips through a fresh context, and a stale entry naming a variant the key
cannot launch is ignored.
"""
import os

import pytest

from gpu_util import require_gpu
from paper_1903_11554_amd.workloads import Problem, config_batch

pytestmark = pytest.mark.gpu


def results(ctx, probs):
    job = ctx.job(probs)
    infos = job.run()
    job.free()
    return [(i["value_mant"], i["value_exp2"], i["sweeps"], i["evals"]) for i in infos]


def test_autotune_records_a_bit_identical_variant(tmp_path, monkeypatch):
    require_gpu()
    from paper_1903_11554_amd import Context
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("TTCROSS_TUNE_CACHE", str(cache))
    probs = [Problem("ising_d", d, 32, 16, 1e-10, seed=d) for d in (5, 6, 7)]
    ctx = Context(0)
    base = results(ctx, probs)                     # the rule's variant (nothing tuned yet)
    res = ctx.autotune(probs, reps=2)
    print(f"autotune {res}", flush=True)
    assert res["rule_mode_bucket"] == 8            # D_7 has 6 modes: the paper-form bucket 8
    assert res["candidates"] >= 4 and 1 <= res["matching"] <= res["candidates"]
    assert res["mode_bucket"] in (8, 10, 12, 16, 24, 32, 0) and res["mode_bucket"] >= 0
    assert res["tuned_ms"] <= res["rule_ms"] and res["rule_ms"] > 0
    assert res["search_group"] in (0, 1, 2, 4, 6)
    assert results(ctx, probs) == base             # the tuned variant gives the rule's bits
    ctx.close()
    lines = [l.split() for l in cache.read_text().splitlines() if not l.startswith("#")]
    assert len(lines) == 1 and len(lines[0]) == 9
    fam, dd, maxm, maxr, mb, pol = (int(x) for x in lines[0][:6])
    assert (fam, dd, maxm, maxr, mb, pol) == (0, 0, 6, 16, res["mode_bucket"], res["rank_policy"])
    assert int(lines[0][8]) == res["search_group"]
    # a fresh context loads the cache; a stale entry (bucket 4 < 6 modes, in the
    # eight-field form without a search group) is ignored
    with open(cache, "a") as f:
        f.write("0 0 6 32 4 0 1.0 0.5\n")
    ctx2 = Context(0)
    assert results(ctx2, probs) == base
    probs32 = [Problem("ising_d", d, 32, 32, 1e-10, seed=d) for d in (5, 6, 7)]
    ref32 = results(ctx2, probs32)
    ctx2.close()
    monkeypatch.delenv("TTCROSS_TUNE_CACHE")
    ctx3 = Context(0)
    assert results(ctx3, probs32) == ref32         # the stale entry changed nothing
    ctx3.close()


def test_autotune_on_the_mixed_batch():
    # config 4's 64 mixed integrals (C_n, D_n, rank-2 exp/cos; up to 32 modes, rank <= 48)
    require_gpu()
    from paper_1903_11554_amd import Context
    probs = config_batch()
    ctx = Context(0)
    base = results(ctx, probs)
    res = ctx.autotune(probs, reps=1)
    print(f"autotune batch {res}", flush=True)
    assert res["rule_mode_bucket"] == 32 and res["matching"] >= 1
    assert results(ctx, probs) == base
    ctx.close()
