"""Seeded synthetic workloads (problem descriptions and random inputs).

This module holds no arithmetic of the method: it only describes integrals to
be computed (family, dimension, node count, rank cap, tolerance, seed,
parameters) and draws random multi-indices for evaluation checks.  Both the
GPU library's tests/benchmarks and the CPU oracle's runs take their inputs from
here, so the two sides see identical inputs.

The paper's workloads are the Ising integrals C_d and D_d (Sec. 5.1) in the
paper form on [0,1]^(d-1); the integrands are generated from their formulas,
so no external data set is involved.  Synthetic product families stand in for
the "rank-2 sum-of-products" test integrands.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class Problem:
    family: str            # ising_c | ising_d | ising_e | ising_c_u | ising_d_u | prod_exp | sum2_exp_cos
    d: int                 # Ising: the paper's d (number of u variables); synthetic: dimension
    n: int                 # Gauss--Legendre nodes per mode
    rank_cap: int
    tol: float
    seed: int = 1
    max_sweeps: int = 0
    params: Optional[dict] = None   # synthetic: {"a": [...], "b": [...]}, d entries each
    precision: str = "fp64"         # "fp64" or "dd" (double-double, paper-form integrands)
    stop: str = "rel2"              # "rel2" (two small relative changes) or "strict" (no accepted pivot)

    def modes(self):
        return self.d - 1 if self.family in ("ising_c", "ising_d", "ising_e") else self.d


def synthetic_params(d, seed):
    """a_j, b_j ~ U[0.5, 4] (seeded numpy PCG64)."""
    r = np.random.default_rng(seed)
    return {"a": r.uniform(0.5, 4.0, d).tolist(), "b": r.uniform(0.5, 4.0, d).tolist()}


def random_multi_indices(npts, m, n, seed):
    """npts x m node indices uniform in [0, n) (int32, seeded)."""
    r = np.random.default_rng(seed)
    return r.integers(0, n, size=(npts, m), dtype=np.int32)


def random_index_set(r, k, n, seed):
    """r distinct rows of k node indices (a stand-in for I_<=k or I_>k)."""
    g = np.random.default_rng(seed)
    rows = set()
    out = []
    while len(out) < r:
        row = tuple(int(v) for v in g.integers(0, n, size=k))
        if row not in rows or k == 0:
            rows.add(row)
            out.append(row)
    return np.array(out, dtype=np.int32).reshape(r, k)


# ------------------------------------------------------------ named workloads
def config_small():
    """C_3 (paper form, 2 modes), 32 nodes, rank <= 8, tol 1e-10; rank-1 product on d = 3."""
    return [
        Problem("ising_c", 3, 32, 8, 1e-10, seed=1),
        Problem("ising_c_u", 3, 32, 8, 1e-10, seed=1),
        Problem("prod_exp", 3, 32, 8, 1e-10, seed=1, params=synthetic_params(3, 1)),
    ]


def config_single_sweep(stop="rel2"):
    """D_5..D_10 (paper form), 64 nodes, rank <= 32, tol 1e-10, plus C_4."""
    probs = [Problem("ising_d", d, 64, 32, 1e-10, seed=d, stop=stop) for d in range(5, 11)]
    probs.append(Problem("ising_c", 4, 64, 32, 1e-10, seed=4, stop=stop))
    return probs


def config_batch(count=64, seed=4):
    """Mixed batch: C_n / D_n with n ~ U{4..16} and rank-2 synthetic with d ~ U{8..32}."""
    g = np.random.default_rng(seed)
    probs = []
    for k in range(count):
        fam = ["ising_c", "ising_d", "sum2_exp_cos"][int(g.integers(0, 3))]
        if fam == "sum2_exp_cos":
            d = int(g.integers(8, 33))
            probs.append(Problem(fam, d, 64, 48, 1e-10, seed=1000 + k,
                                 params=synthetic_params(d, 2000 + k)))
        else:
            d = int(g.integers(4, 17))
            probs.append(Problem(fam, d, 64, 48, 1e-10, seed=1000 + k))
    return probs


def serving_trace(duration_s=30.0, rate=200.0, seed=5, n=64):
    """Poisson arrivals of single-integral requests: [(arrival time in s, Problem)].

    Families as in the mixed batch (C_d, D_d paper form, rank-2 exp/cos
    products) with d ~ U{4..32}, tolerance log-uniform in [1e-12, 1e-6], rank
    cap ~ U{16..64}, n nodes; inter-arrival times exponential with the given
    rate (seeded numpy PCG64).
    """
    g = np.random.default_rng(seed)
    out, t, k = [], 0.0, 0
    while True:
        t += float(g.exponential(1.0 / rate))
        if t >= duration_s:
            break
        fam = ["ising_c", "ising_d", "sum2_exp_cos"][int(g.integers(0, 3))]
        d = int(g.integers(4, 33))
        tol = float(10.0 ** g.uniform(-12, -6))
        rank = int(g.integers(16, 65))
        params = synthetic_params(d, 50000 + k) if fam == "sum2_exp_cos" else None
        out.append((t, Problem(fam, d, n, rank, tol, seed=10000 + k, params=params)))
        k += 1
    return out
