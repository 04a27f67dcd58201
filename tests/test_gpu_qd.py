"""The quad-double path (TT_QD) against 60-digit references.

* The Gauss-Legendre rule in quad-double against mpmath's Legendre roots and
  weights at 80 digits (oracle/gauss.py).
* The TT cross against the 256-bit oracle's cross of the same D_d with 3..6
  nodes (tests/golden/mp256_ising_small.txt, written by a script that calls
  only oracle/), and at full rank against the brute-force tensor sum over the
  same nodes (Thm. 2), both stored at 60 digits.  A quad-double value carries
  about 61 digits; the sums here take a few thousand operations, so 1e-55 is
  the bound.
* The rejections: quad-double beyond 16 modes or rank 32, or with integrands
  outside the paper form, and the entry points that do not take it.
"""
import mpmath as mp
import pytest

from gpu_util import gpu_context
from oracle.gauss import gauss_legendre_01_mp
from paper_1903_11554_amd.workloads import Problem

pytestmark = pytest.mark.gpu


def qd_value(parts, exp2):
    with mp.workdps(90):
        return mp.ldexp(mp.fsum(mp.mpf(c) for c in parts), exp2)


U_QD = mp.mpf(2) ** -200   # a conservative unit for quad-double (four doubles, about 2^-204)


@pytest.mark.parametrize("n", [3, 8, 33, 64])
def test_qd_node_tables_against_80_digit_rule(n):
    """The device's quad-double GL tables against mpmath's 80-digit rule.

    As for double-double: Newton leaves the root x with an absolute error of
    about 8 n u / |P_n'(x)| plus its rounding, t = (x+1)/2 inherits it, and the
    weight 1/((1-x^2) P_n'(x)^2) changes by 2|x| dx/(1-x^2) relative, with
    1 - x^2 formed to u/(1-x^2) relative near the ends of the interval.
    """
    ctx = gpu_context()
    job = ctx.job([Problem("ising_d", 4, n, 4, 1e-40, seed=1, max_sweeps=1, precision="qd")])
    t, w = job.nodes_parts(0, 4)
    job.free()
    with mp.workdps(90):
        tm, wm = gauss_legendre_01_mp(n, 80)
        pairs = sorted(zip(tm, wm))
        for i in range(n):
            ti, wi = pairs[i]
            x = 2 * ti - 1
            dp = abs(n * (x * mp.legendre(n, x) - mp.legendre(n - 1, x)) / (x * x - 1))
            dx = 8 * n * U_QD / dp + U_QD
            bt = dx / 2 + U_QD * ti
            bw = (2 * abs(x) * dx / (1 - x * x) + 8 * U_QD / (1 - x * x) + 8 * n * U_QD) * wi
            gt = mp.fsum(mp.mpf(c) for c in t[i])
            gw = mp.fsum(mp.mpf(c) for c in w[i])
            assert abs(gt - ti) <= bt, (n, i, gt - ti, bt)
            assert abs(gw - wi) <= bw, (n, i, gw - wi, bw)
            assert bw < mp.mpf("1e-55") * wi    # the bound itself is near quad-double precision


def mp256_rank32_cases():
    """The 256-bit oracle's D_d runs (tests/golden/mp256_ising_small.txt) that stay within rank 32."""
    import os
    out = []
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "mp256_ising_small.txt")
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            d, n, v, sweeps, reason, ranks, t2 = line.split()
            d, n = int(d), int(n)
            ranks = [int(r) for r in ranks.split(",")]
            if max(ranks) <= 32:
                m = d - 1
                full = [min(n ** (k + 1), n ** (m - k - 1)) for k in range(m - 1)]
                out.append((d, n, v, ranks, full, t2))
    return out


@pytest.mark.parametrize("case", mp256_rank32_cases(), ids=lambda c: f"D{c[0]}_n{c[1]}")
def test_qd_cross_against_the_256_bit_cross(case):
    """The quad-double GPU cross against the 256-bit oracle's cross of the same problem.

    Where both end on the same ranks the values must agree to 1e-55 (both are
    the same cross formula on the same sets, quad-double rounding about 1e-61
    per operation).  Where the ranks are the full ones the cross is exact
    (Thm. 2) and both equal the brute-force sum over the same nodes, T2.  Where
    the ranks differ (the searches end on ties at the rounding level, R20) the
    GPU run must have gone at least as far and be no further from T2.
    """
    d, n, v, ranks_mp, full, t2 = case
    print(f"qd D_{d} n={n} 256-bit ranks {ranks_mp} full {full}", flush=True)
    ctx = gpu_context()
    job = ctx.job([Problem("ising_d", d, n, 32, 1e-45, seed=d, precision="qd")])
    info = job.run()[0]
    ranks = [len(s[0]) for s in job.index_sets(0)]
    parts, e = job.history_parts(0, 4)[-1]
    job.free()
    val = qd_value(parts, e)
    with mp.workdps(90):
        rel = abs(val / mp.mpf(v) - 1)
        rel_t2 = abs(val / mp.mpf(t2) - 1)
        ref_t2 = abs(mp.mpf(v) / mp.mpf(t2) - 1)
    print(f"  ranks {ranks} sweeps {info['sweeps']} {info['reason']} rel to the 256-bit cross "
          f"{mp.nstr(rel, 3)}, to T2 {mp.nstr(rel_t2, 3)} (256-bit cross to T2 {mp.nstr(ref_t2, 3)})", flush=True)
    assert info["err_flags"] == 0
    if ranks == ranks_mp:
        assert rel <= mp.mpf("1e-55")
    else:
        assert all(g >= r for g, r in zip(ranks, ranks_mp)), (ranks, ranks_mp)
        assert rel_t2 <= ref_t2 + mp.mpf("1e-55")
    if ranks == full:
        assert rel_t2 <= mp.mpf("1e-55")
    # the leading double agrees with the info's value
    assert abs(info["value"] - float(val)) <= 1e-15 * abs(float(val))


def test_qd_rejections():
    from paper_1903_11554_amd import ttcross as binding
    bad = [Problem("ising_d", 18, 8, 8, 1e-40, precision="qd"),      # 17 modes
           Problem("ising_d", 6, 8, 33, 1e-40, precision="qd"),      # rank above 32
           Problem("ising_c_u", 4, 8, 8, 1e-40, precision="qd")]     # u-form
    for p in bad:
        assert binding.footprint(p) == 0
    assert binding.footprint(Problem("ising_d", 17, 8, 32, 1e-40, precision="qd")) > 0
    import torch

    from paper_1903_11554_amd.ttcross import TT_EINVAL, TTError
    ctx = gpu_context()
    p = Problem("ising_d", 5, 8, 8, 1e-40, precision="qd")
    out = torch.empty(8, dtype=torch.float64, device="cuda")
    idx = torch.zeros(8 * 4, dtype=torch.int32, device="cuda")
    with pytest.raises(TTError) as exc:
        ctx.eval_points(p, idx.data_ptr(), out.data_ptr(), 1)
    assert exc.value.status == TT_EINVAL
    job = ctx.job([p])
    with pytest.raises(TTError) as exc:
        job.refresh()
    assert exc.value.status == TT_EINVAL
    job.free()
