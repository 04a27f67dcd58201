"""Parity of the batched integrand evaluation (one point per lane) with the oracle.

The GPU and the oracle evaluate the same formulas in different operation orders
(Horner sums and a single division on the GPU, the literal formula in the
oracle), so values agree to a rounding bound: each side performs at most K
correctly rounded operations on positive, well-conditioned quantities, so the
relative difference is at most 2 K u with u = 2^-53 (stated per family below).
"""
import numpy as np
import pytest

from gpu_util import eps_bound, gpu_context, require_gpu
from oracle.gauss import gauss_legendre_01
from oracle.integrands import weighted_values
from paper_1903_11554_amd.workloads import (Problem, random_index_set, random_multi_indices,
                                            synthetic_params)

pytestmark = pytest.mark.gpu


def op_count(family, m):
    pairs = m * (m + 1) // 2
    if family in ("ising_d", "ising_e"):
        return 4 * pairs + 4 * m + 16
    if family == "ising_c":
        return 6 * m + 16
    if family == "ising_d_u":
        return 8 * pairs + 8 * m + 24
    if family == "ising_c_u":
        return 10 * m + 16
    return 12 * m + 16   # synthetic: exp/cos are within a few ulp


CASES = [
    ("ising_d", 10, 64), ("ising_d", 5, 64), ("ising_d", 2, 7), ("ising_d", 17, 16),
    ("ising_d", 32, 8), ("ising_d", 33, 5), ("ising_c", 4, 64), ("ising_c", 33, 16),
    ("ising_e", 9, 33), ("ising_c_u", 3, 32), ("ising_d_u", 6, 32), ("ising_d_u", 20, 16),
    ("prod_exp", 3, 32), ("sum2_exp_cos", 12, 64), ("sum2_exp_cos", 32, 8),
    ("ising_d", 6, 1), ("ising_c", 5, 256),
]


@pytest.mark.parametrize("family,d,n", CASES)
def test_eval_points_matches_oracle(family, d, n):
    torch = require_gpu()
    ctx = gpu_context()
    params = synthetic_params(d, 7) if family in ("prod_exp", "sum2_exp_cos") else None
    p = Problem(family, d, n, 8, 1e-10, params=params)
    m = p.modes()
    npts = 256 * 7 + 37                      # several workgroups and a ragged tail
    idx = random_multi_indices(npts, m, n, seed=d * 1000 + n)
    print(f"eval_points {family} d={d} n={n} npts={npts}", flush=True)
    idx_dev = torch.from_numpy(idx).cuda()
    out = torch.empty(npts, dtype=torch.float64, device="cuda")
    ctx.eval_points(p, idx_dev.data_ptr(), out.data_ptr(), npts)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    t, w = gauss_legendre_01(n)
    want = weighted_values(family, idx, t, w, params)
    assert np.all(np.isfinite(got))
    rtol = eps_bound(op_count(family, m))
    tiny = np.abs(want).max() * 1e-290
    np.testing.assert_allclose(got, want, rtol=rtol, atol=tiny)


def test_eval_points_empty():
    torch = require_gpu()
    ctx = gpu_context()
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    ctx.eval_points(Problem("ising_d", 5, 8, 4, 1e-10), 0, out.data_ptr(), 0)


@pytest.mark.parametrize("family,d,n,pos,rl,rr", [
    ("ising_d", 10, 64, 4, 20, 17), ("ising_d", 10, 64, 0, 1, 32), ("ising_d", 10, 64, 8, 32, 1),
    ("ising_c", 8, 33, 3, 7, 9), ("sum2_exp_cos", 9, 16, 5, 11, 5), ("ising_d", 20, 12, 9, 64, 64),
])
def test_eval_fibers_matches_oracle(family, d, n, pos, rl, rr):
    torch = require_gpu()
    ctx = gpu_context()
    params = synthetic_params(d, 3) if family in ("prod_exp", "sum2_exp_cos") else None
    p = Problem(family, d, n, 8, 1e-10, params=params)
    m = p.modes()
    left = random_index_set(rl, pos, n, seed=1) if pos > 0 else np.zeros((1, 0), np.int32)
    right = random_index_set(rr, m - pos - 1, n, seed=2) if pos < m - 1 else np.zeros((1, 0), np.int32)
    print(f"eval_fibers {family} d={d} n={n} pos={pos} rl={rl} rr={rr}", flush=True)
    ld = torch.from_numpy(np.ascontiguousarray(left)).cuda() if pos > 0 else None
    rd = torch.from_numpy(np.ascontiguousarray(right)).cuda() if pos < m - 1 else None
    out = torch.empty(rl * n * rr, dtype=torch.float64, device="cuda")
    ctx.eval_fibers(p, pos, ld.data_ptr() if ld is not None else 0, rl,
                    rd.data_ptr() if rd is not None else 0, rr, out.data_ptr())
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(rl, n, rr)
    idx = np.array([list(left[a]) + [i] + list(right[b]) for a in range(rl) for i in range(n)
                    for b in range(rr)], dtype=np.int64)
    t, w = gauss_legendre_01(n)
    want = weighted_values(family, idx, t, w, params).reshape(rl, n, rr)
    np.testing.assert_allclose(got, want, rtol=eps_bound(op_count(family, m)),
                               atol=np.abs(want).max() * 1e-290)


@pytest.mark.parametrize("family", ["ising_d", "ising_c", "ising_e"])
def test_eval_fibers_every_mode_count_and_position(family):
    """The paper form's fibre kernels at every mode count 1..18 and every node position.

    Up to 16 modes the row-summary kernel serves (a compile-time node position per
    case), above that the one-pass kernel; 9 nodes leave a ragged last chunk of
    the four nodes a lane takes, and the set sizes are odd.
    """
    torch = require_gpu()
    ctx = gpu_context()
    n = 9
    t, w = gauss_legendre_01(n)
    for d in range(2, 20):
        p = Problem(family, d, n, 8, 1e-10)
        m = p.modes()
        for pos in range(m):
            rl = 5 if pos > 0 else 1
            rr = 3 if pos < m - 1 else 1
            left = random_index_set(rl, pos, n, seed=d * 100 + pos) if pos > 0 else np.zeros((1, 0), np.int32)
            right = (random_index_set(rr, m - pos - 1, n, seed=d * 100 + pos + 50) if pos < m - 1
                     else np.zeros((1, 0), np.int32))
            print(f"eval_fibers {family} d={d} pos={pos} rl={rl} rr={rr}", flush=True)
            ld = torch.from_numpy(np.ascontiguousarray(left)).cuda() if pos > 0 else None
            rd = torch.from_numpy(np.ascontiguousarray(right)).cuda() if pos < m - 1 else None
            out = torch.full((rl * n * rr,), float("nan"), dtype=torch.float64, device="cuda")
            ctx.eval_fibers(p, pos, ld.data_ptr() if ld is not None else 0, rl,
                            rd.data_ptr() if rd is not None else 0, rr, out.data_ptr())
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            idx = np.array([list(left[a]) + [i] + list(right[b]) for a in range(rl) for i in range(n)
                            for b in range(rr)], dtype=np.int64)
            want = weighted_values(family, idx, t, w)
            np.testing.assert_allclose(got, want, rtol=eps_bound(op_count(family, m)),
                                       atol=np.abs(want).max() * 1e-290, err_msg=f"d={d} pos={pos}")


def test_eval_fibers_graph_replay_matches_eager():
    """Library launches captured in a HIP graph replay to the eager result, replay after replay."""
    torch = require_gpu()
    from paper_1903_11554_amd import Context
    p = Problem("ising_d", 8, 32, 8, 1e-10)
    m, pos, rl, rr = p.modes(), 3, 16, 16
    left = torch.from_numpy(random_index_set(rl, pos, p.n, 21)).cuda()
    right = torch.from_numpy(random_index_set(rr, m - pos - 1, p.n, 22)).cuda()
    side = torch.cuda.Stream()
    ctx = Context(0, stream=side)
    eager = torch.empty(rl * p.n * rr, dtype=torch.float64, device="cuda")
    out = torch.zeros_like(eager)
    with torch.cuda.stream(side):
        ctx.eval_fibers(p, pos, left.data_ptr(), rl, right.data_ptr(), rr, eager.data_ptr())
    side.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        ctx.eval_fibers(p, pos, left.data_ptr(), rl, right.data_ptr(), rr, out.data_ptr())
    for k in range(4):
        out.zero_()                      # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), k
    del graph
    ctx.close()
