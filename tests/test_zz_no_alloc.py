"""tt_mc_integrate_noalloc, the entry point for callers that cannot allocate, against tt_mc_integrate.

Both run the same kernels on the same grid, so every estimate, the mean and
the relative error must be the same doubles.  Two calls in a row, the second
with a smaller input (fewer points and estimators, another integrand class),
check that the static partial-sum array carries nothing from one call into the
next; a size beyond the array is rejected and the context stays usable.  The
estimators themselves are checked against the oracle in tests/test_gpu_mc.py.
"""
import math

import pytest

from gpu_util import gpu_context, require_gpu
from paper_1903_11554_amd.ttcross import MC_LATTICE, MC_RANDOM, TT_EINVAL, TTError
from paper_1903_11554_amd.workloads import Problem, synthetic_params

pytestmark = pytest.mark.gpu

CALLS = [
    # (problem, points, estimators, kind, generating vector): the second call is smaller
    (Problem("ising_d", 8, 16, 8, 1e-10, seed=8), (1 << 17) + 77, 24, MC_RANDOM, None),
    (Problem("sum2_exp_cos", 5, 16, 8, 1e-10, seed=5, params=synthetic_params(5, 7)), 1021, 6, MC_LATTICE,
     [1, 76, 671, 977, 301]),
]


def test_noalloc_matches_the_allocating_entry_point_on_two_calls_in_a_row():
    torch = require_gpu()
    ctx = gpu_context()
    for p, npts, nsets, kind, gen in CALLS:
        print(f"no-alloc mc {p.family} d={p.d} N={npts} S={nsets} kind={kind}", flush=True)
        est, mean, err = ctx.mc_integrate(p, npts, nsets, kind, gen)
        out = torch.full((nsets + 2,), math.nan, dtype=torch.float64, device="cuda")
        ctx.mc_integrate_noalloc(p, npts, nsets, out.data_ptr(), kind, gen)
        torch.cuda.synchronize()
        got = out.cpu().tolist()
        assert got[:nsets] == est, (got[:nsets], est)
        assert got[nsets] == mean and got[nsets + 1] == err, (got[nsets:], mean, err)


def test_noalloc_rejects_partial_sums_beyond_its_static_array():
    torch = require_gpu()
    ctx = gpu_context()
    p = Problem("ising_c", 4, 16, 8, 1e-10, seed=4)
    # 4096 estimators x 256 workgroups of partial sums exceed the 131072 the array holds
    out = torch.zeros(4096 + 2, dtype=torch.float64, device="cuda")
    with pytest.raises(TTError) as exc:
        ctx.mc_integrate_noalloc(p, 1 << 16, 4096, out.data_ptr())
    assert exc.value.status == TT_EINVAL
    with pytest.raises(TTError):
        ctx.mc_integrate_noalloc(p, 1 << 16, 16, 0)   # no output array
    # the largest accepted size: 512 estimators x 256 workgroups
    ctx.mc_integrate_noalloc(p, 1 << 16, 512, out.data_ptr())
    torch.cuda.synchronize()
    est, mean, err = ctx.mc_integrate(p, 1 << 16, 512)
    got = out[:514].cpu().tolist()
    assert got[:512] == est and got[512] == mean and got[513] == err
