"""Host-side checks of the C ABI: the library loads and exports every entry
point that include/ttcross.h declares, and host-only calls behave (no GPU)."""
import ctypes
import os
import re

import pytest

from paper_1903_11554_amd import ttcross as binding
from paper_1903_11554_amd.workloads import Problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ttcross.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tt_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    assert declared_functions() == sorted(binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = binding.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_status_strings():
    lib = binding.load_library()
    for code in (0, 1, 2, -1, -2, -3, -4):
        assert lib.tt_status_string(code).startswith(b"TT_")


def test_footprint_host_only():
    p = Problem("ising_d", 10, 64, 32, 1e-10)
    f = binding.footprint(p)
    m, n, R = 9, 64, 32
    # the cores and interpolation cores dominate: about 2 m R^2 n doubles
    assert 0.5 * 2 * m * R * R * n * 8 < f < 2.0 * 2 * m * R * R * n * 8


@pytest.mark.parametrize("bad", [
    Problem("ising_d", 0, 64, 32, 1e-10),            # d < 1
    Problem("ising_d", 1026, 33, 8, 1e-10),          # more than 1024 modes
    Problem("ising_d", 34, 64, 32, 1e-10, precision="dd"),   # double-double beyond 32 modes
    Problem("ising_c_u", 33, 64, 8, 1e-10),          # u-form beyond 32 modes
    Problem("ising_d", 5, 0, 32, 1e-10),             # no nodes
    Problem("ising_d", 5, 257, 32, 1e-10),           # too many nodes
    Problem("ising_d", 5, 64, 65, 1e-10),            # rank over the cap
    Problem("ising_d", 5, 64, 8, 0.0),               # tol <= 0
    Problem("prod_exp", 5, 64, 8, 1e-10),            # synthetic without params
])
def test_invalid_problems_rejected(bad):
    assert binding.footprint(bad) == 0


def test_large_jobs_accepted():
    # the streaming path: up to 1024 modes, double precision, paper form and synthetic
    assert binding.footprint(Problem("ising_c", 1024, 33, 16, 1e-12)) > 0
    assert binding.footprint(Problem("ising_d", 34, 64, 32, 1e-10)) > 0
    a = [0.1] * 1000
    assert binding.footprint(Problem("prod_exp", 1000, 16, 4, 1e-12, params={"a": a, "b": a})) > 0


def test_ctx_fails_loudly_without_gpu():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    with pytest.raises(binding.TTError):
        binding.Context(0)


def test_stop_rule_field():
    import ctypes
    lib = binding.load_library()
    assert binding.footprint(Problem("ising_d", 6, 64, 32, 1e-10, stop="strict")) == \
        binding.footprint(Problem("ising_d", 6, 64, 32, 1e-10))
    keep = []
    for rule, reserved, ok in [(0, 0, True), (1, 0, True), (2, 0, False), (-1, 0, False), (1, 5, False)]:
        cp = binding._c_problem(Problem("ising_d", 6, 64, 32, 1e-10), keep)
        cp.stop_rule, cp.reserved = rule, reserved
        assert (lib.tt_job_footprint(ctypes.byref(cp)) > 0) == ok, (rule, reserved)
