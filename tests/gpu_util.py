"""Shared helpers of the GPU tests (no method arithmetic here)."""
import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    return torch


_CTX = None


def gpu_context():
    """One library context on cuda:0 bound to torch's current stream."""
    global _CTX
    torch = require_gpu()
    from paper_1903_11554_amd import Context
    if _CTX is None:
        torch.cuda.set_device(0)
        _CTX = Context(0, stream=torch.cuda.current_stream())
    return _CTX


def eps_bound(n_ops):
    """Relative bound for two evaluations that each round n_ops times: 2 n u."""
    return 2.0 * n_ops * 2.0 ** -53
