"""Helpers shared by the GPU tests (no method arithmetic here)."""
import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2010_07422_amd import ircur
    ircur.lib()   # raises if the library is missing: no fallback
    return torch


def to_dev(torch, a, dtype):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def factors_np(ctx):
    At, B = ctx.factors()
    return At.double().cpu().numpy().T.copy(), B.double().cpu().numpy()
