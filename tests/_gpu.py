"""Shared helpers of the GPU tests (not collected by pytest)."""
import sys

import numpy as np
import pytest

try:
    import torch
    HAVE_GPU = torch.cuda.is_available()
except Exception:  # pragma: no cover
    torch = None
    HAVE_GPU = False

EPS64 = np.finfo(np.float64).eps
EPS32 = np.finfo(np.float32).eps
EPS16 = np.finfo(np.float16).eps

gpu = pytest.mark.gpu


def need_gpu():
    if not HAVE_GPU:
        pytest.skip("no GPU")


def say(*a):
    """Name the case before a GPU step (flushed), so a crash names it."""
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().double().cpu().numpy()


def make_mg(N, d, coeffs, **kw):
    from paper_2206_05543_amd._lib import Multigrid
    return Multigrid(N, d, coeffs, **kw)
