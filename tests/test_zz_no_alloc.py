"""The handle-free cycle mg_vcycle_noalloc against mg_vcycle on a handle.

Both run the same kernels with the same launch shapes on the same inputs, so
the results must agree bit for bit; each is also checked against the oracle's
V(1,1) cycle (Section 4) to the cycle-parity bound of the other GPU tests
(1e-12 of the largest entry: a fixed linear map of norm O(1) evaluated in
FP64 in a different operation order).  Calls come in pairs, the second on a
smaller problem, so the second runs on a workspace still holding the first
call's contents.
"""
import numpy as np
import pytest

import oracle as O
from paper_2206_05543_amd import M7, M9
from tests._gpu import dev, gpu, host, make_mg, need_gpu, say, torch

pytestmark = gpu


def _coeffs(d):
    return np.array(M9 if d == 2 else M7)


def _inputs(d, N, batch, seed):
    rng = np.random.default_rng(seed)
    shp = (batch,) + (N - 1,) * d
    return rng.uniform(-1, 1, shp), rng.standard_normal(shp) * N


def _one(d, N, batch, seed):
    from paper_2206_05543_amd._lib import vcycle_noalloc
    c = _coeffs(d)
    u0, b = _inputs(d, N, batch, seed)
    say("noalloc", d, N, batch)
    ub, bb = dev(u0), dev(b)
    vcycle_noalloc(N, d, c, bb, ub, batch=batch)
    with make_mg(N, d, c, batch=batch) as mg:
        uh = dev(u0)
        mg.vcycle(dev(b), uh)
        torch.cuda.synchronize()
    assert torch.equal(ub, uh), (d, N, batch)
    got = host(ub)
    for s in range(batch):
        want = O.vcycle(d, N, c, u0[s], b[s])
        assert np.max(np.abs(got[s] - want)) <= 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("first,second", [
    ((2, 1024, 1), (2, 256, 2)),   # the largest 2D grid that fits, then a batch of 2
    ((3, 128, 1), (3, 32, 3)),     # the largest 3D grid that fits, then a batch of 3
    ((3, 64, 2), (2, 64, 1)),      # a 2D cycle on a workspace left by a 3D one
    ((2, 128, 1), (2, 4, 2)),      # a single-grid problem (exact solve only)
])
def test_noalloc_cycle_matches_handle_cycle(first, second):
    need_gpu()
    _one(*first, seed=11)
    _one(*second, seed=12)


def test_noalloc_cycle_rejects_oversized_workspace():
    need_gpu()
    from paper_2206_05543_amd._lib import MGError, vcycle_noalloc
    u = torch.zeros(2047 * 2047, dtype=torch.float64, device="cuda")
    with pytest.raises(MGError, match="workspace"):
        vcycle_noalloc(2048, 2, M9, u, u.clone())
