"""The benchmark's full-size configurations beyond the FP64 throughput pair.

- Mixed precision, 3D N=512 (1.33e8 unknowns, noisy sine right-hand side):
  FP64, FP32 and FP16 solves to a 1e-10 residual reduction, with the
  residual of the GPU solution recomputed by the oracle's FP64 operator.
- Gradients, 2D N=1024 with a batch of 16 random errors and three cycles:
  loss and gradients with respect to the coefficients, b and e0 against the
  oracle's reverse sweeps, and a central difference on one coefficient.
- Gradients, 3D N=256, two cycles: one batch entry with FP64 checkpoints
  against the oracle; the batch of 4 with FP32 checkpoints (the workload's
  configuration) against the oracle's reverse sweeps over the same rounded
  states, every entry.
"""
import numpy as np
import pytest

import oracle as O
from paper_2206_05543_amd import M7, M9
from paper_2206_05543_amd.workloads import workload
from tests._gpu import dev, gpu, host, make_mg, need_gpu, say, torch

pytestmark = gpu


@pytest.fixture(scope="module")
def noisy512():
    return workload("poisson3d_n512_noisy")


@pytest.mark.parametrize("prec", ["fp64", "fp32_ir", "fp16_ir"])
def test_mixed_precision_full_size(noisy512, prec):
    need_gpu()
    p = noisy512
    say("fullsize-mixed", prec)
    with make_mg(512, 3, M7, precision=prec) as mg:
        u = dev(p["u0"])
        st = mg.solve(dev(p["b"]), u, tol=1e-10)
        got = host(u)
        del u
    assert st["code"] == 0
    r0 = O.norm2(O.residual(3, 512, p["u0"], p["b"]))
    rk = O.norm2(O.residual(3, 512, got, p["b"]))
    assert abs(st["r0"] - r0) <= 1e-10 * r0
    assert rk <= 1.0001e-10 * r0
    assert abs(st["rk"] - rk) <= 1e-6 * rk + 1e-14 * r0


def _grads(mg, c, b, e0, K, ckpt):
    from paper_2206_05543_amd.autograd import kcycles
    cp = torch.tensor(c, dtype=torch.float32, requires_grad=True)
    bt = dev(b).requires_grad_(True)
    et = dev(e0).requires_grad_(True)
    u = kcycles(mg, cp, bt, et, K, ckpt)
    L = (u * u).sum()
    L.backward()
    return float(L.detach()), cp.grad.double().numpy(), host(bt.grad), host(et.grad), cp


def test_gradients_2d_full_size():
    need_gpu()
    w = workload("errors2d_n1024_b16")
    e0 = w["e0"]
    b = np.broadcast_to(w["b"], e0.shape).copy()
    K = 3
    say("fullsize-grad-2d")
    with make_mg(1024, 2, np.array(M9), batch=16) as mg:
        L, gc, gb, ge, cp = _grads(mg, np.array(M9), b, e0, K, torch.float64)
        c64 = cp.detach().double().numpy()
        Lw, cw, bw, ew = O.grad_kcycles(2, 1024, c64, e0, w["b"], K)
        assert abs(L - Lw) <= 1e-12 * Lw
        assert np.max(np.abs(gc - cw)) <= 1e-6 * np.abs(cw).max()
        assert np.max(np.abs(gb.sum(0) - bw)) <= 1e-10 * np.abs(bw).max()
        assert np.max(np.abs(ge - ew)) <= 1e-10 * np.abs(ew).max()
        from paper_2206_05543_amd.autograd import kcycles

        def loss(c):
            with torch.no_grad():
                u = kcycles(mg, torch.tensor(c, dtype=torch.float64), dev(b), dev(e0), K)
                return float((u * u).sum())
        j = 0
        cpl, cmi = c64.copy(), c64.copy()
        cpl[j] += 1e-6
        cmi[j] -= 1e-6
        fd = (loss(cpl) - loss(cmi)) / 2e-6
        assert abs(fd - cw[j]) <= 1e-6 * np.abs(cw).max()


def test_gradients_3d_full_size():
    need_gpu()
    w = workload("errors3d_n256_b4")
    e0 = w["e0"]
    K = 2
    c = np.array(M7)
    # one entry, FP64 checkpoints, against the oracle
    say("fullsize-grad-3d-entry0")
    with make_mg(256, 3, c, batch=1) as mg:
        L, gc, gb, ge, cp = _grads(mg, c, w["b"][None], e0[0:1], K, torch.float64)
    c64 = cp.detach().double().numpy()
    Lw, cw, bw, ew = O.grad_kcycles(3, 256, c64, e0[0:1], w["b"], K)
    assert abs(L - Lw) <= 1e-12 * Lw
    assert np.max(np.abs(gc - cw)) <= 1e-6 * np.abs(cw).max()
    assert np.max(np.abs(gb[0] - bw)) <= 1e-10 * np.abs(bw).max()
    assert np.max(np.abs(ge[0] - ew[0])) <= 1e-10 * np.abs(ew).max()
    # the batch of 4 with FP32 checkpoints against the oracle's FP32-checkpoint
    # reverse sweeps of every entry (gradient reported for FP32 parameters)
    say("fullsize-grad-3d-batch4-fp32ckpt")
    with make_mg(256, 3, c, batch=4) as mg:
        b4 = np.broadcast_to(w["b"], e0.shape).copy()
        L, gc, gb, ge, cp = _grads(mg, c, b4, e0, K, torch.float32)
    Lw, cw, bw, ew = O.grad_kcycles(3, 256, c64, e0, w["b"], K, ckpt="fp32")
    # The two sides round states that agree to ~1e-15 relative, so an entry
    # lying that close to an FP32 rounding boundary (expected: about one of
    # the 2.6e8 checkpointed entries) rounds to neighbouring FP32 values on
    # the two sides.  That changes one state entry by one FP32 ulp, and the
    # field gradients near it by the image of that change under the adjoint
    # cycles (measured: 1.3e-12, i.e. 1.2e-9 of the largest e0-gradient entry,
    # where every other entry agrees to ~1e-19).  Element-wise the bound is
    # therefore set at the scale of such a flip, 1e-8 of the largest entry;
    # in the 2-norm an isolated flip is diluted over the 6.6e7 entries, so
    # there the FP64 operation-order bound of 1e-10 applies.
    assert abs(L - Lw) <= 1e-12 * Lw
    assert np.max(np.abs(gc - cw)) <= 1e-6 * np.abs(cw).max()
    gbs = gb.sum(0)
    assert np.max(np.abs(gbs - bw)) <= 1e-8 * np.abs(bw).max()
    assert np.linalg.norm((gbs - bw).ravel()) <= 1e-10 * np.linalg.norm(bw.ravel())
    assert np.max(np.abs(ge - ew)) <= 1e-8 * np.abs(ew).max()
    assert np.linalg.norm((ge - ew).ravel()) <= 1e-10 * np.linalg.norm(ew.ravel())
