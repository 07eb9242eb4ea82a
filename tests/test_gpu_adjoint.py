"""The hand-written adjoint V-cycle and the autograd wrapper against the CPU
oracle's reverse-mode cycle, the dot-product identity of the forward cycle,
and central finite differences of the k-cycle loss.

Tolerances.  The adjoint of one cycle is a fixed linear map of norm O(1)
(in the units of its inputs), evaluated in FP64 with a different operation
order than the oracle: element-wise agreement to 1e-11 of the largest entry.
Coefficient gradients are sums of O(n) products; 1e-9 relative.  Finite
differences in FP64 with step 1e-6 (the loss is polynomial in c, so the
central difference has O(1e-12) truncation and O(1e-10) cancellation error
relative to the derivative): 1e-6 relative.
"""
import numpy as np
import pytest

import oracle as O
from paper_2206_05543_amd import M7, M9
from tests._gpu import dev, gpu, host, make_mg, need_gpu, say, torch

pytestmark = gpu


def _c(d):
    return np.array(M9 if d == 2 else M7)


@pytest.mark.parametrize("d,N,batch", [(2, 8, 1), (2, 64, 2), (2, 128, 1), (3, 8, 1),
                                       (3, 16, 2), (3, 32, 1)])
def test_adjoint_cycle_matches_oracle(d, N, batch):
    need_gpu()
    rng = np.random.default_rng(10 * N + batch)
    shp = (batch,) + (N - 1,) * d
    u = rng.uniform(-1, 1, shp)
    b = rng.standard_normal(shp) * 10
    ub = rng.standard_normal(shp)
    say("adjoint", d, N, batch)
    with make_mg(N, d, _c(d), batch=batch) as mg:
        ubar_in = torch.empty(shp, dtype=torch.float64, device="cuda")
        bbar = torch.zeros(shp, dtype=torch.float64, device="cuda")
        cbar = mg.vcycle_adjoint(dev(b), dev(u), dev(ub), ubar_in, bbar, [0.0] * mg.ncoef)
        torch.cuda.synchronize()
        g_u, g_b = host(ubar_in), host(bbar)
    want_c = np.zeros(mg.ncoef)
    for s in range(batch):
        wu, wb, wc = O.vcycle_adjoint(d, N, _c(d), u[s], b[s], ub[s])
        assert np.max(np.abs(g_u[s] - wu)) <= 1e-11 * np.abs(wu).max()
        assert np.max(np.abs(g_b[s] - wb)) <= 1e-11 * np.abs(wb).max()
        want_c += wc
    assert np.max(np.abs(np.array(cbar) - want_c)) <= 1e-9 * np.abs(want_c).max()


@pytest.mark.parametrize("d,N", [(2, 256), (3, 64)])
def test_adjoint_dot_product(d, N):
    # <ubar_out, V(u+du, b+db) - V(u, b)> = <ubar_in, du> + <bbar, db>
    need_gpu()
    rng = np.random.default_rng(N)
    shp = (N - 1,) * d
    u, b = rng.uniform(-1, 1, shp), rng.standard_normal(shp) * N
    du, db, ub = rng.standard_normal(shp), rng.standard_normal(shp) * N, rng.standard_normal(shp)
    say("adjoint-dot", d, N)
    with make_mg(N, d, _c(d)) as mg:
        x1, x0 = dev(u + du), dev(u)
        mg.vcycle(dev(b + db), x1)
        mg.vcycle(dev(b), x0)
        ui = torch.empty_like(x0)
        bb = torch.zeros_like(x0)
        mg.vcycle_adjoint(dev(b), dev(u), dev(ub), ui, bb, [0.0] * mg.ncoef)
        torch.cuda.synchronize()
        dout = host(x1) - host(x0)
        lhs = float(np.vdot(ub, dout))
        rhs = float(np.vdot(host(ui), du) + np.vdot(host(bb), db))
    assert abs(lhs - rhs) <= 1e-10 * (abs(lhs) + np.linalg.norm(ub) * np.linalg.norm(dout))


def _loss_gpu(mg, c, b, e0, K):
    from paper_2206_05543_amd.autograd import kcycles
    u = kcycles(mg, torch.tensor(c, dtype=torch.float64), b, e0, K)
    return float((u * u).sum())


@pytest.mark.parametrize("d,N,batch,K", [(2, 64, 2, 3), (3, 32, 2, 2)])
def test_autograd_matches_oracle_and_fd(d, N, batch, K):
    from paper_2206_05543_amd.autograd import kcycles
    need_gpu()
    rng = np.random.default_rng(7 + N)
    shp = (batch,) + (N - 1,) * d
    e0 = rng.uniform(-1, 1, shp)
    b = np.zeros(shp)
    c = _c(d)
    say("autograd", d, N, batch, K)
    with make_mg(N, d, c, batch=batch) as mg:
        cp = torch.tensor(c, dtype=torch.float32, requires_grad=True)
        bt = dev(b).requires_grad_(True)
        et = dev(e0).requires_grad_(True)
        u = kcycles(mg, cp, bt, et, K)
        L = (u * u).sum()
        L.backward()
        gc = cp.grad.double().numpy()
        gb, ge = host(bt.grad), host(et.grad)
        # oracle: same loss through the loop cycle and its reverse sweep, with
        # the FP32 parameters promoted to FP64
        c64 = cp.detach().double().numpy()
        Lw, cw, bw, ew = O.grad_kcycles(d, N, c64, e0, b[0], K)
        assert abs(float(L.detach()) - Lw) <= 1e-12 * Lw
        # gradient w.r.t. the FP32 parameters is reported in FP32
        assert np.max(np.abs(gc - cw)) <= 1e-6 * np.abs(cw).max()
        assert np.max(np.abs(gb.sum(0) - bw)) <= 1e-10 * np.abs(bw).max()
        assert np.max(np.abs(ge - ew)) <= 1e-10 * np.abs(ew).max()
        # central differences on the FP64 promotion of the parameters
        for j in range(len(c)):
            cpl, cmi = c64.copy(), c64.copy()
            cpl[j] += 1e-6
            cmi[j] -= 1e-6
            fd = (_loss_gpu(mg, cpl, dev(b), dev(e0), K) - _loss_gpu(mg, cmi, dev(b), dev(e0), K)) / 2e-6
            assert abs(fd - cw[j]) <= 1e-6 * np.abs(cw).max()


@pytest.mark.parametrize("d,N,batch,K", [(3, 32, 2, 2), (2, 64, 2, 3)])
def test_fp32_checkpoints_match_oracle(d, N, batch, K):
    # FP32 checkpoints: each cycle starts from the FP32 rounding of its input
    # and the derivative passes through the rounding unchanged; the oracle
    # does the same on its own states (grad_kcycles(..., ckpt="fp32")).
    # The two sides round states that agree to ~1e-15, so at most a few
    # entries can round to neighbouring FP32 values (a 2^-24 change of that
    # entry): agreement to 1e-9 of the largest entry.
    from paper_2206_05543_amd.autograd import kcycles
    need_gpu()
    rng = np.random.default_rng(3)
    e0 = rng.uniform(-1, 1, (batch,) + (N - 1,) * d)
    b = np.zeros((N - 1,) * d)
    c = _c(d)
    say("fp32-ckpt", d, N, batch, K)
    with make_mg(N, d, c, batch=batch) as mg:
        cp = torch.tensor(c, dtype=torch.float64, requires_grad=True)
        bt = dev(np.zeros_like(e0)).requires_grad_(True)
        et = dev(e0).requires_grad_(True)
        u = kcycles(mg, cp, bt, et, K, torch.float32)
        L = (u * u).sum()
        L.backward()
        gc, gb, ge = cp.grad.numpy().copy(), host(bt.grad), host(et.grad)
    Lw, cw, bw, ew = O.grad_kcycles(d, N, c, e0, b, K, ckpt="fp32")
    assert abs(float(L.detach()) - Lw) <= 1e-12 * Lw
    assert np.max(np.abs(gc - cw)) <= 1e-9 * np.abs(cw).max()
    assert np.max(np.abs(gb.sum(0) - bw)) <= 1e-9 * np.abs(bw).max()
    assert np.max(np.abs(ge - ew)) <= 1e-9 * np.abs(ew).max()
    # and the rounding is really applied: with FP64 checkpoints the loss and the
    # field gradients move by more than the tolerances above (measured on these
    # inputs: loss 5e-10 relative against the 1e-12 bound, e0-gradient 2e-8
    # against 1e-9; the c-gradient moves by only 4e-10 in 3D, so it is not used)
    L64, _, _, ew64 = O.grad_kcycles(d, N, c, e0, b, K)
    assert abs(float(L.detach()) - L64) > 100 * 1e-12 * L64
    assert np.max(np.abs(ge - ew64)) > 10 * 1e-9 * np.abs(ew).max()
