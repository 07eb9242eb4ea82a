"""Pins of the oracle's reverse-mode V-cycle: the dot-product test against
the forward cycle, symmetry of the cycle's right-hand-side map, complex-step
derivatives of the k-cycle loss through the Kronecker-matrix cycle, and
central finite differences through the loop cycle."""
import numpy as np
import pytest

import oracle as O
from oracle import dense

C9 = np.array([0.28891272760249742, 0.065661983546022137, 0.019698595063806643])
C7 = np.array([16 / 73, 2 / 73])
C27 = np.array([0.1966, 0.0397, 0.0115, 0.0037])  # 27-point 3D stencil


@pytest.mark.parametrize("d,N,c", [(2, 16, C9), (2, 32, C9), (3, 8, C7), (3, 16, C7),
                                   (3, 8, C27)])
def test_dot_product(d, N, c):
    # the cycle is affine in (u, b): V(u + du, b + db) - V(u, b) = E du + B db,
    # so <ubar_out, E du + B db> = <ubar_in, du> + <bbar, db>
    rng = np.random.default_rng(1)
    s = (N - 1,) * d
    u, b = rng.uniform(-1, 1, s), rng.standard_normal(s)
    du, db, ub = rng.standard_normal(s), rng.standard_normal(s), rng.standard_normal(s)
    dout = O.vcycle(d, N, c, u + du, b + db) - O.vcycle(d, N, c, u, b)
    ubar, bbar, _ = O.vcycle_adjoint(d, N, c, u, b, ub)
    lhs = np.vdot(ub, dout)
    rhs = np.vdot(ubar, du) + np.vdot(bbar, db)
    assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + np.linalg.norm(ub) * np.linalg.norm(dout))


@pytest.mark.parametrize("d,N,c", [(2, 32, C9), (3, 8, C7)])
def test_rhs_adjoint_is_forward_cycle(d, N, c):
    # with u = 0 the cycle is b -> B b with B symmetric, so the b-adjoint of
    # one cycle is one forward cycle from zero
    rng = np.random.default_rng(2)
    s = (N - 1,) * d
    g = rng.standard_normal(s)
    _, bbar, _ = O.vcycle_adjoint(d, N, c, np.zeros(s), rng.standard_normal(s), g)
    assert np.allclose(bbar, O.vcycle(d, N, c, np.zeros(s), g), rtol=0,
                       atol=1e-12 * np.max(np.abs(bbar)))


@pytest.mark.parametrize("d,N,c,K", [(2, 16, C9, 3), (2, 8, np.array([0.3, 0.05, 0.02]), 2),
                                     (3, 8, C7, 2), (3, 8, C27, 2), (3, 8, C27[:3], 2)])
def test_coefficient_gradient_vs_complex_step(d, N, c, K):
    rng = np.random.default_rng(3)
    e0 = rng.uniform(-1, 1, (2,) + (N - 1,) * d)
    L, cbar, _, _ = O.grad_kcycles(d, N, c, e0, np.zeros((N - 1,) * d), K)
    Ld = dense.loss_kcycles(d, N, c, e0, K)
    assert abs(L - Ld) <= 1e-12 * abs(L)
    g = dense.complex_step_grad(d, N, c, e0, K)
    assert np.max(np.abs(cbar - g)) <= 1e-9 * np.max(np.abs(g))


@pytest.mark.parametrize("d,N,c,K", [(2, 32, C9, 3), (3, 16, C7, 2)])
def test_coefficient_gradient_vs_central_differences(d, N, c, K):
    rng = np.random.default_rng(4)
    s = (N - 1,) * d
    e0 = rng.uniform(-1, 1, (2,) + s)
    b = np.zeros(s)
    _, cbar, _, _ = O.grad_kcycles(d, N, c, e0, b, K)
    step = 1e-6
    for j in range(len(c)):
        cp, cm = c.copy(), c.copy()
        cp[j] += step
        cm[j] -= step
        fd = (O.loss_kcycles(d, N, cp, e0, b, K) - O.loss_kcycles(d, N, cm, e0, b, K)) / (2 * step)
        assert abs(fd - cbar[j]) <= 1e-6 * np.max(np.abs(cbar))


def test_rhs_gradient_vs_central_differences():
    d, N, c, K = 2, 16, C9, 3
    rng = np.random.default_rng(5)
    s = (N - 1,) * d
    e0 = rng.uniform(-1, 1, (2,) + s)
    b = np.zeros(s)
    _, _, bbar, e0bar = O.grad_kcycles(d, N, c, e0, b, K)
    for _ in range(3):
        v = rng.standard_normal(s)
        t = 1e-4     # the loss is quadratic in b: central differences are exact
        fd = (O.loss_kcycles(d, N, c, e0, b + t * v, K)
              - O.loss_kcycles(d, N, c, e0, b - t * v, K)) / (2 * t)
        assert abs(fd - np.vdot(bbar, v)) <= 1e-7 * abs(fd) + 1e-12
        # the same perturbation of every initial error of the batch
        fd = (O.loss_kcycles(d, N, c, e0 + t * v, b, K)
              - O.loss_kcycles(d, N, c, e0 - t * v, b, K)) / (2 * t)
        assert abs(fd - np.vdot(e0bar.sum(0), v)) <= 1e-7 * abs(fd) + 1e-12



def _frozen_offset_loss(d, N, c, e0, K, offsets):
    # u_{k+1} = E(c) (u_k + delta_k) with the rounding offsets delta_k of the
    # base point held fixed (b = 0): the map whose derivative the
    # straight-through treatment of a rounding is, through the Kronecker
    # cycle matrix, so complex c gives its complex-step derivative
    E, _ = dense.vcycle_maps(d, N, c)
    n = (N - 1) ** d
    L = 0.0
    for s, e in enumerate(e0):
        u = e.ravel().astype(np.result_type(E, e))
        for k in range(K):
            u = E @ (u + offsets[s][k].ravel())
        L = L + np.sum(u * u)
    return L


@pytest.mark.parametrize("d,N,c,K", [(2, 16, C9, 3), (3, 8, C7, 2)])
def test_fp32_checkpoint_gradient(d, N, c, K):
    # FP32 checkpoints: every cycle starts from the FP32 rounding of its
    # input, and the reverse sweep passes derivatives through the rounding
    # unchanged.  Pins: (1) one cycle from an input already in FP32 is the
    # FP64 path exactly; (2) the loss is that of the FP64 cycles from the
    # rounded states, which differs from the FP64 loss (the rounding is
    # applied) by O(2^-24) relative; (3) the coefficient gradient equals the
    # complex-step derivative of the Kronecker-matrix cycles with the base
    # point's rounding offsets frozen, to rounding, and the FP64 path's
    # gradient does not (so the pin tells the two apart).
    rng = np.random.default_rng(6)
    s = (N - 1,) * d
    e0 = rng.uniform(-1, 1, (2,) + s)
    b = np.zeros(s)
    e32 = e0.astype(np.float32).astype(np.float64)
    r64 = O.grad_kcycles(d, N, c, e32, b, 1)
    r32 = O.grad_kcycles(d, N, c, e32, b, 1, ckpt="fp32")
    assert r64[0] == r32[0]
    for a, z in zip(r64[1:], r32[1:]):
        assert np.array_equal(a, z)
    L64, g64, _, _ = O.grad_kcycles(d, N, c, e0, b, K)
    L32, g32, _, _ = O.grad_kcycles(d, N, c, e0, b, K, ckpt="fp32")
    assert L32 != L64 and abs(L32 - L64) <= 1e-5 * L64
    offsets = []
    for e in e0:
        u, offs = e, []
        for _ in range(K):
            r = u.astype(np.float32).astype(np.float64)
            offs.append(r - u)
            u = O.vcycle(d, N, c, r, b)
        offsets.append(offs)
    assert abs(_frozen_offset_loss(d, N, c, e0, K, offsets) - L32) <= 1e-12 * L32
    g = np.zeros(len(c))
    for j in range(len(c)):
        cc = c.astype(complex)
        cc[j] += 1e-30j
        g[j] = np.imag(_frozen_offset_loss(d, N, cc, e0, K, offsets)) / 1e-30
    scale = np.max(np.abs(g))
    assert np.max(np.abs(g32 - g)) <= 1e-11 * scale
    assert np.max(np.abs(g64 - g)) >= 1e-9 * scale
