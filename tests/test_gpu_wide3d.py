"""The 19- and 27-point 3D smoothers (the wider stencils of the closing remark
of Section 3.2: the 7-point family plus edge and corner neighbours) against
the CPU oracle: the wide smoother kernel from a guess, from zero and with the
fused coarse-grid correction in every storage precision and launch shape,
the LDS tail, V(1,1) and W(1,0) cycles and solves, FP32/FP16 refinement, the
adjoint cycle's coefficient gradients for three and four coefficients, and
the handle-free cycle.

Tolerances are those of the 7-point tests (test_gpu_kernels.py,
test_gpu_cycle.py, test_gpu_adjoint.py): the sweep bound 64 eps (max|u| +
h^2 max|b|) holds because the weights of M27 sum to 0.60 in h^2 units
(c0 + 6 c1 + 12 c2 + 8 c3), below the 0.63 of M9 the bound was derived for.
"""
import numpy as np
import pytest

import oracle as O
from paper_2206_05543_amd import M19, M27
from tests._gpu import EPS16, EPS32, EPS64, dev, gpu, host, make_mg, need_gpu, say, torch

pytestmark = gpu

STORE = {"fp64": np.float64, "fp32_ir": np.float32, "fp16_ir": np.float16}
EPS = {"fp64": EPS64, "fp32_ir": EPS32, "fp16_ir": EPS32}
TDT = {"fp64": torch.float64, "fp32_ir": torch.float32, "fp16_ir": torch.float16}
# a stencil with negative edge and corner weights, to catch sign and offset
# mistakes that the (positive) optima could hide
CNEG = (0.21, 0.03, -0.004, 0.006)
SETS = {"M19": M19, "M27": M27, "neg": CNEG}


def _rt(a, prec):
    return a.astype(STORE[prec]).astype(np.float64)


def _sigma(prec, N):
    return 1.0 if prec == "fp64" else float(N) * N


def _tol(prec, *mags, out_mag=0.0):
    t = 64 * EPS[prec] * sum(mags)
    if prec == "fp16_ir":
        t += EPS16 * out_mag
    return t


@pytest.mark.parametrize("cs", list(SETS))
@pytest.mark.parametrize("prec", ["fp64", "fp32_ir", "fp16_ir"])
@pytest.mark.parametrize("N,level", [(8, 0), (32, 0), (32, 1), (128, 0), (256, 0)])
def test_wide_smooth_parity(N, level, prec, cs):
    # N = 256 runs the fine-grid launch shapes (64x16 tiles in FP64, 256x8
    # in FP32/FP16), the others the small- and mid-grid ones
    need_gpu()
    c = np.array(SETS[cs])
    Nl = N >> level
    rng = np.random.default_rng(700 + N + level)
    shp, shc = (Nl - 1,) * 3, (Nl // 2 - 1,) * 3
    sig, sigc = _sigma(prec, Nl), _sigma(prec, Nl // 2)
    us = _rt(rng.uniform(-1, 1, shp), prec)
    b = _rt(rng.uniform(-1, 1, shp) * (1.0 if prec != "fp64" else Nl * Nl), prec)
    ecs = _rt(rng.uniform(-1, 1, shc), prec)
    say("wide-smooth", N, level, prec, cs)
    t = TDT[prec]
    with make_mg(N, 3, c) as mg:
        out, out0, outc = (torch.empty(shp, dtype=t, device="cuda") for _ in range(3))
        mg.sweep("smooth", level, prec, dev(us, t), dev(b, t), out)
        mg.sweep("smooth_zero", level, prec, None, dev(b, t), out0)
        mg.sweep_correct(level, prec, dev(us, t), dev(ecs, t), dev(b, t), outc)
        torch.cuda.synchronize()
        got, got0, gotc = host(out), host(out0), host(outc)
    h2 = 1.0 / (Nl * Nl)
    bm = h2 * sig * np.abs(b).max()
    want = O.smooth(3, Nl, c, us / sig, b) * sig
    assert np.max(np.abs(got - want)) <= _tol(prec, np.abs(us).max(), bm,
                                               out_mag=np.abs(want).max())
    want0 = O.apply_W(3, Nl, c, b) * sig
    assert np.max(np.abs(got0 - want0)) <= _tol(prec, bm, out_mag=np.abs(want0).max())
    v = O.prolong_add(3, Nl, ecs / sigc, us / sig)
    wantc = O.smooth(3, Nl, c, v, b) * sig
    assert np.max(np.abs(gotc - wantc)) <= _tol(prec, np.abs(us).max() + 4 * np.abs(ecs).max(),
                                                 bm, out_mag=np.abs(wantc).max())


@pytest.mark.parametrize("cs", ["M19", "M27"])
@pytest.mark.parametrize("prec", ["fp64", "fp32_ir", "fp16_ir"])
@pytest.mark.parametrize("N,level", [(16, 0), (32, 1), (64, 1)])
def test_wide_coarse_cycle_parity(N, level, prec, cs):
    # zero-guess cycles: the LDS tail (16^3 and below) and the level kernels
    need_gpu()
    c = np.array(SETS[cs])
    Nl = N >> level
    rng = np.random.default_rng(800 + N)
    shp = (Nl - 1,) * 3
    b = _rt(rng.uniform(-1, 1, shp), prec)
    say("wide-coarse", N, level, prec, cs)
    with make_mg(N, 3, c, precision=prec) as mg:
        e = torch.empty(shp, dtype=TDT[prec], device="cuda")
        mg.coarse_cycle(level, prec, dev(b, TDT[prec]), e)
        torch.cuda.synchronize()
        got = host(e)
    want = O.vcycle(3, Nl, c, np.zeros(shp), b) * _sigma(prec, Nl)
    tol = {"fp64": 1e-12, "fp32_ir": 2e-5, "fp16_ir": 2e-2}[prec] * np.abs(want).max()
    assert np.max(np.abs(got - want)) <= tol


@pytest.mark.parametrize("cs", list(SETS))
@pytest.mark.parametrize("N,batch", [(8, 1), (32, 2), (64, 1)])
def test_wide_vcycle_matches_oracle(N, batch, cs):
    need_gpu()
    c = np.array(SETS[cs])
    rng = np.random.default_rng(900 + N)
    shp = (batch,) + (N - 1,) * 3
    u0 = rng.uniform(-1, 1, shp)
    b = rng.standard_normal(shp) * N
    say("wide-vcycle", N, batch, cs)
    with make_mg(N, 3, c, batch=batch) as mg:
        u = dev(u0)
        mg.vcycle(dev(b), u)
        torch.cuda.synchronize()
        got = host(u)
    for s in range(batch):
        want = O.vcycle(3, N, c, u0[s], b[s])
        assert np.max(np.abs(got[s] - want)) <= 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("cycle", ["V11", "W10"])
@pytest.mark.parametrize("cs", ["M19", "M27"])
def test_wide_solve_history_matches_oracle(cs, cycle):
    # the whole solve loop (norm partials of the wide pre-smoother) against
    # the oracle's residual history, cycle by cycle
    need_gpu()
    c = np.array(SETS[cs])
    N = 64
    rng = np.random.default_rng(77)
    u0 = rng.uniform(-1, 1, (N - 1,) * 3)
    b = rng.standard_normal((N - 1,) * 3) * N
    gamma, nu2 = (1, 1) if cycle == "V11" else (2, 0)
    u_or, k_or, hist_or = O.solve(3, N, c, u0, b, tol=1e-10, maxc=100, nu1=1, nu2=nu2,
                                  gamma=gamma)
    say("wide-solve", cs, cycle)
    with make_mg(N, 3, c, cycle=cycle) as mg:
        u = dev(u0)
        st = mg.solve(dev(b), u, tol=1e-10)
        got = host(u)
    assert st["code"] == 0 and st["cycles"] == k_or
    assert np.allclose(st["history"], hist_or, rtol=1e-8, atol=1e-13 * hist_or[0])
    assert np.max(np.abs(got - u_or)) <= 1e-9 * np.abs(u_or).max()


def test_wide_fine_grid_solve_norms():
    # 3D N = 256: the fine level runs the wide smoother's norm variant on
    # the fine-grid launch shape; every reported norm is the oracle's
    # residual of an iterate the solve produced (the first and the last)
    need_gpu()
    c = np.array(M27)
    N = 256
    rng = np.random.default_rng(31)
    u0 = rng.uniform(-1, 1, (N - 1,) * 3)
    b = rng.standard_normal((N - 1,) * 3) * 100.0
    say("wide-solve-256")
    with make_mg(N, 3, c, max_cycles=3) as mg:
        u = dev(u0)
        st = mg.solve(dev(b), u, tol=1e-10)
        got = host(u)
    r0 = O.norm2(O.residual(3, N, u0, b))
    rk = O.norm2(O.residual(3, N, got, b))
    assert st["code"] == -3 and st["cycles"] == 3  # the cycle limit, by design
    assert abs(st["r0"] - r0) <= 1e-12 * r0
    assert abs(st["rk"] - rk) <= 1e-9 * rk
    assert abs(st["b_norm"] - O.norm2(b)) <= 1e-12 * O.norm2(b)


@pytest.mark.parametrize("prec", ["fp32_ir", "fp16_ir"])
def test_wide_refinement_reaches_tolerance(prec):
    need_gpu()
    c = np.array(M27)
    N = 64
    rng = np.random.default_rng(5)
    u0 = rng.uniform(-1, 1, (N - 1,) * 3)
    b = rng.standard_normal((N - 1,) * 3) * N
    ref, _, _ = O.solve(3, N, c, u0, b, tol=1e-14, maxc=100)
    say("wide-ir", prec)
    with make_mg(N, 3, c, precision=prec) as mg:
        u = dev(u0)
        st = mg.solve(dev(b), u, tol=1e-10)
        got = host(u)
    assert st["code"] == 0
    r0 = O.norm2(O.residual(3, N, u0, b))
    assert O.norm2(O.residual(3, N, got, b)) <= 1e-10 * r0
    with make_mg(N, 3, c) as mg:
        u = dev(u0)
        mg.solve(dev(b), u, tol=1e-10)
        err64 = np.linalg.norm(host(u) - ref)
    assert np.linalg.norm(got - ref) <= err64 + 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("cs", ["M19", "M27", "neg"])
@pytest.mark.parametrize("N,batch", [(8, 1), (16, 2), (32, 1)])
def test_wide_adjoint_cycle_matches_oracle(N, batch, cs):
    need_gpu()
    c = np.array(SETS[cs])
    rng = np.random.default_rng(40 + N + batch)
    shp = (batch,) + (N - 1,) * 3
    u = rng.uniform(-1, 1, shp)
    b = rng.standard_normal(shp) * 10
    ub = rng.standard_normal(shp)
    say("wide-adjoint", N, batch, cs)
    with make_mg(N, 3, c, batch=batch) as mg:
        ubar_in = torch.empty(shp, dtype=torch.float64, device="cuda")
        bbar = torch.zeros(shp, dtype=torch.float64, device="cuda")
        cbar = mg.vcycle_adjoint(dev(b), dev(u), dev(ub), ubar_in, bbar, [0.0] * mg.ncoef)
        torch.cuda.synchronize()
        g_u, g_b = host(ubar_in), host(bbar)
    assert len(cbar) == len(c)
    want_c = np.zeros(len(c))
    for s in range(batch):
        wu, wb, wc = O.vcycle_adjoint(3, N, c, u[s], b[s], ub[s])
        assert np.max(np.abs(g_u[s] - wu)) <= 1e-11 * np.abs(wu).max()
        assert np.max(np.abs(g_b[s] - wb)) <= 1e-11 * np.abs(wb).max()
        want_c += wc
    assert np.max(np.abs(np.array(cbar) - want_c)) <= 1e-9 * np.abs(want_c).max()


def test_wide_fused_restriction_entry_points_refuse():
    # the fused smoother + restriction kernels carry the 7-point stencil
    need_gpu()
    from paper_2206_05543_amd._lib import MGError
    N = 16
    z = torch.zeros((N - 1,) * 3, dtype=torch.float64, device="cuda")
    zc = torch.zeros((N // 2 - 1,) * 3, dtype=torch.float64, device="cuda")
    with make_mg(N, 3, M27) as mg:
        with pytest.raises(MGError, match="7-point"):
            mg.sweep_smooth_restrict(0, "fp64", z, z, z.clone(), zc)
        with pytest.raises(MGError, match="7-point"):
            mg.sweep_zero_restrict(0, "fp64", z, z.clone(), zc)


def test_wide_noalloc_cycle_matches_handle_cycle():
    need_gpu()
    from paper_2206_05543_amd._lib import vcycle_noalloc
    N = 64
    rng = np.random.default_rng(2)
    u0 = rng.uniform(-1, 1, (N - 1,) * 3)
    b = rng.standard_normal((N - 1,) * 3) * N
    say("wide-noalloc")
    u1 = dev(u0)
    vcycle_noalloc(N, 3, M27, dev(b), u1)
    with make_mg(N, 3, M27) as mg:
        u2 = dev(u0)
        mg.vcycle(dev(b), u2)
        torch.cuda.synchronize()
    assert torch.equal(u1, u2)
