"""The C ABI's reporting and error paths on the GPU, against the oracle.

- Single-grid problems (N = 4, h0 = 1/4: the hierarchy is the exact coarsest
  solve of Section 4 alone): one cycle, a solve in every precision and the
  adjoint cycle against the oracle's dense solve and reverse sweep.
- ||b||_2 reported by every solve loop (FP64 chained 2D, FP64 3D, FP32 and
  FP16 refinement, batches) against the oracle's norm of b.
- NaN or infinity in b: every precision returns MG_ENONFINITE, and the same
  handle then solves a clean problem as a fresh one does.
- Option values that are not integers, not finite or out of range are
  rejected on the host.
- Sampled timing (MG_OPT_TIMING = 3) times exactly one fused fine-level
  launch per solve and leaves the solve's result bit for bit unchanged.
- Checkpoints written by the library: FP64 copies exactly, FP32 rounds to
  nearest even and leaves the rounded value in the iterate.
"""
import numpy as np
import pytest

import oracle as O
from paper_2206_05543_amd import M7, M9
from paper_2206_05543_amd._lib import MG_EINVAL, MG_ENONFINITE, MGError
from paper_2206_05543_amd.workloads import poisson_problem
from tests._gpu import dev, gpu, host, make_mg, need_gpu, say, torch

pytestmark = gpu

PRECS = ("fp64", "fp32_ir", "fp16_ir")


def _c(d):
    return np.array(M9 if d == 2 else M7)


@pytest.mark.parametrize("d", [2, 3])
def test_single_grid_vcycle_is_the_exact_solve(d):
    # with h0 = 1/4 the only level is solved exactly: V(u, b) = A^-1 b for any u
    need_gpu()
    batch = 2
    rng = np.random.default_rng(40 + d)
    shp = (batch,) + (3,) * d
    u0, b = rng.uniform(-1, 1, shp), rng.standard_normal(shp) * 16
    say("single-grid vcycle", d)
    with make_mg(4, d, _c(d), batch=batch) as mg:
        assert mg.num_levels == 1
        u = dev(u0)
        mg.vcycle(dev(b), u)
        torch.cuda.synchronize()
        got = host(u)
    for s in range(batch):
        want = O.direct_solve(d, 4, b[s])
        assert np.max(np.abs(got[s] - want)) <= 1e-14 * np.abs(want).max()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("d", [2, 3])
def test_single_grid_solve(d, prec):
    # one FP64 cycle reaches the exact solution.  With refinement, the inner
    # exact solve of a 3^d grid (condition number below 6) is limited by the
    # storage of the scaled residual and correction: 2^-24 (FP32) or 2^-11
    # (FP16) relative, about 1e-7 / 1e-3 reduction per step, so 1e-10 of
    # r_0 takes at most 2 / 4 steps
    need_gpu()
    rng = np.random.default_rng(50 + d)
    shp = (3,) * d
    u0, b = rng.uniform(-1, 1, shp), rng.standard_normal(shp) * 16
    want = O.direct_solve(d, 4, b)
    r0 = O.norm2(O.residual(d, 4, u0, b))
    say("single-grid solve", d, prec)
    with make_mg(4, d, _c(d), precision=prec) as mg:
        u = dev(u0)
        st = mg.solve(dev(b), u, tol=1e-10)
        got = host(u)
    assert st["code"] == 0
    assert abs(st["r0"] - r0) <= 1e-12 * r0
    assert abs(st["b_norm"] - O.norm2(b)) <= 1e-13 * O.norm2(b)
    assert O.norm2(O.residual(d, 4, got, b)) <= 1.0001e-10 * r0
    if prec == "fp64":
        assert st["cycles"] == 1
        assert np.max(np.abs(got - want)) <= 1e-14 * np.abs(want).max()
    else:
        assert st["cycles"] <= (2 if prec == "fp32_ir" else 4)


@pytest.mark.parametrize("d", [2, 3])
def test_single_grid_adjoint(d):
    # u_out = A^-1 b does not depend on u: ubar_in = 0, bbar = A^-1 ubar_out,
    # no coefficient gradient
    need_gpu()
    batch = 2
    rng = np.random.default_rng(60 + d)
    shp = (batch,) + (3,) * d
    u, b, ub = rng.uniform(-1, 1, shp), rng.standard_normal(shp), rng.standard_normal(shp)
    say("single-grid adjoint", d)
    with make_mg(4, d, _c(d), batch=batch) as mg:
        ui = torch.full(shp, 7.0, dtype=torch.float64, device="cuda")
        bb = torch.zeros(shp, dtype=torch.float64, device="cuda")
        cb = mg.vcycle_adjoint(dev(b), dev(u), dev(ub), ui, bb, [0.0] * mg.ncoef)
        torch.cuda.synchronize()
        g_u, g_b = host(ui), host(bb)
    for s in range(batch):
        wu, wb, wc = O.vcycle_adjoint(d, 4, _c(d), u[s], b[s], ub[s])
        assert np.array_equal(g_u[s], wu) and not wu.any()
        assert np.max(np.abs(g_b[s] - wb)) <= 1e-14 * np.abs(wb).max()
        assert not wc.any()
    assert cb == [0.0] * len(cb)


@pytest.mark.parametrize("prec", PRECS)
# 2D solves and 3D grids of 200+ nodes per side sum b^2 inside the first
# cycle's fused pre-smoother; smaller 3D grids take a separate pass over b
@pytest.mark.parametrize("d,N,batch", [(2, 256, 1), (2, 64, 3), (3, 64, 1), (3, 32, 2),
                                       (3, 256, 1), (3, 256, 2)])
def test_b_norm_is_reported(d, N, batch, prec):
    need_gpu()
    rng = np.random.default_rng(N + batch)
    shp = (batch,) + (N - 1,) * d
    u0 = rng.uniform(-1, 1, shp)
    b = rng.standard_normal(shp) * N
    say("b-norm", d, N, batch, prec)
    with make_mg(N, d, _c(d), batch=batch, precision=prec) as mg:
        st = mg.solve(dev(b), dev(u0), tol=1e-10)
    assert st["code"] == 0
    want = O.norm2(b)
    assert abs(st["b_norm"] - want) <= 1e-13 * want
    # rk / ||b|| is what a caller reports beside the r_0-relative rule
    assert st["rk"] / st["b_norm"] <= st["rk"] / want * (1 + 1e-12)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("d,N,bad", [(2, 64, np.nan), (2, 256, np.inf), (3, 32, -np.inf),
                                     (3, 64, np.nan)])
def test_non_finite_rhs_then_clean_solve(d, N, bad, prec):
    need_gpu()
    p = poisson_problem(d, N, seed=70, n_modes=8, kmax=N // 4)
    c = _c(d)
    u_or, k_or, hist_or = O.solve(d, N, c, p["u0"], p["b"], tol=1e-10, maxc=100)
    b_bad = p["b"].copy()
    b_bad.flat[b_bad.size // 3] = bad
    say("non-finite", d, N, bad, prec)
    with make_mg(N, d, c, precision=prec) as mg:
        with pytest.raises(MGError) as ei:
            mg.solve(dev(b_bad), dev(p["u0"]), tol=1e-10)
        assert ei.value.code == MG_ENONFINITE
        u = dev(p["u0"])
        st = mg.solve(dev(p["b"]), u, tol=1e-10)
        got = host(u)
    assert st["code"] == 0
    assert abs(st["r0"] - hist_or[0]) <= 1e-10 * hist_or[0]
    assert O.norm2(O.residual(d, N, got, p["b"])) <= 1.0001e-10 * hist_or[0]
    if prec == "fp64":
        assert st["cycles"] == k_or
        assert np.allclose(st["history"], hist_or, rtol=1e-8, atol=1e-13 * hist_or[0])


def test_option_values_are_checked():
    need_gpu()
    from paper_2206_05543_amd._lib import OPT_BATCH, OPT_MAX_CYCLES, OPT_TIMING
    with make_mg(16, 2, M9) as mg:
        for key, v in [(OPT_BATCH, float("nan")), (OPT_BATCH, float("inf")),
                       (OPT_MAX_CYCLES, -float("inf")), (OPT_BATCH, 1e12),
                       (OPT_MAX_CYCLES, 2.5), (OPT_BATCH, 0.0), (999, 1.0),
                       (OPT_TIMING, 4.0), (OPT_TIMING, -1.0)]:
            with pytest.raises(MGError) as ei:
                mg.set_option(key, v)
            assert ei.value.code == MG_EINVAL
        mg.set_option(OPT_MAX_CYCLES, 7.0)  # an integer-valued double is fine


@pytest.mark.parametrize("d", [2, 3])
def test_sampled_timing(d):
    # 2D solves chain the cycles: the one timed launch is the second fused
    # kernel, the first chained post + pre-smoother; 3D: the second cycle's
    # fused pre-smoother (both run on n = 255, where the 3D one is fused)
    need_gpu()
    N = 256
    p = poisson_problem(d, N, seed=81, n_modes=8, kmax=N // 4)
    say("sampled timing", d)
    out = []
    for timing in (0, 3):
        with make_mg(N, d, _c(d), timing=timing) as mg:
            for _ in range(2):
                u = dev(p["u0"])
                st = mg.solve(dev(p["b"]), u, tol=1e-10)
            out.append(host(u))
            if timing:
                _, n_sr = mg.timing("smooth_restrict", 0)
                _, n_ppr = mg.timing("post_pre_restrict", 0)
                assert (n_sr, n_ppr) == ((0, 2) if d == 2 else (2, 0))
                for lev in range(1, mg.num_levels):
                    assert mg.timing("smooth", lev)[1] == 0
    assert st["code"] == 0
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("d,N,batch", [(2, 64, 2), (3, 32, 1)])
def test_checkpoints(d, N, batch):
    need_gpu()
    rng = np.random.default_rng(80 + N)
    shp = (batch,) + (N - 1,) * d
    u0 = rng.uniform(-1, 1, shp) * 1e3
    say("checkpoint", d, N, batch)
    with make_mg(N, d, _c(d), batch=batch) as mg:
        u = dev(u0)
        c64 = torch.empty(shp, dtype=torch.float64, device="cuda")
        mg.checkpoint(u, c64)
        c32 = torch.empty(shp, dtype=torch.float32, device="cuda")
        mg.checkpoint(u, c32)
        torch.cuda.synchronize()
        g64, g32 = c64.cpu().numpy(), c32.cpu().numpy()
        gu = host(u)
        with pytest.raises(TypeError):
            mg.checkpoint(u, torch.empty(shp, dtype=torch.float16, device="cuda"))
    want32 = u0.astype(np.float32)
    assert np.array_equal(g64, u0)
    assert np.array_equal(g32, want32)
    assert np.array_equal(gu, want32.astype(np.float64))
