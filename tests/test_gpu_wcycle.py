"""Parity of the W(1,0) cycle (MG_CYCLE_W10) with the oracle's general cycle.

Section 4 compares the smoothers under V(1,1) and W(1,0).  The oracle's
cycle takes nu1 = 1, nu2 = 0, gamma = 2 for W(1,0) (pinned on the CPU
against the dense matrix recursion); here the library's W cycle is compared
with it element by element, through whole solves (residual histories), at
the full workload sizes, and in FP32 refinement.
"""
import numpy as np
import pytest

import oracle as O
from paper_2206_05543_amd import M7, M9, JACOBI_2D, M5
from paper_2206_05543_amd._lib import MGError
from paper_2206_05543_amd.workloads import poisson_problem, workload
from tests._gpu import dev, gpu, host, make_mg, need_gpu, say, torch

pytestmark = gpu


def _c(d):
    return np.array(M9 if d == 2 else M7)


@pytest.mark.parametrize("d,N,batch", [(2, 8, 1), (2, 64, 1), (2, 256, 2), (2, 1024, 1),
                                       (3, 8, 1), (3, 32, 2), (3, 64, 1), (3, 128, 1)])
def test_wcycle_parity(d, N, batch):
    need_gpu()
    rng = np.random.default_rng(N + 3 * batch)
    shp = (batch,) + (N - 1,) * d
    u0 = rng.uniform(-1, 1, shp)
    b = rng.standard_normal(shp) * 10
    say("wcycle", d, N, batch)
    with make_mg(N, d, _c(d), batch=batch, cycle="W10") as mg:
        u = dev(u0)
        mg.vcycle(dev(b), u)
        torch.cuda.synchronize()
        got = host(u)
    for s in range(batch):
        want = O.cycle(d, N, _c(d), u0[s], b[s], nu1=1, nu2=0, gamma=2)
        scale = max(np.abs(want).max(), np.abs(u0[s]).max())
        assert np.max(np.abs(got[s] - want)) <= 1e-12 * scale


@pytest.mark.parametrize("d,N,tail_N", [(2, 256, 4), (2, 256, 8), (2, 256, 16), (2, 256, 32),
                                        (2, 256, 64), (3, 64, 4), (3, 64, 8), (3, 64, 16)])
def test_wcycle_tail_depths(d, N, tail_N):
    # the coarse levels' W(1,0) visits run in the single-workgroup tail from
    # tail_N down; every split between host levels and tail levels gives the
    # oracle's cycle
    need_gpu()
    rng = np.random.default_rng(N + tail_N)
    shp = (2,) + (N - 1,) * d
    u0 = rng.uniform(-1, 1, shp)
    b = rng.standard_normal(shp) * 10
    say("wcycle-tail", d, N, tail_N)
    with make_mg(N, d, _c(d), batch=2, cycle="W10", tail_N=tail_N) as mg:
        u = dev(u0)
        mg.vcycle(dev(b), u)
        torch.cuda.synchronize()
        got = host(u)
    for s in range(2):
        want = O.cycle(d, N, _c(d), u0[s], b[s], nu1=1, nu2=0, gamma=2)
        scale = max(np.abs(want).max(), np.abs(u0[s]).max())
        assert np.max(np.abs(got[s] - want)) <= 1e-12 * scale


@pytest.mark.parametrize("d,N,coeffs", [(2, 64, M9), (2, 64, JACOBI_2D), (2, 64, M5),
                                        (2, 256, M9), (3, 32, M7), (3, 64, M7)],
                         ids=["2d64-M9", "2d64-J", "2d64-M5", "2d256-M9", "3d32-M7", "3d64-M7"])
def test_wcycle_solve_history(d, N, coeffs):
    need_gpu()
    p = poisson_problem(d, N, seed=13, n_modes=8, kmax=N // 4)
    c = np.array(coeffs)
    u_or, k_or, hist_or = O.solve(d, N, c, p["u0"], p["b"], tol=1e-10, maxc=100,
                                  nu1=1, nu2=0, gamma=2)
    say("wsolve", d, N, coeffs)
    with make_mg(N, d, c, cycle="W10") as mg:
        u = dev(p["u0"])
        st = mg.solve(dev(p["b"]), u, tol=1e-10)
        got = host(u)
    assert st["code"] == 0
    assert st["cycles"] == k_or
    assert np.allclose(st["history"], hist_or, rtol=1e-8, atol=1e-13 * hist_or[0])
    assert np.max(np.abs(got - u_or)) <= 1e-9 * np.abs(u_or).max()


@pytest.mark.parametrize("name", ["poisson2d_n4096", "poisson3d_n256"])
def test_full_size_wcycle(name):
    need_gpu()
    p = workload(name)
    d = 2 if "2d" in name else 3
    N = 4096 if d == 2 else 256
    c = _c(d)
    say("full-size-w", name)
    with make_mg(N, d, c, cycle="W10") as mg:
        u = dev(p["u0"])
        mg.vcycle(dev(p["b"]), u)
        torch.cuda.synchronize()
        got = host(u)
    want = O.cycle(d, N, c, p["u0"], p["b"], nu1=1, nu2=0, gamma=2)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("prec", ["fp32_ir", "fp16_ir"])
def test_wcycle_refinement(prec):
    # low-precision W(1,0) cycles inside FP64 refinement reach the same
    # relative residual; the oracle computes the residual of the result
    need_gpu()
    d, N = 3, 64
    p = poisson_problem(d, N, seed=17, n_modes=8, kmax=N // 4)
    say("wcycle-ir", prec)
    with make_mg(N, d, _c(d), precision=prec, cycle="W10") as mg:
        u = dev(p["u0"])
        st = mg.solve(dev(p["b"]), u, tol=1e-10)
        got = host(u)
    assert st["code"] == 0
    r0 = O.norm2(O.residual(d, N, p["u0"], p["b"]))
    assert O.norm2(O.residual(d, N, got, p["b"])) <= 1.0001e-10 * r0


def test_adjoint_rejects_wcycle():
    need_gpu()
    d, N = 2, 16
    z = torch.zeros((N - 1) ** d, dtype=torch.float64, device="cuda")
    say("wcycle-adjoint-rejected")
    with make_mg(N, d, _c(d), cycle="W10") as mg:
        with pytest.raises(MGError):
            mg.vcycle_adjoint(z, z, z, z.clone(), z.clone(), [0.0] * 3)
        # switching back restores the adjoint
        mg.set_cycle("V11")
        mg.vcycle_adjoint(z, z, z, z.clone(), z.clone(), [0.0] * 3)
