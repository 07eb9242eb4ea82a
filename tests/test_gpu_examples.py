"""The analytic problems of Section 4 (Examples 1-3) through the library.

Parity: whole solves of each example with every smoother under V(1,1) and
W(1,0) follow the oracle's residual histories and end on its iterate.  At
larger sizes, where only properties are checked: second-order
discretisation error against the exact solutions (Examples 1 and 3), the
observed rates below the two-grid LFA factors and in the smoothers' order,
Example 2 at Example 1's rates, and M7 at well under half of Jacobi's GPU
time in 3D.
"""
import numpy as np
import pytest

import oracle as O
from oracle import lfa
from paper_2206_05543_amd import SMOOTHERS
from paper_2206_05543_amd.workloads import example_problem
from tests._gpu import dev, gpu, host, make_mg, need_gpu, say

pytestmark = gpu

CYCLES = {"V": ("V11", (1, 1, 1)), "W": ("W10", (1, 0, 2))}


def _gpu_solve(p, N, c, cycle, tol=1e-10):
    with make_mg(N, p["d"], c, cycle=CYCLES[cycle][0], max_cycles=200) as mg:
        u = dev(p["u0"])
        st = mg.solve(dev(p["b"]), u, tol=tol)
        return host(u), st


def _rho_hat(st):
    k = st["cycles"]
    return (st["rk"] / st["r0"]) ** (1.0 / k)


CASES = ([(1, 128, s, cy) for s in SMOOTHERS[2] for cy in "VW"]
         + [(2, 128, s, cy) for s in ("J", "M9") for cy in "VW"]
         + [(3, 32, s, cy) for s in SMOOTHERS[3] for cy in "VW"])


@pytest.mark.parametrize("example,N,smoother,cycle", CASES,
                         ids=[f"ex{e}-{n}-{s}-{c}" for e, n, s, c in CASES])
def test_example_solve_parity(example, N, smoother, cycle):
    need_gpu()
    p = example_problem(example, N, seed=example)
    d = p["d"]
    c = np.array(SMOOTHERS[d][smoother])
    nu1, nu2, gamma = CYCLES[cycle][1]
    u_or, k_or, hist_or = O.solve(d, N, c, p["u0"], p["b"], tol=1e-10, maxc=200,
                                  nu1=nu1, nu2=nu2, gamma=gamma)
    say("example", example, N, smoother, cycle)
    got, st = _gpu_solve(p, N, c, cycle)
    assert st["code"] == 0
    assert st["cycles"] == k_or
    assert np.allclose(st["history"], hist_or, rtol=1e-8, atol=1e-13 * hist_or[0])
    assert np.max(np.abs(got - u_or)) <= 1e-9 * np.abs(u_or).max()


@pytest.mark.parametrize("example,Ns", [(1, (1024, 2048)), (3, (128, 256))])
def test_second_order_error_at_scale(example, Ns):
    need_gpu()
    errs = []
    for N in Ns:
        p = example_problem(example, N)
        d = p["d"]
        c = np.array(SMOOTHERS[d]["M9" if d == 2 else "M7"])
        say("example-error", example, N)
        got, st = _gpu_solve(p, N, c, "V", tol=1e-13)
        assert st["code"] == 0
        errs.append(np.abs(got - p["u"]).max())
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.03)


def _rates(example, N, cycle, smoothers=None):
    p = example_problem(example, N)
    d = p["d"]
    out = {}
    for name, c in SMOOTHERS[d].items():
        if smoothers and name not in smoothers:
            continue
        say("example-rates", example, N, name, cycle)
        _, st = _gpu_solve(p, N, np.array(c), cycle)
        assert st["code"] == 0
        nu = sum(CYCLES[cycle][1][:2])
        out[name] = (st["cycles"], _rho_hat(st),
                     lfa.two_grid_factor(d, np.array(c), nu, 256 if d == 2 else 64),
                     st["elapsed_ms"])
    return out


@pytest.mark.parametrize("cycle", ["V", "W"])
def test_rates_at_scale_2d(cycle):
    need_gpu()
    r1 = _rates(1, 1024, cycle)
    r2 = _rates(2, 1024, cycle)
    for s, (k, rho, tg, _) in r1.items():
        assert rho <= tg, s
        assert r2[s][1] == pytest.approx(rho, rel=0.02), s
    if cycle == "W":
        assert sorted(r1, key=lambda s: r1[s][1]) == ["M9", "M5", "Vanka", "TW5", "J"]
    else:
        assert r1["M9"][1] < min(r1[s][1] for s in ("M5", "Vanka", "TW5", "J"))
        assert r1["J"][1] > max(r1[s][1] for s in ("M5", "Vanka", "TW5"))


def test_m7_time_against_jacobi_3d():
    need_gpu()
    for cycle in ("V", "W"):
        r = _rates(3, 128, cycle)
        assert r["M7"][1] <= r["M7"][2] and r["J"][1] <= r["J"][2]
        assert r["M7"][0] <= 0.55 * r["J"][0]
        assert r["M7"][3] <= 0.7 * r["J"][3]
