"""The minimax coefficient search against the optima the paper prints.

Section 3.1 (the best 5-point stencil, mu = 9/41 at M5; Theorem 3.1,
mu = (9 + 8 sqrt 10)/215 at M9) and Section 3.2 (Theorem 3.2, mu = 25/73 at
M7): the search over each family recovers the printed smoothing factor and,
with the optimal damping folded in, the smoother's coefficients.  The 3D
19- and 27-point families, which the paper mentions without coefficients,
are checked by what holds for any correct search: the family's symbol
equals the stencil's Fourier sum taken offset by offset, the families nest
(so their optima cannot be worse than 25/73), and the optimum does not
depend on the sampling of the high frequencies.  Their optimal values are
pinned without the search's optimiser: an exhaustive scan of the free
ratios (coarse over a wide box, fine around the optimum) finds no stencil
that beats the searched one on the same frequency sample, the smoothing
factor of the searched stencil recomputed with the continuous extremes of
the symbol (bounded local maximisation, not sampling) matches, and every
small move of the ratios raises that continuous smoothing factor.
"""
import itertools
import math

from scipy.optimize import minimize

import numpy as np
import pytest

from oracle import lfa, search
from paper_2206_05543_amd import M5, M7, M9

MU_M9 = (9.0 + 8.0 * math.sqrt(10.0)) / 215.0


@pytest.mark.parametrize("d,family,mu,coeffs", [
    (2, "5pt", 9.0 / 41.0, M5[:2]),
    (2, "9pt", MU_M9, M9),
    (3, "7pt", 25.0 / 73.0, M7),
], ids=["M5", "M9-thm3.1", "M7-thm3.2"])
def test_search_recovers_paper_optimum(d, family, mu, coeffs):
    r = search.search(d, family)
    assert r["mu"] == pytest.approx(mu, rel=1e-6)
    assert np.allclose(r["coeffs"], coeffs, rtol=1e-5)


def _brute_symbol(d, weights, th):
    # sum over the stencil's offsets o of w(o) exp(i theta . o), real part;
    # weights: function of the number of nonzero offset components
    out = np.zeros(len(th))
    for o in itertools.product((-1, 0, 1), repeat=d):
        w = weights[sum(abs(v) for v in o)]
        out += w * np.cos(th @ np.array(o, dtype=float))
    return out


@pytest.mark.parametrize("d,k", [(2, 1), (2, 2), (3, 1), (3, 2), (3, 3)])
def test_family_symbol_is_the_stencils_fourier_sum(d, k):
    rng = np.random.default_rng(d * 10 + k)
    c = rng.uniform(0.1, 1.0, k + 1)
    th = rng.uniform(-np.pi, np.pi, (500, d))
    w = list(c) + [0.0] * (4 - len(c))
    want = lfa.symbol_A(d, th) * _brute_symbol(d, w, th)
    got = search.symbol_product(d, c, np.cos(th))
    assert np.max(np.abs(got - want)) < 1e-12


def test_wider_3d_families():
    r7 = search.search(3, "7pt", m=24, refine_m=60)
    r19 = search.search(3, "19pt", m=24, refine_m=60)
    r27 = search.search(3, "27pt", m=24, refine_m=60)
    # nested families: each optimum is at least as good as the narrower one
    assert r19["mu"] <= r7["mu"] + 1e-9
    assert r27["mu"] <= r19["mu"] + 1e-9
    assert r27["mu"] < 0.9 * 25.0 / 73.0
    # the sampled optimum holds on random high frequencies off the grid
    rng = np.random.default_rng(0)
    th = rng.uniform(-np.pi, np.pi, (200000, 3))
    high = np.any(np.abs(th) >= np.pi / 2, axis=1)
    th = th[high]
    for r in (r19, r27):
        c = np.asarray(r["coeffs"])
        w = list(c) + [0.0] * (4 - len(c))
        amp = np.abs(1.0 - lfa.symbol_A(3, th) * _brute_symbol(3, w, th))
        assert amp.max() <= r["mu"] * (1.0 + 2e-3)


@pytest.fixture(scope="module")
def wide_optima():
    return {fam: search.search(3, fam, m=24, refine_m=60) for fam in ("19pt", "27pt")}


def _mu_sampled(ratios, x):
    """mu_opt of the stencils with the given ratios (rows, c0 = 1) on the
    cosine sample x, evaluated for many stencils at once."""
    s1 = x.sum(1)
    s2 = x[:, 0] * x[:, 1] + x[:, 0] * x[:, 2] + x[:, 1] * x[:, 2]
    s3 = x.prod(1)
    a = 2.0 * (3.0 - s1)
    out = np.empty(len(ratios))
    for i in range(0, len(ratios), 2000):
        g = ratios[i:i + 2000]
        m = 1.0 + 2.0 * g[:, 0:1] * s1 + 4.0 * g[:, 1:2] * s2
        if g.shape[1] > 2:
            m = m + 8.0 * g[:, 2:3] * s3
        p = a * m
        l0, l1 = p.min(1), p.max(1)
        with np.errstate(divide="ignore", invalid="ignore"):
            out[i:i + 2000] = np.where(l0 > 0, (l1 - l0) / (l1 + l0), 1.0)
    return out


def _grid(axes):
    return np.stack(np.meshgrid(*axes, indexing="ij"), -1).reshape(-1, len(axes))


@pytest.mark.parametrize("fam", ["19pt", "27pt"])
def test_wider_3d_optimum_beats_an_exhaustive_ratio_scan(wide_optima, fam):
    r = wide_optima[fam]["ratios"]
    x = lfa.high_cos_grid(3, 16)
    mu_r = _mu_sampled(r[None, :], x)[0]
    # coarse scan of a wide box of ratios (face weight 0..0.6, edge weight
    # -0.15..0.25, corner weight -0.1..0.1 of the centre weight; spacing
    # 0.005 in 2 free ratios, 0.01 in 3)
    if fam == "19pt":
        axes = [np.linspace(0.0, 0.6, 121), np.linspace(-0.15, 0.25, 81)]
        step = 0.005
    else:
        axes = [np.linspace(0.0, 0.6, 61), np.linspace(-0.15, 0.25, 41),
                np.linspace(-0.1, 0.1, 21)]
        step = 0.01
    G = _grid(axes)
    mus = _mu_sampled(G, x)
    assert mus.min() >= mu_r - 1e-12
    # the scan's best stencil lies next to the searched one, in the interior
    # of the box (so the box holds the basin)
    g = G[np.argmin(mus)]
    assert np.max(np.abs(g - r)) <= 3 * step
    assert all(a[0] < v < a[-1] for a, v in zip(axes, g))
    # fine scan around the optimum, spacing 5e-4
    fine = _grid([np.linspace(v - 0.01, v + 0.01, 41) for v in r])
    assert _mu_sampled(fine, x).min() >= mu_r - 1e-12


def _mu_continuous(ratios):
    """mu_opt with the extremes of the symbol product over the continuous
    high frequencies: candidates from a sample, each polished by bounded
    local optimisation on the boxes {x_k <= 0} whose union is T^H."""
    c = np.concatenate([[1.0], ratios])
    x = lfa.high_cos_grid(3, 40)
    p = search.symbol_product(3, c, x)
    ext = []
    for sgn in (1.0, -1.0):
        best = sgn * (p.max() if sgn > 0 else p.min())
        for i in np.argsort(-sgn * p)[:12]:
            for k in range(3):
                if x[i][k] > 0:
                    continue
                bnds = [(-1.0, 1.0)] * 3
                bnds[k] = (-1.0, 0.0)
                res = minimize(lambda v: -sgn * search.symbol_product(3, c, v[None, :])[0],
                               x[i], method="L-BFGS-B", bounds=bnds,
                               options=dict(ftol=1e-15, gtol=1e-13))
                best = max(best, -res.fun)
        ext.append(sgn * best)
    l1, l0 = ext
    return (l1 - l0) / (l1 + l0)


@pytest.mark.parametrize("fam", ["19pt", "27pt"])
def test_wider_3d_optimum_on_the_continuous_symbol(wide_optima, fam):
    r = wide_optima[fam]
    mu = _mu_continuous(r["ratios"])
    # the sampled value is a lower bound of the continuous one and close to it
    assert r["mu"] <= mu + 1e-12
    assert mu <= r["mu"] * (1 + 1e-4)
    # a local minimum of the continuous smoothing factor: every move of the
    # ratios by 0.2% (each sign pattern) raises it
    k = len(r["ratios"])
    for dv in itertools.product((-1, 0, 1), repeat=k):
        if any(dv):
            moved = r["ratios"] * (1.0 + 2e-3 * np.array(dv))
            assert _mu_continuous(moved) > mu
    # the optimal smoothing factors of the two families to four digits
    assert mu == pytest.approx({"19pt": 0.2266, "27pt": 0.1970}[fam], abs=1e-4)
