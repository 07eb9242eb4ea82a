"""Pins of the oracle's stencil and transfer operators against closed forms:
discrete sine eigenpairs of A_h and of the SPAI smoother, exactness on
per-coordinate quadratics, the action of full weighting and linear
interpolation on sine modes, transposes by dot products, and the direct
solver against LAPACK."""
import numpy as np
import pytest

import oracle as O
from oracle import dense
from paper_2206_05543_amd.workloads import grid_coords

C9 = np.array([0.28891272760249742, 0.065661983546022137, 0.019698595063806643])
C7 = np.array([16 / 73, 2 / 73])


def sine(d, N, ks):
    """prod_a sin(k_a pi x_a) on the interior nodes, numpy order (z, y, x)."""
    x = grid_coords(N)
    out = np.sin(ks[0] * np.pi * x)
    for a in range(1, d):
        out = np.multiply.outer(np.sin(ks[a] * np.pi * x), out)
    return out


def lam_A(N, ks):
    # eigenvalue of A_h on the sine mode: 4/h^2 sum_a sin^2(k_a pi h / 2)
    return 4.0 * N * N * sum(np.sin(k * np.pi / (2 * N)) ** 2 for k in ks)


def sym_M_h2(d, c, N, ks):
    # (M phi)/phi = h^2 [c0 + 2 c1 sum cos th + 4 c2 cos th1 cos th2] in 2D;
    # in 3D the edge term 4 c2 sum_{a<b} cos th_a cos th_b and the corner
    # term 8 c3 prod cos th_a (each neighbour pair of offsets +-1 along an
    # axis contributes 2 cos th, and the neighbour sets are products)
    th = [k * np.pi / N for k in ks]
    cs = [np.cos(t) for t in th]
    s = c[0] + 2 * c[1] * sum(cs)
    if d == 2:
        s += 4 * c[2] * cs[0] * cs[1]
    else:
        if len(c) > 2:
            s += 4 * c[2] * (cs[0] * cs[1] + cs[0] * cs[2] + cs[1] * cs[2])
        if len(c) > 3:
            s += 8 * c[3] * cs[0] * cs[1] * cs[2]
    return s / (N * N)


MODES = {2: [(1, 1), (3, 7), (15, 2), (8, 8), (16, 31)],
         3: [(1, 1, 1), (2, 5, 7), (8, 1, 15), (4, 4, 4)]}


@pytest.mark.parametrize("d,N", [(2, 16), (2, 32), (3, 8), (3, 16)])
def test_A_sine_eigenpairs(d, N):
    for ks in MODES[d]:
        if max(ks) >= N:
            continue
        phi = sine(d, N, ks)
        Aphi = O.apply_A(d, N, phi)
        lam = lam_A(N, ks)
        assert np.max(np.abs(Aphi - lam * phi)) <= 1e-12 * lam


@pytest.mark.parametrize("d,N", [(2, 8), (2, 64), (3, 8), (3, 32)])
def test_A_exact_on_quadratics(d, N):
    x = grid_coords(N)
    q = x * (1 - x)
    if d == 2:
        u = np.multiply.outer(q, q)
        f = 2 * (np.multiply.outer(q, np.ones_like(q)) + np.multiply.outer(np.ones_like(q), q))
    else:
        one = np.ones_like(q)
        u = np.multiply.outer(q, np.multiply.outer(q, q))
        f = 2 * (np.multiply.outer(one, np.multiply.outer(q, q))
                 + np.multiply.outer(q, np.multiply.outer(one, q))
                 + np.multiply.outer(q, np.multiply.outer(q, one)))
    assert np.max(np.abs(O.apply_A(d, N, u) - f)) <= 1e-11


C19 = np.array([0.2034, 0.0383, 0.0076])        # 19-point: centre, faces, edges
C27 = np.array([0.1966, 0.0397, 0.0115, 0.0037])  # 27-point: + corners


@pytest.mark.parametrize("d,N,c", [(2, 16, C9), (2, 32, np.array([0.3, -0.1, 0.07])),
                                   (3, 8, C7), (3, 16, np.array([0.2, 0.05])),
                                   (3, 8, C19), (3, 16, C27),
                                   (3, 8, np.array([0.1, -0.02, 0.03, -0.05]))])
def test_smoother_sine_eigenpairs(d, N, c):
    for ks in MODES[d]:
        if max(ks) >= N:
            continue
        phi = sine(d, N, ks)
        m = sym_M_h2(d, c, N, ks)
        assert np.max(np.abs(O.apply_W(d, N, c, phi) - m * phi)) <= 1e-15
        # smoothing with b = 0: S phi = (1 - A~ M~) phi
        s = 1.0 - lam_A(N, ks) * m
        assert np.max(np.abs(O.smooth(d, N, c, phi, np.zeros_like(phi)) - s * phi)) <= 1e-12


def test_smoother_high_modes_reach_mu_opt():
    # The sine modes with max(k, l) >= N/2 are the high frequencies; the
    # largest |S| over them tends to mu_opt (Theorem 3.1), from below.
    N = 256
    k = np.arange(1, N)
    th = k * np.pi / N
    cx = np.cos(th)
    a = 2 * (2 - cx[:, None] - cx[None, :])
    m = C9[0] + 2 * C9[1] * (cx[:, None] + cx[None, :]) + 4 * C9[2] * cx[:, None] * cx[None, :]
    s = np.abs(1 - a * m)
    high = (k[:, None] >= N // 2) | (k[None, :] >= N // 2)
    mu = (9 + 8 * np.sqrt(10)) / 215
    assert mu - 2e-3 < s[high].max() <= mu + 1e-12
    # and these are exactly the oracle smoother's eigenvalues
    for ks in [(N // 2, 1), (N - 1, N // 2), (3, N - 2)]:
        phi = sine(2, N, ks)
        out = O.smooth(2, N, C9, phi, np.zeros_like(phi))
        assert np.allclose(out, (1 - a[ks[1] - 1, ks[0] - 1] * m[ks[1] - 1, ks[0] - 1]) * phi,
                           atol=1e-12)


def _r1(N, k):
    # full weighting of the fine mode sin(k pi x): (1 + cos th)/2 times the
    # coarse mode for k < N/2, -(1 - cos th')/2 times coarse mode N - k for
    # k > N/2, and 0 for k = N/2
    if k == N // 2:
        return 0.0, 1
    if k < N // 2:
        return (1 + np.cos(k * np.pi / N)) / 2, k
    kk = N - k
    return -(1 - np.cos(kk * np.pi / N)) / 2, kk


@pytest.mark.parametrize("d,N", [(2, 16), (2, 32), (3, 8), (3, 16)])
def test_restriction_on_sine_modes(d, N):
    for ks in MODES[d] + [tuple([N // 2] + [1] * (d - 1)), tuple([N - 3] * d)]:
        if max(ks) >= N:
            continue
        phi = sine(d, N, ks)
        got = O.restrict(d, N, phi)
        fac, kc = 1.0, []
        for k in ks:
            f, kk = _r1(N, k)
            fac *= f
            kc.append(kk)
        want = fac * sine(d, N // 2, kc)
        assert np.max(np.abs(got - want)) <= 1e-14


@pytest.mark.parametrize("d,N", [(2, 16), (2, 32), (3, 8), (3, 16)])
def test_prolongation_on_sine_modes(d, N):
    # P psi_k = prod over directions of
    #   [(1 + cos th)/2 phi_k - (1 - cos th)/2 phi_{N-k}],  th = k pi / N
    for kc in [(1, 1, 1), (3, 2, 5), (N // 2 - 1, 1, N // 2 - 1)]:
        kc = kc[:d]
        if max(kc) >= N // 2:
            continue
        got = O.prolong_add(d, N, sine(d, N // 2, kc), np.zeros((N - 1,) * d))
        x = grid_coords(N)
        want = None
        for a, k in enumerate(kc):
            th = k * np.pi / N
            f = ((1 + np.cos(th)) / 2 * np.sin(k * np.pi * x)
                 - (1 - np.cos(th)) / 2 * np.sin((N - k) * np.pi * x))
            want = f if want is None else np.multiply.outer(f, want)
        assert np.max(np.abs(got - want)) <= 1e-14


@pytest.mark.parametrize("d,N", [(2, 16), (3, 8)])
def test_transposes_by_dot_products(d, N):
    rng = np.random.default_rng(7)
    f = rng.standard_normal((N - 1,) * d)
    g = rng.standard_normal((N // 2 - 1,) * d)
    Rf = O.restrict(d, N, f)
    assert abs(np.vdot(Rf, g) - np.vdot(f, O.restrict_T(d, N, g))) < 1e-12
    Pg = O.prolong_add(d, N, g, np.zeros_like(f))
    assert abs(np.vdot(Pg, f) - np.vdot(g, O.prolong_T(d, N, f))) < 1e-12
    # linear interpolation is 2^d times the transpose of full weighting
    assert np.allclose(Pg, 2 ** d * O.restrict_T(d, N, g), atol=1e-14)
    # A and M are symmetric under zero extension
    c = C9 if d == 2 else C7
    assert abs(np.vdot(O.apply_A(d, N, f), f * 0 + Pg) - np.vdot(f, O.apply_A(d, N, Pg))) < 1e-9
    assert abs(np.vdot(O.apply_W(d, N, c, f), Pg) - np.vdot(f, O.apply_W(d, N, c, Pg))) < 1e-13


@pytest.mark.parametrize("d,N", [(2, 4), (3, 4), (2, 16), (3, 8)])
def test_direct_solve_against_lapack(d, N):
    rng = np.random.default_rng(3)
    b = rng.standard_normal((N - 1,) * d)
    x = O.direct_solve(d, N, b)
    xr = np.linalg.solve(dense.A(d, N), b.ravel()).reshape(b.shape)
    assert np.max(np.abs(x - xr)) <= 1e-12 * np.max(np.abs(xr))
    assert np.max(np.abs(O.apply_A(d, N, x) - b)) <= 1e-10 * np.max(np.abs(b))


@pytest.mark.parametrize("d,N", [(2, 16), (3, 8)])
def test_dense_matrices_match_loop_operators(d, N):
    # the Kronecker-product matrices (dense.py) and the loop operators
    # (mg_oracle.c) are independent codings of the same definitions
    rng = np.random.default_rng(11)
    v = rng.standard_normal((N - 1,) * d)
    c = C9 if d == 2 else C7
    assert np.allclose(dense.A(d, N) @ v.ravel(), O.apply_A(d, N, v).ravel(), atol=1e-10)
    assert np.allclose(dense.W(d, N, c) @ v.ravel(), O.apply_W(d, N, c, v).ravel(), atol=1e-15)
    assert np.allclose(dense.R(d, N) @ v.ravel(), O.restrict(d, N, v).ravel(), atol=1e-14)
    g = rng.standard_normal((N // 2 - 1,) * d)
    assert np.allclose(dense.P(d, N) @ g.ravel(),
                       O.prolong_add(d, N, g, np.zeros_like(v)).ravel(), atol=1e-14)


@pytest.mark.parametrize("which,count", [(2, 12), (3, 8)])
def test_3d_edge_and_corner_sums(which, count):
    # the loop operators against the Kronecker sums of shift matrices, and
    # the neighbour count on a node far from the boundary
    N = 8
    rng = np.random.default_rng(which)
    v = rng.standard_normal((N - 1,) * 3)
    got = O.apply_K(3, N, which, v)
    want = (dense.K(3, N, which) @ v.ravel()).reshape(v.shape)
    assert np.max(np.abs(got - want)) <= 1e-14
    one = np.zeros((N - 1,) * 3)
    one[3, 3, 3] = 1.0
    assert O.apply_K(3, N, which, one).sum() == count


def test_wide_3d_smoother_high_modes_reach_searched_mu():
    # the sine modes with some index >= N/2 are the high frequencies; the
    # largest |S| over them tends to the searched optimum mu of the 27-point
    # family from below, and the oracle's smoother has exactly these
    # eigenvalues
    from oracle import search
    r = search.search(3, "27pt", m=24, refine_m=60)
    c = np.asarray(r["coeffs"])
    N = 64
    k = np.arange(1, N)
    x = np.cos(k * np.pi / N)
    X = np.stack(np.meshgrid(x, x, x, indexing="ij"), -1).reshape(-1, 3)
    K = np.stack(np.meshgrid(k, k, k, indexing="ij"), -1).reshape(-1, 3)
    s = np.abs(1.0 - search.symbol_product(3, c, X))
    high = np.any(K >= N // 2, axis=1)
    assert r["mu"] - 5e-3 < s[high].max() <= r["mu"] * (1 + 1e-4)
    for ks in [(N // 2, 1, 3), (N - 1, 5, N // 2), (2, N - 2, 40)]:
        phi = sine(3, N, ks)
        out = O.smooth(3, N, c, phi, np.zeros_like(phi))
        lam = 1.0 - lam_A(N, ks) * sym_M_h2(3, c, N, ks)
        assert np.max(np.abs(out - lam * phi)) <= 1e-12
