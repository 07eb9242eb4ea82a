"""Pins of the oracle's multigrid cycle and solver: the two-grid operator
assembled from the loop code against the Dirichlet LFA, the V-cycle operator
against the Kronecker-matrix recursion, symmetry of the cycle's approximate
inverse, direct solves on tiny grids and the closed-form discrete solution of
sine-mode right-hand sides."""
import numpy as np
import pytest

import oracle as O
from oracle import dense, lfa
from paper_2206_05543_amd.workloads import poisson_problem, sine_sum, workload

C9 = np.array([0.28891272760249742, 0.065661983546022137, 0.019698595063806643])
C7 = np.array([16 / 73, 2 / 73])
C27 = np.array([0.1966, 0.0397, 0.0115, 0.0037])  # 27-point 3D stencil
CJ2 = np.array([0.2, 0.0, 0.0])
CM5 = np.array([12 / 41, 2 / 41, 0.0])
CJ3 = np.array([1 / 7, 0.0])


def _loop_two_grid(d, N, c, nu1, nu2):
    """Columns of the two-grid error operator from the loop operators."""
    n = (N - 1) ** d
    cols = []
    for i in range(n):
        u = np.zeros(n)
        u[i] = 1.0
        u = u.reshape((N - 1,) * d)
        z = np.zeros_like(u)
        for _ in range(nu1):
            u = O.smooth(d, N, c, u, z)
        ec = O.direct_solve(d, N // 2, O.restrict(d, N, O.residual(d, N, u, z)))
        u = O.prolong_add(d, N, ec, u)
        for _ in range(nu2):
            u = O.smooth(d, N, c, u, z)
        cols.append(u.ravel())
    return np.array(cols).T


@pytest.mark.parametrize("d,N,c,nu1,nu2", [(2, 16, C9, 1, 0), (2, 16, C9, 1, 1),
                                           (2, 32, C9, 1, 1), (2, 16, CM5, 1, 1),
                                           (3, 8, C7, 1, 1), (3, 8, CJ3, 1, 1),
                                           (3, 8, C27, 1, 1)])
def test_two_grid_spectral_radius_equals_dirichlet_lfa(d, N, c, nu1, nu2):
    E = _loop_two_grid(d, N, c, nu1, nu2)
    rho = np.max(np.abs(np.linalg.eigvals(E)))
    assert abs(rho - lfa.dirichlet_two_grid_factor(d, c, nu1 + nu2, N)) < 1e-11


def _loop_cycle_maps(d, N, c, gamma=1, nu1=1, nu2=1):
    n = (N - 1) ** d
    E = np.zeros((n, n))
    B = np.zeros((n, n))
    z = np.zeros((N - 1,) * d)
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        E[:, i] = O.cycle(d, N, c, e.reshape(z.shape), z, nu1, nu2, gamma).ravel()
        B[:, i] = O.cycle(d, N, c, z, e.reshape(z.shape), nu1, nu2, gamma).ravel()
    return E, B


@pytest.mark.parametrize("d,N,c,gamma,nu1,nu2", [
    (2, 16, C9, 1, 1, 1), (2, 32, C9, 1, 1, 1), (2, 16, CJ2, 2, 1, 1), (3, 8, C7, 1, 1, 1),
    (3, 8, C7, 2, 1, 1), (2, 16, C9, 2, 1, 0), (2, 32, CM5, 2, 1, 0), (3, 8, C7, 2, 1, 0),
    (3, 8, C27, 1, 1, 1), (3, 8, C27[:3], 1, 1, 1)])
def test_cycle_operator_matches_matrix_recursion(d, N, c, gamma, nu1, nu2):
    E, B = _loop_cycle_maps(d, N, c, gamma, nu1, nu2)
    Ed, Bd = dense.vcycle_maps(d, N, c, nu1, nu2, gamma)
    assert np.max(np.abs(E - Ed)) < 1e-12
    assert np.max(np.abs(B - Bd)) < 1e-12 * np.max(np.abs(Bd))
    if nu1 == nu2:
        # the cycle's approximate inverse is symmetric (nu1 = nu2, symmetric M)
        assert np.max(np.abs(B - B.T)) < 1e-12 * np.max(np.abs(B))
    # consistency: E = I - B A
    assert np.max(np.abs(E - (np.eye(len(E)) - B @ dense.A(d, N)))) < 1e-10


def test_w10_two_level_reduces_to_presmoothed_two_grid():
    # with one coarse level below (N = 8: the 3^d grid is solved exactly) the
    # W(1,0) error operator is the two-grid operator with one pre-smoothing
    # step, whatever gamma, since repeating an exact solve changes nothing
    for d, c in [(2, C9), (3, C7)]:
        E, _ = _loop_cycle_maps(d, 8, c, 2, 1, 0)
        assert np.max(np.abs(E - dense.two_grid(d, 8, c, 1, 0))) < 1e-12


def test_vcycle_contraction_rates():
    # spectral radius of the V(1,1) error operator: M9 < M5 < damped Jacobi
    rho = {}
    for name, c in [("M9", C9), ("M5", CM5), ("J", CJ2)]:
        E, _ = _loop_cycle_maps(2, 32, c)
        rho[name] = np.max(np.abs(np.linalg.eigvals(E)))
    assert rho["M9"] < rho["M5"] < rho["J"]
    assert rho["M9"] < 0.14 and rho["J"] > 0.3


@pytest.mark.parametrize("d,N,c", [(2, 16, C9), (2, 8, C9), (3, 8, C7), (3, 16, C7)])
def test_solve_reaches_direct_solution(d, N, c):
    rng = np.random.default_rng(5)
    b = rng.standard_normal((N - 1,) * d)
    u0 = rng.uniform(-1, 1, b.shape)
    u, k, hist = O.solve(d, N, c, u0, b, tol=1e-12, maxc=60)
    assert k > 0 and hist[-1] <= 1e-12 * hist[0]
    x = np.linalg.solve(dense.A(d, N), b.ravel()).reshape(b.shape)
    # ||u - x|| <= ||A^{-1}|| ||r_k||, lambda_min = 4 d N^2 sin^2(pi / 2N)
    lam_min = 4.0 * d * N * N * np.sin(np.pi / (2 * N)) ** 2
    assert np.linalg.norm(u - x) <= 1.001 * hist[-1] / lam_min + 1e-14 * np.linalg.norm(x)


def _closed_form(d, N, modes, weights):
    # A_h phi = lambda phi for sine modes, so the discrete solution of
    # A_h u = sum w phi is sum (w / lambda) phi
    lam = 4.0 * N * N * sum(np.sin(modes[:, a] * np.pi / (2 * N)) ** 2 for a in range(d))
    return sine_sum(d, N, modes, weights / lam)


@pytest.mark.parametrize("d,N,c", [(2, 64, C9), (3, 32, C7)])
def test_solve_sine_rhs_closed_form(d, N, c):
    p = poisson_problem(d, N, seed=0, n_modes=8, kmax=N // 4)
    u, k, hist = O.solve(d, N, c, p["u0"], p["b"], tol=1e-10, maxc=60)
    assert k > 0
    assert hist[k] <= 1e-10 * hist[0] < hist[k - 1]
    ref = _closed_form(d, N, p["modes"], p["weights"])
    # error <= ||A^-1|| ||r_k|| with ||A^-1|| = 1/lambda_min < 1/(d pi^2 .. )
    bound = hist[k] / (2 * d * 4.0) / np.linalg.norm(ref)
    assert np.linalg.norm(u - ref) / np.linalg.norm(ref) <= max(bound, 1e-13)


def test_config0_cycle_count_and_rate():
    # 2D N=64, eight modes, M9: the random initial guess is mostly high
    # frequency, which the first cycles remove fast; the per-cycle reduction
    # then grows towards the V-cycle's spectral radius (about 0.13) from
    # below, so 8-11 cycles reach 1e-10.
    p = workload("poisson2d_n64")
    u, k, hist = O.solve(2, 64, C9, p["u0"], p["b"], tol=1e-10, maxc=60)
    ratios = hist[1:] / hist[:-1]
    assert 8 <= k <= 11
    assert np.all(ratios < 0.13) and np.all(np.diff(ratios) > 0)


def test_w_cycle_converges_faster_per_cycle():
    p = poisson_problem(2, 32, seed=2, n_modes=4, kmax=8)
    _, kv, _ = O.solve(2, 32, CJ2, p["u0"], p["b"], 1e-8, 80, 1, 1, 1)
    _, kw, _ = O.solve(2, 32, CJ2, p["u0"], p["b"], 1e-8, 80, 1, 1, 2)
    assert 0 < kw <= kv


def test_openmp_build_is_bit_identical():
    # the all-core build splits only loops whose outputs are independent, so
    # its cycle equals the checker build's bit for bit
    from paper_2206_05543_amd import M7, M9
    rng = np.random.default_rng(17)
    for d, N in ((2, 128), (3, 32)):
        u = rng.uniform(-1, 1, (N - 1,) * d)
        b = rng.standard_normal((N - 1,) * d) * N
        c = np.array(M9 if d == 2 else M7)
        assert np.array_equal(O.vcycle(d, N, c, u, b), O.vcycle(d, N, c, u, b, parallel=True))
