"""Explicit matrices of every operator of the multigrid cycle on tiny grids
(He, Liu and Wang, arXiv 2206.05543, Sections 1, 3 and 4).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Built from Kronecker products of 1D matrices, independently of the loop code
in mg_oracle.c, so the two can check each other.  Ordering: x fastest, i.e.
the flat index is i + n j (+ n^2 k), so the x-direction factor is the last
Kronecker factor.  Every function accepts complex coefficients, which the
complex-step derivative uses (all products are bilinear, never conjugated).
"""
import numpy as np


def _kron_all(mats):
    out = np.array([[1.0]])
    for m in mats:
        out = np.kron(out, m)
    return out


def _tri(n, diag, off):
    return diag * np.eye(n) + off * (np.eye(n, k=1) + np.eye(n, k=-1))


def A(d, N):
    """A_h = sum over directions of (1/h^2) tridiag(-1, 2, -1) (eq. (A_h))."""
    n = N - 1
    T = _tri(n, 2.0, -1.0) * N * N
    I = np.eye(n)
    out = np.zeros((n ** d, n ** d))
    for ax in range(d):
        out += _kron_all([T if a == ax else I for a in range(d)])
    return out


def K(d, N, which):
    """K_0 = I, K_1 = face-neighbour sum, K_2 = diagonal-neighbour sum (2D)
    or edge-neighbour sum (3D), K_3 = corner-neighbour sum (3D), zero
    extension (the stencil families of Section 3 and the 19-/27-point
    extensions of the 3D family): the sum over the products with exactly
    `which` shift factors S (the rest identities)."""
    n = N - 1
    I, S = np.eye(n), _tri(n, 0.0, 1.0)
    if which == 0:
        return np.eye(n ** d)
    assert which <= d
    out = np.zeros((n ** d, n ** d))
    for axes in _subsets(d, which):
        out += _kron_all([S if a in axes else I for a in range(d)])
    return out


def _subsets(d, k):
    import itertools
    return [set(s) for s in itertools.combinations(range(d), k)]


def W(d, N, c):
    """M = h^2 sum_j c_j K_j."""
    h2 = 1.0 / (N * N)
    return h2 * sum(c[j] * K(d, N, j) for j in range(len(c)))


def R(d, N):
    """Full weighting to N/2 intervals: 1D rows [1/4, 1/2, 1/4] centred on
    fine node 2J, tensor product in d directions (Section 4)."""
    n, nc = N - 1, N // 2 - 1
    R1 = np.zeros((nc, n))
    for J in range(nc):
        R1[J, 2 * J] = 0.25
        R1[J, 2 * J + 1] = 0.5
        R1[J, 2 * J + 2] = 0.25
    return _kron_all([R1] * d)


def P(d, N):
    """Linear interpolation from N/2 intervals (tensor product), which is
    2^d R^T for full weighting."""
    n, nc = N - 1, N // 2 - 1
    P1 = np.zeros((n, nc))
    for J in range(nc):
        P1[2 * J, J] = 0.5
        P1[2 * J + 1, J] = 1.0
        P1[2 * J + 2, J] = 0.5
    return _kron_all([P1] * d)


def smoother(d, N, c):
    """S = I - M A (eq. (smoother))."""
    return np.eye((N - 1) ** d) - W(d, N, c) @ A(d, N)


def vcycle_maps(d, N, c, nu1=1, nu2=1, gamma=1):
    """(E, B) with cycle(u, b) = E u + B b: E = S^nu2 C^gamma-recursion S^nu1
    with coarse-grid correction through the recursive approximate inverse of
    the coarse level; B = (I - E) A^{-1}; the N = 4 level is an exact solve."""
    Ah = A(d, N)
    if N <= 4:
        n = Ah.shape[0]
        return np.zeros((n, n)), np.linalg.inv(Ah)
    _, Bc = vcycle_maps(d, N // 2, c, nu1, nu2, gamma)
    Ec = np.eye(Bc.shape[0]) - Bc @ A(d, N // 2)
    # gamma coarse cycles from zero: e = sum_{g<gamma} Ec^g Bc bc
    Bg = np.zeros_like(Bc, dtype=np.result_type(Bc, Ec))
    Ep = np.eye(Bc.shape[0])
    for _ in range(gamma):
        Bg = Bg + Ep @ Bc
        Ep = Ep @ Ec
    S = smoother(d, N, c)
    Cg = np.eye(Ah.shape[0]) - P(d, N) @ Bg @ R(d, N) @ Ah
    E = np.linalg.matrix_power(S, nu2) @ Cg @ np.linalg.matrix_power(S, nu1)
    B = (np.eye(Ah.shape[0]) - E) @ np.linalg.inv(Ah)
    return E, B


def two_grid(d, N, c, nu1, nu2):
    """S^nu2 (I - P A_H^{-1} R A_h) S^nu1 with the rediscretised A_H."""
    Ah = A(d, N)
    S = smoother(d, N, c)
    C = np.eye(Ah.shape[0]) - P(d, N) @ np.linalg.inv(A(d, N // 2)) @ R(d, N) @ Ah
    return np.linalg.matrix_power(S, nu2) @ C @ np.linalg.matrix_power(S, nu1)


def loss_kcycles(d, N, c, e0, K, b=None):
    """sum_s ||u_K||^2, u_K = E^K e0_s (+ the b terms), with bilinear products
    so that complex coefficients give the complex-step derivative."""
    E, B = vcycle_maps(d, N, c)
    n = (N - 1) ** d
    L = 0.0
    for e in np.asarray(e0).reshape(-1, n):
        u = e.astype(np.result_type(E, e))
        for _ in range(K):
            u = E @ u + (B @ b.ravel() if b is not None else 0.0)
        L = L + np.sum(u * u)
    return L


def complex_step_grad(d, N, c, e0, K, h=1e-30):
    """dL/dc_j = Im L(c + i h e_j) / h, exact to rounding for the polynomial
    dependence of the cycle on c."""
    c = np.asarray(c, dtype=float)
    g = np.zeros(c.size)
    for j in range(c.size):
        cc = c.astype(complex)
        cc[j] += 1j * h
        g[j] = np.imag(loss_kcycles(d, N, cc, e0, K)) / h
    return g
