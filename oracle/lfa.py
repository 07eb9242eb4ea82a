"""Local Fourier analysis of the SPAI smoothers (Sections 2-4 of He, Liu and
Wang, arXiv 2206.05543).

TEST INFRASTRUCTURE ONLY (see the package docstring).

All symbols are taken with h = 1: the product of the symbol of A_h (which
carries 1/h^2) and of M (which carries h^2) does not depend on h.  The
smoother coefficients c follow the oracle convention: M = h^2 sum_j c_j K_j,
K_0 = I, K_1 = face-neighbour sum, K_2 = diagonal-neighbour sum (2D).
"""
import itertools

import numpy as np


def symbol_A(d, th):
    """h^2 times the symbol of A_h: 2 (d - sum_k cos th_k) (Section 3.1,
    eq. (symbol-Lh2D); Section 3.2, eq. (symbol-Lh3D)).  th has shape
    (..., d)."""
    return 2.0 * (d - np.cos(th).sum(axis=-1))


def symbol_M(d, c, th):
    """Symbol of M divided by h^2: c0 + 2 c1 sum cos th_k + 4 c2 cos th_1 cos
    th_2 (2D, the Upsilon family of Section 3.1); c0 + 2 c1 sum cos th_k (3D,
    the T family of Section 3.2), plus 4 c2 sum_{k<l} cos th_k cos th_l for
    the 12 edge neighbours and 8 c3 prod cos th_k for the 8 corners when c
    has 3 or 4 entries (the 19- and 27-point extensions)."""
    cs = np.cos(th)
    s = c[0] + 2.0 * c[1] * cs.sum(axis=-1)
    if d == 2:
        s = s + 4.0 * c[2] * cs[..., 0] * cs[..., 1]
    else:
        if len(c) > 2:
            s = s + 4.0 * c[2] * (cs[..., 0] * cs[..., 1] + cs[..., 0] * cs[..., 2] +
                                  cs[..., 1] * cs[..., 2])
        if len(c) > 3:
            s = s + 8.0 * c[3] * cs[..., 0] * cs[..., 1] * cs[..., 2]
    return s


def high_cos_grid(d, m):
    """Points x = (cos th_1, ..) with th in the high frequencies T^H, i.e. the
    set [-1,1]^d minus (0,1]^d (Section 2; Appendix A), sampled with m+1
    points per direction on [-1, 1] (m even, so 0 is included)."""
    x = np.linspace(-1.0, 1.0, m + 1)
    g = np.stack(np.meshgrid(*([x] * d), indexing="ij"), axis=-1).reshape(-1, d)
    low = np.all(g > 0.0, axis=-1)
    return g[~low]


def product_on_high(d, c, m=2000):
    """Samples of A~(th) M~(th) over T^H, as a function of the cosines."""
    x = high_cos_grid(d, m)
    a = 2.0 * (d - x.sum(axis=-1))
    mm = c[0] + 2.0 * c[1] * x.sum(axis=-1)
    if d == 2:
        mm = mm + 4.0 * c[2] * x[:, 0] * x[:, 1]
    else:
        if len(c) > 2:
            mm = mm + 4.0 * c[2] * (x[:, 0] * x[:, 1] + x[:, 0] * x[:, 2] + x[:, 1] * x[:, 2])
        if len(c) > 3:
            mm = mm + 8.0 * c[3] * x[:, 0] * x[:, 1] * x[:, 2]
    return a * mm


def smoothing_factor(d, c, omega=1.0, m=2000):
    """mu_loc = max over T^H of |1 - omega A~ M~| (Section 2)."""
    return float(np.max(np.abs(1.0 - omega * product_on_high(d, c, m))))


def optimal_mu_omega(d, c, m=2000):
    """(mu_opt, omega_opt, lambda0, lambda1) from the extreme values of A~ M~
    on T^H: mu = (l1 - l0)/(l1 + l0), omega = 2/(l0 + l1) (Section 2, eqs.
    (mu_opt) and (omega_opt))."""
    p = product_on_high(d, c, m)
    l0, l1 = float(p.min()), float(p.max())
    return (l1 - l0) / (l1 + l0), 2.0 / (l0 + l1), l0, l1


def _harmonics(d):
    return np.array(list(itertools.product((0, 1), repeat=d)), dtype=float)


def _tg_matrices(d, c, nu, th, coarse):
    """Two-grid symbols K^ S^nu on the 2^d harmonics th + pi*alpha of each
    low frequency th (shape (M, d)): full weighting and linear interpolation
    both have the symbol prod (1 + cos th_k)/2; the coarse operator is
    rediscretised with H = 2h or formed by Galerkin projection R A P."""
    alph = _harmonics(d)
    tha = th[:, None, :] + np.pi * alph[None, :, :]          # (M, 2^d, d)
    a = symbol_A(d, tha)
    s = 1.0 - a * symbol_M(d, c, tha)
    t = np.prod((1.0 + np.cos(tha)) / 2.0, axis=-1)          # (M, 2^d)
    if coarse == "rediscretized":
        aH = 0.5 * (d - np.cos(2.0 * th).sum(axis=-1))      # H = 2, h = 1
    elif coarse == "galerkin":
        aH = np.sum(t * a * t, axis=-1)
    else:
        raise ValueError(coarse)
    nh = len(alph)
    K = np.eye(nh)[None] - t[:, :, None] * (t * a)[:, None, :] / aH[:, None, None]
    return K * (s ** nu)[:, None, :]


def _max_spectral_radius(mats):
    return float(np.max(np.abs(np.linalg.eigvals(mats))))


def two_grid_factor(d, c, nu, n, coarse="rediscretized"):
    """rho_h(nu): max over sampled low frequencies th = 2 pi k / n in
    T^L = [-pi/2, pi/2)^d, th != 0, of the spectral radius of the two-grid
    symbol (Section 4, Table 1).  Any split nu = nu1 + nu2 has the same
    spectral radius."""
    ks = np.arange(-n // 4, n // 4)
    kk = np.stack(np.meshgrid(*([ks] * d), indexing="ij"), -1).reshape(-1, d)
    kk = kk[np.any(kk != 0, axis=1)]
    th = 2.0 * np.pi * kk.astype(float) / n
    return _max_spectral_radius(_tg_matrices(d, c, nu, th, coarse))


def dirichlet_two_grid_factor(d, c, nu, N):
    """Spectral radius of the two-grid operator on the Dirichlet grid with N
    intervals.  The sine modes sin(k pi x) of the grid couple in groups of
    2^d frequencies th = k pi/N and th + pi (k = 1..N/2-1 per direction), on
    which the two-grid operator acts exactly as the LFA symbol; a mode with
    some k = N/2 is annihilated by full weighting, so only the smoother acts
    on it."""
    ks = np.arange(1, N // 2)
    kk = np.stack(np.meshgrid(*([ks] * d), indexing="ij"), -1).reshape(-1, d)
    th = np.pi * kk.astype(float) / N
    rho = _max_spectral_radius(_tg_matrices(d, c, nu, th, "rediscretized"))
    full = np.arange(1, N)
    kk = np.stack(np.meshgrid(*([full] * d), indexing="ij"), -1).reshape(-1, d)
    kk = kk[np.any(kk == N // 2, axis=1)]
    th = np.pi * kk.astype(float) / N
    s = 1.0 - symbol_A(d, th) * symbol_M(d, c, th)
    return max(rho, float(np.max(np.abs(s) ** nu)))
