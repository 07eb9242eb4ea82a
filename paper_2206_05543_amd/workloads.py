"""Seeded synthetic inputs for the Poisson problems the solver is run on.

This module only draws random numbers and samples source terms; it holds none
of the multigrid arithmetic, so both the GPU path and the CPU oracle read
their inputs from here.

The paper tests analytic problems only (Section 4, Examples 1-3); these
generators stand in for them with seeded sine-mode sums of the same kind:
f = sum_m c_m sin(k_m pi x) sin(l_m pi y) [sin(p_m pi z)], sampled at the
interior nodes of the grid with h = 1/N, g = 0 (Section 1, eq. (Poisson)).

Draw order with numpy.random.default_rng(seed) (PCG64): all k, then all l,
[then all p], then the mode coefficients (standard normal, divided by
k^2 + l^2 [+ p^2]), then the initial guess (uniform [-1, 1]), then the noise.
"""
import numpy as np


def grid_coords(N):
    """Interior node coordinates i/N, i = 1..N-1."""
    return np.arange(1, N, dtype=np.float64) / N


def sine_modes(rng, d, n_modes, kmax):
    ks = [rng.integers(1, kmax + 1, size=n_modes) for _ in range(d)]
    w = rng.standard_normal(n_modes)
    w = w / sum(k.astype(np.float64) ** 2 for k in ks)
    return np.stack(ks, axis=1), w


def sine_sum(d, N, modes, weights):
    """sum_m w_m prod_a sin(k_{m,a} pi x_a) on the interior nodes, shape
    (N-1,)*d in numpy order (z, y, x), i.e. x is the fastest index."""
    x = grid_coords(N)
    out = np.zeros((N - 1,) * d)
    for kk, w in zip(modes, weights):
        sx = np.sin(kk[0] * np.pi * x)
        sy = np.sin(kk[1] * np.pi * x)
        plane = np.multiply.outer(sy, sx)
        if d == 2:
            out += w * plane
        else:
            sz = w * np.sin(kk[2] * np.pi * x)
            for z in range(N - 1):
                out[z] += sz[z] * plane
    return out


def poisson_problem(d, N, seed, n_modes, kmax, noise=0.0, batch=1):
    """Right-hand side b (sine-mode sum plus optional uniform noise) and
    initial guess u0 ~ U[-1, 1]; returns dict(b, u0, modes, weights)."""
    rng = np.random.default_rng(seed)
    modes, weights = sine_modes(rng, d, n_modes, kmax)
    b = sine_sum(d, N, modes, weights)
    u0 = rng.uniform(-1.0, 1.0, size=(batch,) + (N - 1,) * d)
    if noise:
        b = b + rng.uniform(-noise, noise, size=b.shape)
    if batch == 1:
        u0 = u0[0]
    return {"b": b, "u0": u0, "modes": modes, "weights": weights}


def random_errors(d, N, seed, batch):
    """b = 0 and a batch of initial errors e0 ~ U[-1, 1] (the k-cycle
    error-reduction workloads)."""
    rng = np.random.default_rng(seed)
    e0 = rng.uniform(-1.0, 1.0, size=(batch,) + (N - 1,) * d)
    return {"b": np.zeros((N - 1,) * d), "e0": e0}


def example_problem(example, N, seed=0):
    """The analytic problems of Section 4 (Examples 1-3), g = 0: b = f at the
    interior nodes, the exact solution u there, and the initial guess drawn
    uniformly from (0, 1) as in the paper's experiments.

    Example 1 (2D): u = (x^2 - x^4)(y^4 - y^2).
    Example 2 (2D): u = x ln(x) y ln(y); f is singular as x or y -> 0.
    Example 3 (3D): u = sin(pi x) sin(pi y) sin(pi z), f = 3 pi^2 u.
    Arrays are in numpy order (y, x) / (z, y, x).
    """
    x = grid_coords(N)
    if example == 1:
        X = x[None, :]
        Y = x[:, None]
        u = (X ** 2 - X ** 4) * (Y ** 4 - Y ** 2)
        f = (2.0 * (1.0 - 6.0 * X ** 2) * (Y ** 2 - Y ** 4)
             + 2.0 * (1.0 - 6.0 * Y ** 2) * (X ** 2 - X ** 4))
        d = 2
    elif example == 2:
        X = x[None, :]
        Y = x[:, None]
        u = X * np.log(X) * Y * np.log(Y)
        f = -X * np.log(X) / Y - Y * np.log(Y) / X
        d = 2
    elif example == 3:
        s = np.sin(np.pi * x)
        u = s[:, None, None] * s[None, :, None] * s[None, None, :]
        f = 3.0 * np.pi ** 2 * u
        d = 3
    else:
        raise ValueError("example must be 1, 2 or 3")
    rng = np.random.default_rng(seed)
    u0 = rng.uniform(0.0, 1.0, size=(N - 1,) * d)
    return {"d": d, "b": np.ascontiguousarray(f), "u": np.ascontiguousarray(u), "u0": u0}


# The five workloads: (dimension, N, seed, modes, max index, noise, batch).
WORKLOADS = {
    "poisson2d_n64": dict(d=2, N=64, seed=0, n_modes=8, kmax=16),
    "poisson2d_n4096": dict(d=2, N=4096, seed=1, n_modes=16, kmax=64),
    "poisson3d_n256": dict(d=3, N=256, seed=2, n_modes=16, kmax=64),
    "poisson3d_n512_noisy": dict(d=3, N=512, seed=3, n_modes=16, kmax=64,
                                 noise=1e-3),
}
ERROR_WORKLOADS = {
    "errors2d_n1024_b16": dict(d=2, N=1024, seed=4, batch=16),
    "errors3d_n256_b4": dict(d=3, N=256, seed=5, batch=4),
}


def workload(name, **override):
    if name in WORKLOADS:
        kw = dict(WORKLOADS[name])
        kw.update(override)
        return poisson_problem(**kw)
    kw = dict(ERROR_WORKLOADS[name])
    kw.update(override)
    return random_errors(**kw)
