"""CPU oracle for the SPAI-smoothed geometric multigrid cycle.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library: ``mg_oracle.c`` holds plain FP64 loops of the method
(He, Liu and Wang, arXiv 2206.05543; Sections 1-4), ``lfa.py`` the local
Fourier analysis of Sections 2-4, ``search.py`` the minimax search for
stencil coefficients of Section 3 and ``dense.py`` explicit matrices of every
operator on tiny grids.

Arrays follow the paper's grid: N intervals per direction, h = 1/N, the
(N-1)^d interior nodes stored x fastest, batch outermost.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mg_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


_OMP_PATH = os.path.join(_HERE, "liboracle_omp.so")
_lib_omp = None
_FLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-fPIC", "-shared"]


def build(force=True):
    """Compile mg_oracle.c with gcc: -O2, no FMA contraction, single thread
    (liboracle.so, the checker), and the same source with -fopenmp
    (liboracle_omp.so, the all-core CPU baseline; bit-identical results)."""
    for path, extra in ((_LIB_PATH, []), (_OMP_PATH, ["-fopenmp"])):
        if force or not os.path.exists(path) or (
                os.path.getmtime(path) < os.path.getmtime(_SRC)):
            subprocess.check_call(["gcc"] + _FLAGS + extra + ["-o", path + ".tmp", _SRC, "-lm"])
            os.replace(path + ".tmp", path)
    return _LIB_PATH


def _bind(L):
    dp = ctypes.POINTER(ctypes.c_double)
    i = ctypes.c_int
    L.or_num_threads.restype = i
    L.or_apply_A.argtypes = [i, i, dp, dp]
    L.or_apply_K.argtypes = [i, i, i, dp, dp]
    L.or_apply_W.argtypes = [i, i, dp, dp, dp]
    L.or_residual.argtypes = [i, i, dp, dp, dp]
    L.or_smooth.argtypes = [i, i, dp, dp, dp, dp]
    L.or_restrict.argtypes = [i, i, dp, dp]
    L.or_prolong_add.argtypes = [i, i, dp, dp]
    L.or_restrict_T_add.argtypes = [i, i, dp, dp]
    L.or_prolong_T_add.argtypes = [i, i, dp, dp]
    L.or_direct_solve.argtypes = [i, i, dp, dp]
    L.or_cycle.argtypes = [i, i, dp, i, i, i, dp, dp]
    L.or_vcycle.argtypes = [i, i, dp, dp, dp]
    L.or_solve.argtypes = [i, i, dp, i, i, i, dp, dp, ctypes.c_double, i, dp]
    L.or_solve.restype = i
    L.or_norm2.argtypes = [ctypes.c_long, dp]
    L.or_norm2.restype = ctypes.c_double
    L.or_vcycle_adjoint.argtypes = [i, i, dp, dp, dp, dp, dp, dp, dp]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or (
                os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build(force=False)
        _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def lib_omp():
    """The OpenMP build (threads from OMP_NUM_THREADS, else all cores)."""
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(_OMP_PATH) or (
                os.path.getmtime(_OMP_PATH) < os.path.getmtime(_SRC)):
            build(force=False)
        _lib_omp = _bind(ctypes.CDLL(_OMP_PATH))
    return _lib_omp


def _p(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def npts(d, N):
    return (N - 1) ** d


def shape(d, N):
    return (N - 1,) * d


def _coeffs(d, c):
    """The C side's coefficient array: 3 entries in 2D (centre, faces,
    diagonals); 4 in 3D (centre, faces, edges, corners), where 2 or 3 given
    entries (the 7- and 19-point families) are padded with zeros."""
    c = _f64(c).ravel()
    if d == 2:
        assert c.size == 3, "2D takes 3 coefficients"
        return c
    assert c.size in (2, 3, 4), "3D takes 2, 3 or 4 coefficients"
    return np.concatenate([c, np.zeros(4 - c.size)])


def apply_A(d, N, u):
    """A_h u, the 5-/7-point negative Laplacian (eq. (A_h))."""
    u = _f64(u)
    out = np.empty_like(u)
    lib().or_apply_A(d, N, _p(u), _p(out))
    return out


def apply_K(d, N, which, v):
    v = _f64(v)
    out = np.empty_like(v)
    lib().or_apply_K(d, N, which, _p(v), _p(out))
    return out


def apply_W(d, N, c, r):
    """M r with M = h^2 sum_j c_j K_j, zero extension (Section 3)."""
    r = _f64(r)
    c = _coeffs(d, c)
    out = np.empty_like(r)
    lib().or_apply_W(d, N, _p(c), _p(r), _p(out))
    return out


def residual(d, N, u, b):
    u, b = _f64(u), _f64(b)
    out = np.empty_like(u)
    lib().or_residual(d, N, _p(u), _p(b), _p(out))
    return out


def smooth(d, N, c, u, b):
    """u + M (b - A_h u) (eq. (smoother), omega folded into M)."""
    u, b = _f64(u), _f64(b)
    c = _coeffs(d, c)
    out = np.empty_like(u)
    lib().or_smooth(d, N, _p(c), _p(u), _p(b), _p(out))
    return out


def restrict(d, N, r):
    """Full weighting onto the grid with N/2 intervals (Section 4)."""
    r = _f64(r)
    out = np.empty(shape(d, N // 2))
    lib().or_restrict(d, N, _p(r), _p(out))
    return out


def prolong_add(d, N, ec, u):
    """u + P ec, linear interpolation from the grid with N/2 intervals."""
    ec, u = _f64(ec), _f64(u).copy()
    lib().or_prolong_add(d, N, _p(ec), _p(u))
    return u


def restrict_T(d, N, bc):
    bc = _f64(bc)
    out = np.zeros(shape(d, N))
    lib().or_restrict_T_add(d, N, _p(bc), _p(out))
    return out


def prolong_T(d, N, uf):
    uf = _f64(uf)
    out = np.zeros(shape(d, N // 2))
    lib().or_prolong_T_add(d, N, _p(uf), _p(out))
    return out


def direct_solve(d, N, b):
    b = _f64(b)
    out = np.empty_like(b)
    lib().or_direct_solve(d, N, _p(b), _p(out))
    return out


def cycle(d, N, c, u, b, nu1=1, nu2=1, gamma=1):
    """One multigrid cycle (V for gamma=1, W for gamma=2), returns the new u."""
    u, b = _f64(u).copy(), _f64(b)
    c = _coeffs(d, c)
    lib().or_cycle(d, N, _p(c), nu1, nu2, gamma, _p(u), _p(b))
    return u


def vcycle(d, N, c, u, b, parallel=False):
    """One V(1,1) cycle; parallel=True runs the OpenMP build (same result)."""
    if not parallel:
        return cycle(d, N, c, u, b, 1, 1, 1)
    u, b = _f64(u).copy(), _f64(b)
    c = _coeffs(d, c)
    lib_omp().or_cycle(d, N, _p(c), 1, 1, 1, _p(u), _p(b))
    return u


def num_threads(parallel=False):
    """Threads the oracle's loops run on (1 for the plain build)."""
    return (lib_omp() if parallel else lib()).or_num_threads()


def solve(d, N, c, u, b, tol=1e-10, maxc=100, nu1=1, nu2=1, gamma=1):
    """Cycle until ||r_k|| <= tol ||r_0||.  Returns (u, cycles, history of
    ||r_k||_2); cycles is negative if maxc was reached (Section 4)."""
    u, b = _f64(u).copy(), _f64(b)
    c = _coeffs(d, c)
    hist = np.zeros(maxc + 1)
    k = lib().or_solve(d, N, _p(c), nu1, nu2, gamma, _p(u), _p(b), tol, maxc,
                       _p(hist))
    return u, k, hist[: abs(k) + 1].copy()


def norm2(v):
    v = _f64(v).ravel()
    return lib().or_norm2(v.size, _p(v))


def vcycle_adjoint(d, N, c, u, b, ubar_out):
    """Reverse-mode derivative of one V(1,1) cycle.  Returns (ubar_in, bbar,
    cbar) for the loss gradient ubar_out = dL/du_out."""
    u, b, ubar_out = _f64(u), _f64(b), _f64(ubar_out)
    nc = np.size(c)
    c = _coeffs(d, c)
    ubar_in = np.empty_like(u)
    bbar = np.zeros_like(u)
    cbar = np.zeros(c.size)
    lib().or_vcycle_adjoint(d, N, _p(c), _p(u), _p(b), _p(ubar_out),
                            _p(ubar_in), _p(bbar), _p(cbar))
    return ubar_in, bbar, cbar[:nc]


def _checkpoint(u, ckpt):
    """The cycle-start state as stored: unchanged ("fp64") or rounded to
    FP32 to nearest even ("fp32"), the value the forward pass continues
    from."""
    if ckpt == "fp64":
        return u
    assert ckpt == "fp32", ckpt
    return u.astype(np.float32).astype(np.float64)


def loss_kcycles(d, N, c, e0, b, K, ckpt="fp64"):
    """L = sum over the batch of ||u_K||^2 with u_K = V^K(e0, b); with
    ckpt="fp32" every cycle starts from the FP32 rounding of its input."""
    L = 0.0
    for e in _f64(e0).reshape((-1,) + shape(d, N)):
        u = e
        for _ in range(K):
            u = vcycle(d, N, c, _checkpoint(u, ckpt), b)
        L += float(np.dot(u.ravel(), u.ravel()))
    return L


def grad_kcycles(d, N, c, e0, b, K, ckpt="fp64"):
    """(L, dL/dc, dL/db, dL/de0) for loss_kcycles by reverse sweeps of
    vcycle_adjoint over per-cycle states.  With ckpt="fp32" the states are
    the FP32-rounded cycle inputs and the reverse sweep passes derivatives
    through each rounding unchanged (straight-through: the rounding is
    piecewise constant, so its derivative is taken as the identity)."""
    nc = np.size(c)
    c = _coeffs(d, c)
    cbar = np.zeros(c.size)
    bbar = np.zeros(shape(d, N))
    e0 = _f64(e0).reshape((-1,) + shape(d, N))
    e0bar = np.zeros_like(e0)
    L = 0.0
    for s, e in enumerate(e0):
        states, u = [], e
        for _ in range(K):
            states.append(_checkpoint(u, ckpt))
            u = vcycle(d, N, c, states[-1], b)
        L += float(np.dot(u.ravel(), u.ravel()))
        ubar = 2.0 * u
        for k in range(K - 1, -1, -1):
            ubar, bb, cb = vcycle_adjoint(d, N, c, states[k], b, ubar)
            bbar += bb
            cbar += cb
        e0bar[s] = ubar
    return L, cbar[:nc], bbar, e0bar


def descend(d, N, c0, e0, b, K, max_iter=200, rtol=1e-7, armijo=1e-4):
    """Coefficient fit by plain gradient descent with Armijo backtracking on
    loss_kcycles, gradients from grad_kcycles (reading of the unstated
    procedure for the coefficient-recovery experiment).  First trial step:
    1% of |c|; the trial step doubles after an accepted step and halves
    until L(c - a g) <= L(c) - armijo a |g|^2.  Stops when the accepted step
    is below rtol |c| or after max_iter steps.  Returns (c, L, steps)."""
    c = np.array(c0, dtype=np.float64)
    L, g, _, _ = grad_kcycles(d, N, c, e0, b, K)
    alpha = None
    it = 0
    for it in range(1, max_iter + 1):
        gn = float(np.linalg.norm(g))
        if gn == 0.0:
            break
        alpha = 1e-2 * float(np.linalg.norm(c)) / gn if alpha is None else 2.0 * alpha
        while True:
            cn = c - alpha * g
            Ln = loss_kcycles(d, N, cn, e0, b, K)
            if Ln <= L - armijo * alpha * gn * gn:
                break
            alpha *= 0.5
            if alpha * gn <= 1e-16 * float(np.linalg.norm(c)):
                break
        step = alpha * gn
        if Ln > L:
            break
        c = cn
        L, g, _, _ = grad_kcycles(d, N, c, e0, b, K)
        if step <= rtol * float(np.linalg.norm(c)):
            break
    return c, L, it
