"""Parity of every building-block kernel with the CPU oracle, element by
element, on seeded inputs: the fused residual + SPAI smoother (from a guess
and from zero), the fused residual + full-weighting restriction, linear
interpolation + correction and the LDS coarse tail, in FP64 and in the scaled
FP32 / FP16 storage of the refinement hierarchies.

Tolerances.  FP64 smoothing out = u + h^2 K (b - h^-2 L u): the residual
b - h^-2 L u carries an absolute rounding error of at most about
8 eps (|b| + 4d h^-2 |u|); K has weights summing to about 0.63 (M9) or 0.38
(M7) in h^2 units; so |out_gpu - out_oracle| <= 64 eps (max|u| + h^2 max|b|)
bounds every ordering and FMA contraction the kernel may use.  The same
bound with eps of FP32 holds for the FP32 storage; FP16 storage adds the
rounding of the stored output, one half-ulp, i.e. eps16 |out|.
"""
import numpy as np
import pytest

import oracle as O
from paper_2206_05543_amd import M7, M9
from tests._gpu import (EPS16, EPS32, EPS64, dev, gpu, host, make_mg, need_gpu, say,
                        torch)

pytestmark = gpu

CASES_2D = [16, 64, 512, 1024]
CASES_3D = [8, 32, 128]
STORE = {"fp64": np.float64, "fp32_ir": np.float32, "fp16_ir": np.float16}
EPS = {"fp64": EPS64, "fp32_ir": EPS32, "fp16_ir": EPS32}


def _coeffs(d):
    return np.array(M9 if d == 2 else M7)


def _rand(rng, shape, scale=1.0):
    return scale * rng.uniform(-1.0, 1.0, shape)


def _roundtrip(a, prec):
    """The values the GPU actually sees after storage rounding."""
    return a.astype(STORE[prec]).astype(np.float64)


def _tdt(prec):
    return {"fp64": torch.float64, "fp32_ir": torch.float32, "fp16_ir": torch.float16}[prec]


def _sigma(prec, N):
    # stored = sigma * true; the low-precision hierarchies store e / h^2
    return 1.0 if prec == "fp64" else float(N) * N


def _tol(prec, *mags, out_mag=0.0):
    t = 64 * EPS[prec] * sum(mags)
    if prec == "fp16_ir":
        t += EPS16 * out_mag
    return t


@pytest.mark.parametrize("prec", ["fp64", "fp32_ir", "fp16_ir"])
@pytest.mark.parametrize("d,N", [(2, n) for n in CASES_2D] + [(3, n) for n in CASES_3D])
@pytest.mark.parametrize("level", [0, 1])
def test_smooth_parity(d, N, level, prec):
    need_gpu()
    Nl = N >> level
    if Nl < 4:
        pytest.skip("level does not exist")
    rng = np.random.default_rng(100 + N + level)
    shp = (Nl - 1,) * d
    c = _coeffs(d)
    sig = _sigma(prec, Nl)
    # stored iterate O(1), rhs O(1) in the scaled form; true units for fp64
    us = _roundtrip(_rand(rng, shp), prec)
    b = _roundtrip(_rand(rng, shp, 1.0 if prec != "fp64" else Nl * Nl), prec)
    say("smooth", d, N, level, prec)
    with make_mg(N, d, c) as mg:
        out = torch.empty(shp, dtype=_tdt(prec), device="cuda")
        mg.sweep("smooth", level, prec, dev(us, _tdt(prec)), dev(b, _tdt(prec)), out)
        out0 = torch.empty_like(out)
        mg.sweep("smooth_zero", level, prec, None, dev(b, _tdt(prec)), out0)
        torch.cuda.synchronize()
        got, got0 = host(out), host(out0)
    want = O.smooth(d, Nl, c, us / sig, b) * sig
    want0 = O.apply_W(d, Nl, c, b) * sig
    h2 = 1.0 / (Nl * Nl)
    tol = _tol(prec, np.abs(us).max(), h2 * sig * np.abs(b).max(), out_mag=np.abs(want).max())
    tol0 = _tol(prec, h2 * sig * np.abs(b).max(), out_mag=np.abs(want0).max())
    assert np.max(np.abs(got - want)) <= tol
    assert np.max(np.abs(got0 - want0)) <= tol0


@pytest.mark.parametrize("prec", ["fp64", "fp32_ir", "fp16_ir"])
@pytest.mark.parametrize("d,N", [(2, n) for n in CASES_2D] + [(3, n) for n in CASES_3D])
def test_restrict_parity(d, N, prec):
    need_gpu()
    rng = np.random.default_rng(200 + N)
    shp, shc = (N - 1,) * d, (N // 2 - 1,) * d
    sig = _sigma(prec, N)
    us = _roundtrip(_rand(rng, shp), prec)
    b = _roundtrip(_rand(rng, shp, 1.0 if prec != "fp64" else N * N), prec)
    say("restrict", d, N, prec)
    with make_mg(N, d, _coeffs(d)) as mg:
        out = torch.empty(shc, dtype=_tdt(prec), device="cuda")
        mg.sweep("restrict", 0, prec, dev(us, _tdt(prec)), dev(b, _tdt(prec)), out)
        torch.cuda.synchronize()
        got = host(out)
    want = O.restrict(d, N, O.residual(d, N, us / sig, b))
    tol = _tol(prec, np.abs(b).max(), 4 * d * N * N / sig * np.abs(us).max(),
               out_mag=np.abs(want).max())
    assert np.max(np.abs(got - want)) <= tol


@pytest.mark.parametrize("prec", ["fp64", "fp32_ir", "fp16_ir"])
@pytest.mark.parametrize("d,N,level", [(2, n, 0) for n in CASES_2D] + [(2, 1024, 1)] +
                         [(3, n, 0) for n in CASES_3D + [256]] + [(3, 256, 1)])
def test_zero_smooth_restrict_parity(d, N, level, prec):
    # the fused zero-guess pre-smoother + restriction (2D tile kernel; 3D
    # march, with the large-grid shapes at N = 256 level 0): e = M b and
    # bc = R (b - A e), against the oracle's smoother and restriction
    need_gpu()
    Nl = N >> level
    rng = np.random.default_rng(300 + N + level)
    shp, shc = (Nl - 1,) * d, (Nl // 2 - 1,) * d
    c = _coeffs(d)
    sig = _sigma(prec, Nl)
    b = _roundtrip(_rand(rng, shp, 1.0 if prec != "fp64" else Nl * Nl), prec)
    say("zero-smooth-restrict", d, N, level, prec)
    with make_mg(N, d, c) as mg:
        e = torch.empty(shp, dtype=_tdt(prec), device="cuda")
        bc = torch.empty(shc, dtype=_tdt(prec), device="cuda")
        mg.sweep_zero_restrict(level, prec, dev(b, _tdt(prec)), e, bc)
        torch.cuda.synchronize()
        got_e, got_c = host(e), host(bc)
    e_true = O.apply_W(d, Nl, c, b)
    want_e = e_true * sig
    want_c = O.restrict(d, Nl, O.residual(d, Nl, e_true, b))
    h2 = 1.0 / (Nl * Nl)
    tol_e = _tol(prec, h2 * sig * np.abs(b).max(), out_mag=np.abs(want_e).max())
    tol_c = _tol(prec, np.abs(b).max(), 4 * d * Nl * Nl / sig * np.abs(want_e).max(),
                 out_mag=np.abs(want_c).max())
    assert np.max(np.abs(got_e - want_e)) <= tol_e
    assert np.max(np.abs(got_c - want_c)) <= tol_c


@pytest.mark.parametrize("prec", ["fp64", "fp32_ir", "fp16_ir"])
@pytest.mark.parametrize("d,N,level,batch", [(2, n, 0, 1) for n in CASES_2D] +
                         [(2, 1024, 1, 1), (2, 2048, 0, 1), (2, 4096, 0, 1), (2, 64, 0, 3),
                          (2, 8, 0, 2)] +
                         [(3, n, 0, 1) for n in CASES_3D + [256]] +
                         [(3, 256, 1, 1), (3, 32, 0, 2), (3, 8, 0, 3)])
def test_smooth_restrict_parity(d, N, level, batch, prec):
    # the fused pre-smoother + restriction: out = u + M (b - A u) and
    # bc = R (b - A out), against the oracle's smoother, residual and
    # restriction (2D strips, 3D tiles, both with ragged last tiles and
    # chunks along the march; the large-grid shapes at 2D N >= 2048 and 3D
    # N = 256; several batch entries; the smallest grid with a coarse level)
    need_gpu()
    Nl = N >> level
    rng = np.random.default_rng(400 + N + level + batch)
    shp, shc = (Nl - 1,) * d, (Nl // 2 - 1,) * d
    c = _coeffs(d)
    sig = _sigma(prec, Nl)
    us = _roundtrip(_rand(rng, (batch,) + shp), prec)
    b = _roundtrip(_rand(rng, (batch,) + shp, 1.0 if prec != "fp64" else Nl * Nl), prec)
    say("smooth-restrict", N, level, batch, prec)
    with make_mg(N, d, c, batch=batch) as mg:
        out = torch.empty((batch,) + shp, dtype=_tdt(prec), device="cuda")
        bc = torch.empty((batch,) + shc, dtype=_tdt(prec), device="cuda")
        mg.sweep_smooth_restrict(level, prec, dev(us, _tdt(prec)), dev(b, _tdt(prec)), out, bc)
        torch.cuda.synchronize()
        got, got_c = host(out), host(bc)
    h2 = 1.0 / (Nl * Nl)
    for e in range(batch):
        v_true = O.smooth(d, Nl, c, us[e] / sig, b[e])
        want = v_true * sig
        want_c = O.restrict(d, Nl, O.residual(d, Nl, v_true, b[e]))
        tol = _tol(prec, np.abs(us[e]).max(), h2 * sig * np.abs(b[e]).max(),
                   out_mag=np.abs(want).max())
        # the second residual sees the stored new iterate: its rounding
        # (half an ulp of S) passes through A (weights summing to 4d / h^2)
        tol_c = _tol(prec, np.abs(b[e]).max(), 4 * d * Nl * Nl / sig * np.abs(want).max(),
                     out_mag=np.abs(want_c).max())
        if prec == "fp16_ir":
            tol_c += 4 * d * Nl * Nl / sig * EPS16 * np.abs(want).max()
        assert np.max(np.abs(got[e] - want)) <= tol, e
        assert np.max(np.abs(got_c[e] - want_c)) <= tol_c, e


@pytest.mark.parametrize("prec", ["fp64", "fp32_ir", "fp16_ir"])
@pytest.mark.parametrize("N,level,batch", [(n, 0, 1) for n in CASES_2D] +
                         [(1024, 1, 1), (2048, 0, 1), (4096, 0, 1), (64, 0, 3), (8, 0, 2)])
def test_post_pre_restrict_parity(N, level, batch, prec):
    # the sweeps between two 2D V(1,1) cycles as one kernel: w = t + P ec,
    # u_{k+1} = w + M (b - A w), t2 = u_{k+1} + M (b - A u_{k+1}) and
    # bc = R (b - A t2), against the oracle's interpolation, smoother,
    # residual and restriction (strips with ragged last strips and row
    # chunks, the large-grid shape at N >= 4096, several batch entries)
    need_gpu()
    d = 2
    Nl = N >> level
    rng = np.random.default_rng(500 + N + level + batch)
    shp, shc = (Nl - 1,) * d, (Nl // 2 - 1,) * d
    c = _coeffs(d)
    sig, sigc = _sigma(prec, Nl), _sigma(prec, Nl // 2)
    ts = _roundtrip(_rand(rng, (batch,) + shp), prec)
    ecs = _roundtrip(_rand(rng, (batch,) + shc), prec)
    b = _roundtrip(_rand(rng, (batch,) + shp, 1.0 if prec != "fp64" else Nl * Nl), prec)
    say("post-pre-restrict", N, level, batch, prec)
    T = _tdt(prec)
    with make_mg(N, d, c, batch=batch) as mg:
        out = torch.empty((batch,) + shp, dtype=T, device="cuda")
        out_t = torch.empty((batch,) + shp, dtype=T, device="cuda")
        bc = torch.empty((batch,) + shc, dtype=T, device="cuda")
        mg.sweep_post_pre_restrict(level, prec, dev(ts, T), dev(ecs, T), dev(b, T), out, out_t,
                                   bc)
        torch.cuda.synchronize()
        got, got_t, got_c = host(out), host(out_t), host(bc)
    h2 = 1.0 / (Nl * Nl)
    for e in range(batch):
        w = O.prolong_add(d, Nl, ecs[e] / sigc, ts[e] / sig)
        u1 = O.smooth(d, Nl, c, w, b[e])
        t2 = O.smooth(d, Nl, c, u1, b[e])
        want_c = O.restrict(d, Nl, O.residual(d, Nl, t2, b[e]))
        bmag = h2 * sig * np.abs(b[e]).max()
        # each stage as in the single-sweep tests; the stored u_{k+1} (half
        # an ulp of S) enters the next sweep through A (weights 4d / h^2)
        # and K (weights below 1 in h^2 units)
        tol1 = _tol(prec, 2 * np.abs(w).max() * sig, bmag, out_mag=np.abs(u1).max() * sig)
        tol2 = 2 * tol1 + _tol(prec, np.abs(u1).max() * sig, bmag,
                               out_mag=np.abs(t2).max() * sig)
        tol_c = _tol(prec, np.abs(b[e]).max(), 4 * d * Nl * Nl / sig * np.abs(t2).max() * sig,
                     out_mag=np.abs(want_c).max()) + 4 * d * Nl * Nl / sig * tol2
        assert np.max(np.abs(got[e] - u1 * sig)) <= tol1, e
        assert np.max(np.abs(got_t[e] - t2 * sig)) <= tol2, e
        assert np.max(np.abs(got_c[e] - want_c)) <= tol_c, e


def test_post_pre_restrict_rejects_bad_requests():
    # 2D only, and only where a coarser level exists; nothing is launched
    need_gpu()
    from paper_2206_05543_amd._lib import MGError
    f = lambda N, d: torch.zeros((N - 1,) * d, dtype=torch.float64, device="cuda")
    fc = lambda N, d: torch.zeros((N // 2 - 1,) * d, dtype=torch.float64, device="cuda")
    with make_mg(16, 3, _coeffs(3)) as mg:
        with pytest.raises(MGError, match="2D only"):
            mg.sweep_post_pre_restrict(0, "fp64", f(16, 3), fc(16, 3), f(16, 3), f(16, 3),
                                       f(16, 3), fc(16, 3))
    with make_mg(8, 2, _coeffs(2)) as mg:
        last = mg.num_levels - 1
        with pytest.raises((MGError, ValueError)):
            mg.sweep_post_pre_restrict(last, "fp64", f(4, 2), fc(4, 2), f(4, 2), f(4, 2),
                                       f(4, 2), fc(4, 2))


@pytest.mark.parametrize("prec", ["fp64", "fp32_ir", "fp16_ir"])
@pytest.mark.parametrize("d,N", [(2, n) for n in CASES_2D] + [(3, n) for n in CASES_3D])
def test_prolong_parity(d, N, prec):
    need_gpu()
    rng = np.random.default_rng(300 + N)
    shp, shc = (N - 1,) * d, (N // 2 - 1,) * d
    sig, sigc = _sigma(prec, N), _sigma(prec, N // 2)
    us = _roundtrip(_rand(rng, shp), prec)
    ecs = _roundtrip(_rand(rng, shc), prec)
    say("prolong", d, N, prec)
    with make_mg(N, d, _coeffs(d)) as mg:
        out = dev(us, _tdt(prec))
        mg.sweep("prolong_add", 0, prec, dev(ecs, _tdt(prec)), None, out)
        torch.cuda.synchronize()
        got = host(out)
    want = O.prolong_add(d, N, ecs / sigc, us / sig) * sig
    tol = _tol(prec, np.abs(us).max(), 4 * np.abs(ecs).max(), out_mag=np.abs(want).max())
    assert np.max(np.abs(got - want)) <= tol


@pytest.mark.parametrize("prec", ["fp64", "fp32_ir", "fp16_ir"])
@pytest.mark.parametrize("d,N", [(2, n) for n in CASES_2D] + [(3, n) for n in CASES_3D])
@pytest.mark.parametrize("level", [0, 1])
def test_smooth_correct_parity(d, N, level, prec):
    # post-smoothing with the coarse-grid correction fused into the sweep
    need_gpu()
    Nl = N >> level
    if Nl < 8:
        pytest.skip("needs a coarser level")
    rng = np.random.default_rng(500 + N + level)
    shp, shc = (Nl - 1,) * d, (Nl // 2 - 1,) * d
    c = _coeffs(d)
    sig, sigc = _sigma(prec, Nl), _sigma(prec, Nl // 2)
    us = _roundtrip(_rand(rng, shp), prec)
    ecs = _roundtrip(_rand(rng, shc), prec)
    b = _roundtrip(_rand(rng, shp, 1.0 if prec != "fp64" else Nl * Nl), prec)
    say("smooth-correct", d, N, level, prec)
    with make_mg(N, d, c) as mg:
        out = torch.empty(shp, dtype=_tdt(prec), device="cuda")
        mg.sweep_correct(level, prec, dev(us, _tdt(prec)), dev(ecs, _tdt(prec)),
                         dev(b, _tdt(prec)), out)
        torch.cuda.synchronize()
        got = host(out)
    v = O.prolong_add(d, Nl, ecs / sigc, us / sig)
    want = O.smooth(d, Nl, c, v, b) * sig
    h2 = 1.0 / (Nl * Nl)
    tol = _tol(prec, np.abs(us).max() + 4 * np.abs(ecs).max(), h2 * sig * np.abs(b).max(),
               out_mag=np.abs(want).max())
    assert np.max(np.abs(got - want)) <= tol


@pytest.mark.parametrize("prec", ["fp64", "fp32_ir", "fp16_ir"])
@pytest.mark.parametrize("d,N,level", [(2, 64, 0), (2, 64, 1), (2, 128, 1), (2, 16, 1), (2, 8, 1),
                                       (3, 32, 1), (3, 16, 1), (3, 8, 1)])
def test_coarse_tail_parity(d, N, level, prec):
    # a zero-guess V(1,1) cycle below `level`, run entirely by the LDS tail
    # kernel when N >> level is within the tail range, else by the level
    # kernels down to the tail
    need_gpu()
    Nl = N >> level
    rng = np.random.default_rng(400 + N)
    shp = (Nl - 1,) * d
    sig = _sigma(prec, Nl)
    b = _roundtrip(_rand(rng, shp), prec)
    say("coarse-cycle", d, N, level, prec)
    with make_mg(N, d, _coeffs(d), precision=prec) as mg:
        e = torch.empty(shp, dtype=_tdt(prec), device="cuda")
        mg.coarse_cycle(level, prec, dev(b, _tdt(prec)), e)
        torch.cuda.synchronize()
        got = host(e)
    want = O.vcycle(d, Nl, _coeffs(d), np.zeros(shp), b) * sig
    # the cycle is a fixed linear map of norm O(1) in the scaled units; its
    # rounding errors are bounded by a few hundred eps times the magnitudes
    scale = np.abs(want).max()
    tol = {"fp64": 1e-12, "fp32_ir": 2e-5, "fp16_ir": 2e-2}[prec] * scale
    assert np.max(np.abs(got - want)) <= tol
