"""ctypes binding of libspaimg.so (include/spaimg.h).

Argument marshalling only: every grid operation runs in the library's HIP
kernels.  torch tensors serve as device memory (``data_ptr()``) and the
caller's current HIP stream is passed through.  There is no CPU fallback:
if the library is missing this module raises on first use.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspaimg.so")

MG_OK, MG_EINVAL, MG_EHIP, MG_ENOCONV, MG_ENONFINITE = 0, -1, -2, -3, -4
OPT_PRECISION, OPT_BATCH, OPT_MAX_CYCLES, OPT_TAIL_N, OPT_TIMING = 1, 2, 3, 4, 5
OPT_INNER_CYCLES, OPT_CYCLE = 6, 7
CYCLE = {"V11": 0, "W10": 1}
PREC = {"fp64": 0, "fp32_ir": 1, "fp16_ir": 2}
OP = {"smooth": 0, "smooth_zero": 1, "restrict": 2, "prolong_add": 3}
TIME = {"smooth": 0, "smooth_zero": 1, "restrict": 2, "prolong": 3, "tail": 4,
        "ir_step": 5, "residual": 6, "smooth_correct": 7, "zero_smooth_restrict": 8,
        "smooth_restrict": 9, "post_pre_restrict": 10}
STORAGE = {0: torch.float64, 1: torch.float32, 2: torch.float16}
CKPT = {torch.float64: 0, torch.float32: 1}

_lib = None


class MGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libspaimg error {code}: {msg}")
        self.code = code


class MGStats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("cycles_run", ctypes.c_int),
                ("r0_norm", ctypes.c_double), ("rk_norm", ctypes.c_double),
                ("b_norm", ctypes.c_double),
                ("res_hist", ctypes.POINTER(ctypes.c_double)),
                ("hist_cap", ctypes.c_int), ("elapsed_ms", ctypes.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        dp = ctypes.POINTER(ctypes.c_double)
        L.mg_setup.argtypes = [i, i, dp, i, ctypes.POINTER(vp)]
        L.mg_set_option.argtypes = [vp, i, dbl]
        L.mg_set_coeffs.argtypes = [vp, dp, i]
        L.mg_vcycle.argtypes = [vp, vp, vp, vp]
        L.mg_vcycle_noalloc.argtypes = [i, i, dp, i, i, vp, vp, vp]
        L.mg_solve.argtypes = [vp, vp, vp, dbl, ctypes.POINTER(MGStats), vp]
        L.mg_vcycle_adjoint.argtypes = [vp, vp, vp, i, vp, vp, vp, dp, vp]
        L.mg_checkpoint.argtypes = [vp, vp, vp, i, vp]
        L.mg_sweep.argtypes = [vp, i, i, i, vp, vp, vp, vp]
        L.mg_coarse_cycle.argtypes = [vp, i, i, vp, vp, vp]
        L.mg_sweep_correct.argtypes = [vp, i, i, vp, vp, vp, vp, vp]
        L.mg_sweep_zero_restrict.argtypes = [vp, i, i, vp, vp, vp, vp]
        L.mg_sweep_smooth_restrict.argtypes = [vp, i, i, vp, vp, vp, vp, vp]
        L.mg_sweep_post_pre_restrict.argtypes = [vp, i, i, vp, vp, vp, vp, vp, vp, vp]
        L.mg_residual_norm.argtypes = [vp, vp, vp, dp, vp]
        L.mg_get_timing.argtypes = [vp, i, i, dp, ctypes.POINTER(i)]
        L.mg_reset_timing.argtypes = [vp]
        L.mg_num_levels.argtypes = [vp]
        L.mg_destroy.argtypes = [vp]
        L.mg_destroy.restype = None
        L.mg_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc != MG_OK:
        raise MGError(rc, lib().mg_last_error().decode())
    return rc


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dbl_array(vals):
    arr = (ctypes.c_double * len(vals))(*[float(v) for v in vals])
    return arr


NOALLOC_SCRATCH_BYTES = 32 << 20


def vcycle_noalloc(N, d, coeffs, b, u, batch=1):
    """One FP64 V(1,1) cycle u <- V(u, b) without a handle (mg_vcycle_noalloc):
    no allocation, internal buffers in the library's static workspace."""
    n = int(N) - 1
    for t, name in ((b, "b"), (u, "u")):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError(f"{name} must be a CUDA tensor")
        if t.dtype != torch.float64 or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous float64 tensor")
        if t.numel() != int(batch) * n ** int(d):
            raise ValueError(f"{name} has {t.numel()} elements, the problem needs "
                             f"{int(batch) * n ** int(d)}")
    _check(lib().mg_vcycle_noalloc(int(N), int(d), _dbl_array(coeffs), len(coeffs), int(batch),
                                   ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                   _stream()))
    return u


class Multigrid:
    """Handle on one solver instance (mg_setup ... mg_destroy)."""

    def __init__(self, N, d, coeffs, batch=1, precision="fp64", max_cycles=100,
                 tail_N=0, timing=0, cycle="V11"):
        self.N, self.d = int(N), int(d)
        self.n = self.N - 1
        self.ncoef = len(coeffs)
        h = ctypes.c_void_p()
        c = _dbl_array(coeffs)
        _check(lib().mg_setup(self.N, self.d, c, len(coeffs), ctypes.byref(h)))
        self._h = h
        self.batch = 1
        self.precision = "fp64"
        self.set_option(OPT_MAX_CYCLES, max_cycles)
        self.max_cycles = int(max_cycles)
        if batch != 1:
            self.set_batch(batch)
        if precision != "fp64":
            self.set_precision(precision)
        if tail_N:
            self.set_option(OPT_TAIL_N, tail_N)
        if timing:
            self.set_option(OPT_TIMING, timing)
        self.cycle = "V11"
        if cycle != "V11":
            self.set_cycle(cycle)

    # ---- options
    def set_option(self, key, value):
        _check(lib().mg_set_option(self._h, key, float(value)))

    def set_batch(self, batch):
        self.set_option(OPT_BATCH, batch)
        self.batch = int(batch)

    def set_precision(self, precision):
        self.set_option(OPT_PRECISION, PREC[precision])
        self.precision = precision

    def set_cycle(self, cycle):
        """"V11" (V(1,1)) or "W10" (W(1,0)) for vcycle, solve and refinement."""
        self.set_option(OPT_CYCLE, CYCLE[cycle])
        self.cycle = cycle

    def set_coeffs(self, coeffs):
        _check(lib().mg_set_coeffs(self._h, _dbl_array(coeffs), len(coeffs)))

    @property
    def num_levels(self):
        return lib().mg_num_levels(self._h)

    # ---- argument checks (shapes only; the library checks the rest)
    def level_numel(self, level):
        n = (self.N >> level) - 1
        return self.batch * n ** self.d

    def _field(self, t, level=0, dtype=torch.float64, name="field"):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError(f"{name} must be a CUDA tensor")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.numel() != self.level_numel(level):
            raise ValueError(f"{name} has {t.numel()} elements, level {level} needs "
                             f"{self.level_numel(level)}")
        return ctypes.c_void_p(t.data_ptr())

    # ---- entry points
    def vcycle(self, b, u):
        _check(lib().mg_vcycle(self._h, self._field(b, name="b"), self._field(u, name="u"),
                               _stream()))
        return u

    def solve(self, b, u, tol=1e-10):
        hist = (ctypes.c_double * (self.max_cycles + 2))()
        st = MGStats()
        st.res_hist = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
        st.hist_cap = self.max_cycles + 2
        rc = lib().mg_solve(self._h, self._field(b, name="b"), self._field(u, name="u"),
                            float(tol), ctypes.byref(st), _stream())
        out = {"cycles": st.cycles, "cycles_run": st.cycles_run, "r0": st.r0_norm,
               "rk": st.rk_norm, "b_norm": st.b_norm, "elapsed_ms": st.elapsed_ms,
               "history": [hist[j] for j in range(min(st.cycles + 1, st.hist_cap))],
               "code": rc}
        if rc not in (MG_OK, MG_ENOCONV):
            _check(rc)
        return out

    def checkpoint(self, u, ckpt):
        """ckpt <- u (FP64) or its FP32 rounding, which then replaces u."""
        if ckpt.dtype not in CKPT:
            raise TypeError("checkpoints are float64 or float32")
        _check(lib().mg_checkpoint(self._h, self._field(u, name="u"),
                                   self._field(ckpt, dtype=ckpt.dtype, name="ckpt"),
                                   CKPT[ckpt.dtype], _stream()))
        return ckpt

    def vcycle_adjoint(self, b, u_in, ubar_out, ubar_in, bbar_acc, cbar_acc):
        """u_in: the cycle's checkpoint, float64 or float32."""
        if u_in.dtype not in CKPT:
            raise TypeError("checkpoints are float64 or float32")
        cb = (ctypes.c_double * self.ncoef)(*[float(x) for x in cbar_acc])
        _check(lib().mg_vcycle_adjoint(
            self._h, self._field(b, name="b"),
            self._field(u_in, dtype=u_in.dtype, name="u_in"), CKPT[u_in.dtype],
            self._field(ubar_out, name="ubar_out"), self._field(ubar_in, name="ubar_in"),
            self._field(bbar_acc, name="bbar_acc"), cb, _stream()))
        return [cb[j] for j in range(self.ncoef)]

    def sweep(self, op, level, prec, u, b, out):
        code = PREC[prec]
        dt = STORAGE[code]
        o = OP[op]
        lu = level + 1 if o == 3 else level
        lo = level + 1 if o == 2 else level
        pu = None if o == 1 else self._field(u, lu, dt, "u")
        pb = None if o == 3 else self._field(b, level, dt, "b")
        po = self._field(out, lo, dt, "out")
        _check(lib().mg_sweep(self._h, o, level, code, pu, pb, po, _stream()))
        return out

    def sweep_correct(self, level, prec, u, ec, b, out):
        dt = STORAGE[PREC[prec]]
        _check(lib().mg_sweep_correct(
            self._h, level, PREC[prec], self._field(u, level, dt, "u"),
            self._field(ec, level + 1, dt, "ec"), self._field(b, level, dt, "b"),
            self._field(out, level, dt, "out"), _stream()))
        return out

    def sweep_zero_restrict(self, level, prec, b, e, bc):
        dt = STORAGE[PREC[prec]]
        _check(lib().mg_sweep_zero_restrict(
            self._h, level, PREC[prec], self._field(b, level, dt, "b"),
            self._field(e, level, dt, "e"), self._field(bc, level + 1, dt, "bc"), _stream()))
        return e, bc

    def sweep_smooth_restrict(self, level, prec, u, b, out, bc):
        dt = STORAGE[PREC[prec]]
        _check(lib().mg_sweep_smooth_restrict(
            self._h, level, PREC[prec], self._field(u, level, dt, "u"),
            self._field(b, level, dt, "b"), self._field(out, level, dt, "out"),
            self._field(bc, level + 1, dt, "bc"), _stream()))
        return out, bc

    def sweep_post_pre_restrict(self, level, prec, u, ec, b, out, out_t, bc):
        dt = STORAGE[PREC[prec]]
        _check(lib().mg_sweep_post_pre_restrict(
            self._h, level, PREC[prec], self._field(u, level, dt, "u"),
            self._field(ec, level + 1, dt, "ec"), self._field(b, level, dt, "b"),
            self._field(out, level, dt, "out"), self._field(out_t, level, dt, "out_t"),
            self._field(bc, level + 1, dt, "bc"), _stream()))
        return out, out_t, bc

    def set_inner_cycles(self, m):
        self.set_option(OPT_INNER_CYCLES, m)

    def coarse_cycle(self, level, prec, b, e):
        code = PREC[prec]
        dt = STORAGE[code]
        _check(lib().mg_coarse_cycle(self._h, level, code, self._field(b, level, dt, "b"),
                                     self._field(e, level, dt, "e"), _stream()))
        return e

    def residual_norm(self, b, u):
        out = ctypes.c_double()
        _check(lib().mg_residual_norm(self._h, self._field(b, name="b"),
                                      self._field(u, name="u"), ctypes.byref(out), _stream()))
        return out.value

    def timing(self, kind, level=0):
        ms, cnt = ctypes.c_double(), ctypes.c_int()
        _check(lib().mg_get_timing(self._h, TIME[kind], level, ctypes.byref(ms),
                                   ctypes.byref(cnt)))
        return ms.value, cnt.value

    def reset_timing(self):
        _check(lib().mg_reset_timing(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().mg_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
