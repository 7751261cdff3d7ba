"""Thin Python binding of the SHLR C ABI (``include/shlr.h``).

Argument marshalling only: every step of the reconstruction runs in the HIP
kernels of ``libshlr.so``.  PyTorch supplies device memory and the stream.
Importing this module raises if the shared library is missing; there is no
fallback implementation.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libshlr.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2107_11650_amd.build` "
                      "(or __graft_entry__.build()); there is no CPU fallback")

_lib = ctypes.CDLL(LIB_PATH)

MODEL_PI = 0
MODEL_PARAM = 1
PREC_MIXED = 0
PREC_FP64 = 1
PREC_MIXED_R32 = 2   # opt-in: FP32 Householder reduction (see include/shlr.h)

STATUS = {
    0: "SHLR_OK", 1: "SHLR_E_INVALID_ARG", 2: "SHLR_E_SINGULAR", 3: "SHLR_E_NONFINITE",
    4: "SHLR_E_WORKSPACE", 5: "SHLR_E_DEVICE", 6: "SHLR_E_UNSUPPORTED", 7: "SHLR_E_STATE",
    8: "SHLR_E_EIG_NOCONV",
}

EXPORTED = [
    "shlr_plan_create", "shlr_plan_destroy", "shlr_workspace_size", "shlr_bind", "shlr_set_spirit_kernel",
    "shlr_calibrate_spirit", "shlr_init", "shlr_iterate", "shlr_iterate_graph", "shlr_get_kspace",
    "shlr_reconstruct", "shlr_fft_lines", "shlr_lowrank_workspace_size", "shlr_lowrank_lines",
    "shlr_last_error", "shlr_version", "shlr_timing_enable", "shlr_timing_enable_phases", "shlr_timing_read",
    "shlr_unrolled_sizes", "shlr_unrolled_forward", "shlr_unrolled_backward", "shlr_autotune",
    "shlr_params_default", "shlr_unit_status", "shlr_set_eig_check", "shlr_set_weights",
    "shlr_lowrank_lines_noalloc", "shlr_ssos", "shlr_rlne", "shlr_mssim", "shlr_t2_fit",
]
EVAL_WORK_BYTES = 65536
TIMING_PHASES = ("xupdate", "gram", "eig", "reproj", "spirit", "tridiag")


class ShlrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class CParams(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int32), ("precision", ctypes.c_int32), ("n_slices", ctypes.c_int32),
        ("M", ctypes.POINTER(ctypes.c_int32)), ("N", ctypes.POINTER(ctypes.c_int32)),
        ("J", ctypes.c_int32), ("L", ctypes.c_int32), ("k_row", ctypes.c_int32), ("k_col", ctypes.c_int32),
        ("use_vc", ctypes.c_int32), ("use_w", ctypes.c_int32), ("spirit_ksize", ctypes.c_int32),
        ("hard_dc", ctypes.c_int32), ("normalize", ctypes.c_int32), ("max_iter", ctypes.c_int32),
        ("n_cg", ctypes.c_int32),
        ("lam", ctypes.c_double), ("lambda1", ctypes.c_double), ("lambda2", ctypes.c_double),
        ("beta", ctypes.c_double), ("tau", ctypes.c_double), ("tol", ctypes.c_double), ("d0", ctypes.c_double),
        ("slot_budget", ctypes.c_int64),
    ]


class CInfo(ctypes.Structure):
    _fields_ = [("iters_done", ctypes.c_int32), ("converged", ctypes.c_int32), ("rel_change", ctypes.c_double),
                ("scale", ctypes.c_double), ("device_flags", ctypes.c_uint32)]


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_lib.shlr_plan_create.argtypes = [ctypes.POINTER(CParams), ctypes.POINTER(_vp)]
_lib.shlr_plan_destroy.argtypes = [_vp]
_lib.shlr_plan_destroy.restype = None
_lib.shlr_workspace_size.argtypes = [_vp, ctypes.POINTER(ctypes.c_size_t)]
_lib.shlr_bind.argtypes = [_vp, _vp, ctypes.c_size_t, _vp]
_lib.shlr_set_spirit_kernel.argtypes = [_vp, _vp]
_lib.shlr_calibrate_spirit.argtypes = [_vp, _i32, ctypes.c_double]
_lib.shlr_init.argtypes = [_vp, _vp, _vp]
_lib.shlr_iterate.argtypes = [_vp, _i32, ctypes.POINTER(CInfo)]
_lib.shlr_iterate_graph.argtypes = [_vp, _i32, ctypes.POINTER(CInfo)]
_lib.shlr_get_kspace.argtypes = [_vp, _vp]
_lib.shlr_reconstruct.argtypes = [_vp, _vp, _vp, _vp, ctypes.POINTER(CInfo)]
_lib.shlr_fft_lines.argtypes = [_i32, _i32, _i32, _i32, _vp, _vp, _vp]
_lib.shlr_lowrank_workspace_size.argtypes = [_i32, _i32, _i32, _i32, _i32, _i32, ctypes.POINTER(ctypes.c_size_t)]
_lib.shlr_lowrank_lines.argtypes = [_i32, _i32, _i32, _i32, _i32, _i32, _i32, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]
_lib.shlr_unrolled_sizes.argtypes = [_vp, _i32, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
_lib.shlr_unrolled_forward.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, ctypes.c_size_t]
_lib.shlr_unrolled_backward.argtypes = [_vp, _i32, _vp, _vp, ctypes.c_size_t, _vp, ctypes.c_size_t, _vp,
                                        ctypes.POINTER(ctypes.c_double)]
_lib.shlr_autotune.argtypes = [_vp, _i32, ctypes.c_char_p, ctypes.c_size_t]
_lib.shlr_params_default.argtypes = [_i32, _vp]
_lib.shlr_unit_status.argtypes = [_vp, _i32, _vp, _vp, _vp]
_lib.shlr_set_eig_check.argtypes = [_vp, ctypes.c_double]
_lib.shlr_set_weights.argtypes = [_vp, _vp, _vp]
_lib.shlr_ssos.argtypes = [_i32, _i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp]
_lib.shlr_rlne.argtypes = [_i32, ctypes.c_int64, _vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_double), _vp]
_lib.shlr_mssim.argtypes = [_i32, _i32, _i32, _vp, _vp, ctypes.c_double, _vp, ctypes.POINTER(ctypes.c_double), _vp]
_lib.shlr_t2_fit.argtypes = [_i32, _i32, ctypes.c_int64, _vp, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                             _vp, _vp, _vp, _vp, _vp]
_lib.shlr_lowrank_lines_noalloc.argtypes = [_i32, _i32, _i32, _i32, _i32, _i32, _i32, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double, _vp, _vp, _vp, _vp, _vp]
_lib.shlr_timing_enable.argtypes = [_vp, _i32]
_lib.shlr_timing_enable_phases.argtypes = [_vp, ctypes.c_uint32]
_lib.shlr_timing_read.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]
_lib.shlr_last_error.restype = ctypes.c_char_p
_lib.shlr_version.restype = ctypes.c_char_p
for _f in EXPORTED:
    if _f not in ("shlr_plan_destroy", "shlr_last_error", "shlr_version"):
        getattr(_lib, _f).restype = ctypes.c_int


def _check(code):
    if code != 0:
        raise ShlrError(code, _lib.shlr_last_error().decode())


def version() -> str:
    return _lib.shlr_version().decode()


def library():
    return _lib


@dataclass
class Params:
    """Mirror of ``shlr_params`` (see include/shlr.h for the meaning of each field)."""
    model: int = MODEL_PI
    precision: int = PREC_MIXED
    M: tuple = (64,)
    N: tuple = (64,)
    J: int = 4
    L: int = 1
    k_row: int = 8
    k_col: int = 8
    use_vc: bool = False
    use_w: bool = True
    spirit_ksize: int = 0
    hard_dc: bool = False
    normalize: bool = True
    max_iter: int = 20
    n_cg: int = 10
    lam: float = 1e4
    lambda1: float = 0.0
    lambda2: float = 2.0
    beta: float = 10.0
    tau: float | None = None
    tol: float = 0.0
    d0: float = 1.0
    slot_budget: int = 0

    def to_c(self):
        n = len(self.M)
        Ma = (ctypes.c_int32 * n)(*[int(v) for v in self.M])
        Na = (ctypes.c_int32 * n)(*[int(v) for v in self.N])
        c = CParams(model=self.model, precision=self.precision, n_slices=n, M=Ma, N=Na, J=self.J, L=self.L,
                    k_row=self.k_row, k_col=self.k_col, use_vc=int(self.use_vc), use_w=int(self.use_w),
                    spirit_ksize=self.spirit_ksize, hard_dc=int(self.hard_dc), normalize=int(self.normalize),
                    max_iter=self.max_iter, n_cg=self.n_cg, lam=self.lam, lambda1=self.lambda1,
                    lambda2=self.lambda2, beta=self.beta, tau=self.beta if self.tau is None else self.tau,
                    tol=self.tol, d0=self.d0, slot_budget=int(self.slot_budget))
        return c, (Ma, Na)

    @classmethod
    def paper_defaults(cls, model=MODEL_PI, **fields):
        """Params holding the library's defaults for a model (shlr_params_default: the iteration cap,
        tolerance and initial multipliers of Algorithms S1 / S2), then the given fields."""
        c = CParams()
        _check(_lib.shlr_params_default(int(model), ctypes.byref(c)))
        base = dict(model=c.model, precision=c.precision, use_vc=bool(c.use_vc), use_w=bool(c.use_w),
                    spirit_ksize=c.spirit_ksize, hard_dc=bool(c.hard_dc), normalize=bool(c.normalize),
                    max_iter=c.max_iter, n_cg=c.n_cg, tol=c.tol, d0=c.d0)
        base.update(fields)
        return cls(**base)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    """A bound SHLR plan: workspace from torch, work on torch's current stream."""

    def __init__(self, params: Params, device="cuda"):
        import torch
        self.params = params
        c, keep = params.to_c()
        h = ctypes.c_void_p()
        _check(_lib.shlr_plan_create(ctypes.byref(c), ctypes.byref(h)))
        self._h = h
        nb = ctypes.c_size_t()
        _check(_lib.shlr_workspace_size(h, ctypes.byref(nb)))
        self.ws_bytes = nb.value
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
        off = (-self.ws.data_ptr()) % 256
        self._ws_ptr = ctypes.c_void_p(self.ws.data_ptr() + off)
        _check(_lib.shlr_bind(h, self._ws_ptr, ctypes.c_size_t(self.ws_bytes), _stream()))

    @property
    def cdtype(self):
        import torch
        return torch.complex128 if self.params.precision == PREC_FP64 else torch.complex64

    def _prep(self, y, mask):
        import torch
        y = y.to(self.cdtype).contiguous()
        mask = mask.to(torch.uint8).contiguous()
        return y, mask

    def init(self, y, mask):
        y, mask = self._prep(y, mask)
        self._y, self._mask = y, mask
        _check(_lib.shlr_init(self._h, _ptr(y), _ptr(mask)))

    def set_spirit_kernel(self, g):
        import numpy as np
        g = np.ascontiguousarray(np.asarray(g, dtype=np.complex128))
        _check(_lib.shlr_set_spirit_kernel(self._h, g.ctypes.data_as(ctypes.c_void_p)))

    def calibrate_spirit(self, acs=24, reg=1e-3):
        _check(_lib.shlr_calibrate_spirit(self._h, int(acs), float(reg)))

    def iterate(self, n, graph=False):
        info = CInfo()
        f = _lib.shlr_iterate_graph if graph else _lib.shlr_iterate
        _check(f(self._h, int(n), ctypes.byref(info)))
        return info

    def iterate_async(self, n, graph=False):
        f = _lib.shlr_iterate_graph if graph else _lib.shlr_iterate
        _check(f(self._h, int(n), None))

    def set_weights(self, w_row, w_col=None):
        """Replace W (Eq. 2): w_row / w_col complex tensors (any device) holding the row / column line
        weights of every slice back to back (w_col None for the parameter model).  shlr_init must follow."""
        import torch
        dev = self.ws.device
        wr = torch.as_tensor(w_row).to(device=dev, dtype=torch.complex128).contiguous()
        wc = None if w_col is None else torch.as_tensor(w_col).to(device=dev, dtype=torch.complex128).contiguous()
        _check(_lib.shlr_set_weights(self._h, _ptr(wr), None if wc is None else _ptr(wc)))

    def set_eig_check(self, rel_residual_limit):
        """Residual bound of the eigenpair check (see shlr_set_eig_check)."""
        _check(_lib.shlr_set_eig_check(self._h, float(rel_residual_limit)))

    def unit_status(self):
        """Per stop unit (slice, or FE position of the parameter model): (iterations run, last relative
        change, still active) as numpy arrays."""
        import numpy as np
        n = len(self.params.M) if self.params.model == MODEL_PI else int(self.params.M[0])
        it = np.zeros(n, dtype=np.int32)
        rel = np.zeros(n, dtype=np.float64)
        act = np.zeros(n, dtype=np.int32)
        _check(_lib.shlr_unit_status(self._h, n, it.ctypes.data_as(ctypes.c_void_p),
                                     rel.ctypes.data_as(ctypes.c_void_p), act.ctypes.data_as(ctypes.c_void_p)))
        return it, rel, act.astype(bool)

    def autotune(self, reps=3):
        """Time the launch choices on this plan's shapes and keep the fastest; returns the report.
        The plan must be initialised again afterwards."""
        buf = ctypes.create_string_buffer(1 << 16)
        _check(_lib.shlr_autotune(self._h, int(reps), buf, ctypes.c_size_t(len(buf))))
        return buf.value.decode()

    def timing_enable(self, on=True):
        _check(_lib.shlr_timing_enable(self._h, int(on)))

    def timing_enable_phases(self, phases):
        """Time only the named phases (names of TIMING_PHASES); an empty list stops timing."""
        mask = 0
        for p in phases:
            mask |= 1 << TIMING_PHASES.index(p)
        _check(_lib.shlr_timing_enable_phases(self._h, ctypes.c_uint32(mask)))

    def timing_read(self):
        """Accumulated per-phase device time: {phase: (ms, launches)}."""
        ms = (ctypes.c_double * len(TIMING_PHASES))()
        cnt = (ctypes.c_int32 * len(TIMING_PHASES))()
        _check(_lib.shlr_timing_read(self._h, ms, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(TIMING_PHASES)}

    def kspace(self, out=None):
        import torch
        if out is None:
            out = torch.empty_like(self._y)
        _check(_lib.shlr_get_kspace(self._h, _ptr(out)))
        return out

    def reconstruct(self, y, mask):
        import torch
        y, mask = self._prep(y, mask)
        self._y, self._mask = y, mask
        out = torch.empty_like(y)
        info = CInfo()
        _check(_lib.shlr_reconstruct(self._h, _ptr(y), _ptr(mask), _ptr(out), ctypes.byref(info)))
        return out, info

    # -- reverse mode through unrolled iterations (see shlr_unrolled_* in include/shlr.h) --

    def unrolled_sizes(self, n_iter):
        ck, wk = ctypes.c_size_t(), ctypes.c_size_t()
        _check(_lib.shlr_unrolled_sizes(self._h, int(n_iter), ctypes.byref(ck), ctypes.byref(wk)))
        return ck.value, wk.value

    def unrolled_forward(self, y, mask, n_iter):
        """K after n_iter iterations; keeps the checkpoints for unrolled_backward."""
        import torch
        y, mask = self._prep(y, mask)
        self._y, self._mask = y, mask
        ck, _ = self.unrolled_sizes(n_iter)
        self._ckpt = torch.empty(ck + 256, dtype=torch.uint8, device=y.device)
        off = (-self._ckpt.data_ptr()) % 256
        self._ckpt_ptr = ctypes.c_void_p(self._ckpt.data_ptr() + off)
        self._ckpt_bytes = ck
        out = torch.empty_like(y)
        _check(_lib.shlr_unrolled_forward(self._h, int(n_iter), _ptr(y), _ptr(mask), _ptr(out), self._ckpt_ptr,
                                          ctypes.c_size_t(ck)))
        return out

    def unrolled_backward(self, gk, n_iter):
        """(gY, dL/dlambda) for L = Re <gk, K_n> after unrolled_forward(n_iter)."""
        import torch
        gk = gk.to(self.cdtype).contiguous()
        _, wk = self.unrolled_sizes(n_iter)
        work = torch.empty(wk + 256, dtype=torch.uint8, device=gk.device)
        off = (-work.data_ptr()) % 256
        gy = torch.empty_like(gk)
        gl = ctypes.c_double()
        _check(_lib.shlr_unrolled_backward(self._h, int(n_iter), _ptr(gk), self._ckpt_ptr,
                                           ctypes.c_size_t(self._ckpt_bytes), ctypes.c_void_p(work.data_ptr() + off),
                                           ctypes.c_size_t(wk), _ptr(gy), ctypes.byref(gl)))
        self._ckpt = None
        return gy, gl.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.shlr_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_check(params: Params):
    """Validate params on the host only; returns the workspace size in bytes."""
    c, keep = params.to_c()
    h = ctypes.c_void_p()
    _check(_lib.shlr_plan_create(ctypes.byref(c), ctypes.byref(h)))
    nb = ctypes.c_size_t()
    try:
        _check(_lib.shlr_workspace_size(h, ctypes.byref(nb)))
    finally:
        _lib.shlr_plan_destroy(h)
    return nb.value


def fft_lines(x, inverse=False):
    """Centred unitary DFT of the rows of a contiguous complex tensor (…, n)."""
    import torch
    prec = PREC_MIXED if x.dtype == torch.complex64 else PREC_FP64
    x = x.contiguous()
    out = torch.empty_like(x)
    n = x.shape[-1]
    _check(_lib.shlr_fft_lines(prec, n, x.numel() // max(n, 1), int(inverse), _ptr(x), _ptr(out), _stream()))
    return out


def lowrank_workspace_size(precision, n_mat, J, n, k, use_vc):
    nb = ctypes.c_size_t()
    _check(_lib.shlr_lowrank_workspace_size(precision, n_mat, J, n, k, int(use_vc), ctypes.byref(nb)))
    return nb.value


def lowrank_lines(h, D, k, beta, tau, thr, use_vc=False, use_w=True, ranks=False, r32=False):
    """One Z/D step on a batch of lines (see shlr_lowrank_lines). D is updated in place.

    h: (B, J, n) complex; D: (B, p, q) complex.  Returns b (B, J, n) [and ranks (B,)].
    r32 (complex64 only): the opt-in FP32 Householder reduction (SHLR_PREC_MIXED_R32).
    """
    import torch
    prec = (PREC_MIXED_R32 if r32 else PREC_MIXED) if h.dtype == torch.complex64 else PREC_FP64
    B, J, n = h.shape
    assert D.is_contiguous() and h.is_contiguous()
    nb = lowrank_workspace_size(prec, B, J, n, k, use_vc)
    ws = torch.empty(nb + 256, dtype=torch.uint8, device=h.device)
    off = (-ws.data_ptr()) % 256
    b = torch.empty_like(h)
    rk = torch.zeros(B, dtype=torch.int32, device=h.device) if ranks else None
    _check(_lib.shlr_lowrank_lines(prec, B, J, n, k, int(use_vc), int(use_w), float(beta), float(tau), float(thr),
                                   _ptr(h), _ptr(D), _ptr(b), _ptr(rk) if ranks else None,
                                   ctypes.c_void_p(ws.data_ptr() + off), ctypes.c_size_t(nb), _stream()))
    return (b, rk) if ranks else b


def lowrank_lines_noalloc(h, D, k, beta, tau, thr, use_vc=False, use_w=True, ranks=False, r32=False):
    """lowrank_lines through shlr_lowrank_lines_noalloc (the library's fixed scratch, no workspace)."""
    import torch
    prec = (PREC_MIXED_R32 if r32 else PREC_MIXED) if h.dtype == torch.complex64 else PREC_FP64
    B, J, n = h.shape
    assert D.is_contiguous() and h.is_contiguous()
    b = torch.empty_like(h)
    rk = torch.zeros(B, dtype=torch.int32, device=h.device) if ranks else None
    _check(_lib.shlr_lowrank_lines_noalloc(prec, B, J, n, k, int(use_vc), int(use_w), float(beta), float(tau),
                                           float(thr), _ptr(h), _ptr(D), _ptr(b), _ptr(rk) if ranks else None,
                                           _stream()))
    return (b, rk) if ranks else b


# -- evaluation step (see shlr_ssos / shlr_rlne / shlr_mssim / shlr_t2_fit in include/shlr.h) --

def _real_prec(t):
    import torch
    return PREC_FP64 if t.dtype in (torch.float64, torch.complex128) else PREC_MIXED


def _eval_work(device):
    import torch
    return torch.empty(EVAL_WORK_BYTES // 8, dtype=torch.float64, device=device)


def ssos(k):
    """SSOS images of multi-coil k-space (..., J, M, N) complex -> (..., M, N) real (same precision)."""
    import torch
    k = k.contiguous()
    J, M, N = k.shape[-3:]
    n_img = k.numel() // (J * M * N)
    work = torch.empty_like(k)
    out = torch.empty(k.shape[:-3] + (M, N), dtype=torch.float64 if k.dtype == torch.complex128 else torch.float32,
                      device=k.device)
    _check(_lib.shlr_ssos(_real_prec(k), n_img, J, M, N, _ptr(k), _ptr(work), _ptr(out), _stream()))
    return out


def rlne(ref, rec, roi=None):
    """Eq. S10 between two real device images (optionally over a uint8 ROI)."""
    ref, rec = ref.contiguous(), rec.to(ref.dtype).contiguous()
    w = _eval_work(ref.device)
    v = ctypes.c_double()
    _check(_lib.shlr_rlne(_real_prec(ref), ref.numel(), _ptr(ref), _ptr(rec),
                          None if roi is None else _ptr(roi.contiguous()), _ptr(w), ctypes.byref(v), _stream()))
    return v.value


def mssim(ref, rec, dyn_range=0.0):
    """Eq. S11 between two real M x N device images."""
    ref, rec = ref.contiguous(), rec.to(ref.dtype).contiguous()
    M, N = ref.shape[-2:]
    w = _eval_work(ref.device)
    v = ctypes.c_double()
    _check(_lib.shlr_mssim(_real_prec(ref), M, N, _ptr(ref), _ptr(rec), float(dyn_range), _ptr(w), ctypes.byref(v),
                           _stream()))
    return v.value


def t2_fit(img, te, roi_frac=0.1, t2_min=5.0, t2_max=500.0):
    """T2 map of echo images img (L, ...) real on the device: returns (t2, rho, roi) tensors."""
    import numpy as np
    import torch
    img = img.contiguous()
    L = img.shape[0]
    npix = img.numel() // L
    te = np.ascontiguousarray(np.asarray(te, dtype=np.float64))
    t2 = torch.empty(img.shape[1:], dtype=img.dtype, device=img.device)
    rho = torch.empty_like(t2)
    roi = torch.empty(img.shape[1:], dtype=torch.uint8, device=img.device)
    w = _eval_work(img.device)
    _check(_lib.shlr_t2_fit(_real_prec(img), L, npix, te.ctypes.data_as(ctypes.c_void_p), _ptr(img),
                            float(roi_frac), float(t2_min), float(t2_max), _ptr(t2), _ptr(rho), _ptr(roi), _ptr(w),
                            _stream()))
    return t2, rho, roi


def _unrolled_function():
    import torch

    class UnrolledSHLR(torch.autograd.Function):
        """K_n = n_iter SHLR iterations of (Y, lambda); backward through the library's reverse mode."""

        @staticmethod
        def forward(ctx, y, lam, mask, n_iter, params):
            import dataclasses
            prm = dataclasses.replace(params, lam=float(lam), normalize=False)
            plan = Plan(prm, device=y.device)
            k = plan.unrolled_forward(y.detach(), mask, n_iter)
            ctx.plan, ctx.n_iter = plan, n_iter
            return k

        @staticmethod
        def backward(ctx, gk):
            gy, gl = ctx.plan.unrolled_backward(gk, ctx.n_iter)
            ctx.plan.close()
            ctx.plan = None
            return gy, torch.tensor(gl, dtype=torch.float64), None, None, None

    return UnrolledSHLR


_UNROLLED = None


def unrolled(y, lam, mask, n_iter, params: Params):
    """Differentiable K_n of n_iter iterations (model PI, soft data consistency, no SPIRiT).

    y: complex tensor in the layout of Y (slices packed); lam: real 0-dim tensor (data-consistency
    weight); the other fields of ``params`` are fixed.  Y is used as given (no normalisation).
    """
    global _UNROLLED
    if _UNROLLED is None:
        _UNROLLED = _unrolled_function()
    return _UNROLLED.apply(y, lam, mask, int(n_iter), params)
