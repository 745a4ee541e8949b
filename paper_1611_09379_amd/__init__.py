"""MI355X (gfx950) FMM-based NUFFT / INUFFT of Gumerov & Duraiswami.

Thin ctypes binding over libfmmnufft.so (C ABI in include/fmmnufft.h).  It
only marshals arguments: every step of the transforms runs in the library's
HIP kernels.  Tensors are PyTorch CUDA tensors (ROCm): y float64, data
complex128 (plain FP64 path) or complex64 (mixed path).  If the library is
missing, importing the binding's functions raises: there is no fallback.

    g = nufft_fwd(y, f, eps)        # forward, Eq. (p2): g_j = f(y_j)
    f = inufft(y, g, eps)           # inverse, Eq. (p6), M = N
    f = nufft_adj(y, g, N, eps)     # adjoint of Eq. (p2): f = K^H g
    plan = Plan.forward(N, y, eps)  # setup once per point set (Section 3.3)
    g = plan(f)                     # evaluation, repeated per input
    gs = nufft_fwd_batched(ys, fs, eps)   # many forward transforms at once
    batch = Batch.forward(ys, Ns, eps)    # batch setup; batch(fs) evaluates
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfmmnufft.so")

FN_OK, FN_EINVAL, FN_ENOMEM, FN_EHIP, FN_ESINGULAR, FN_ERANGE, FN_EPREC = range(7)
FN_C128, FN_C64 = 0, 1
FN_EPS_MACHINE = 0.0   # eps that requests the path's precision floor eps_th(N)
STATUS_NAMES = {0: "FN_OK", 1: "FN_EINVAL", 2: "FN_ENOMEM", 3: "FN_EHIP",
                4: "FN_ESINGULAR", 5: "FN_ERANGE", 6: "FN_EPREC"}

ABI_SYMBOLS = (
    "nufft_fwd", "inufft", "nufft_adj", "nufft_spec_fwd", "inufft_spec",
    "nufft_plan_fwd", "nufft_plan_inv", "nufft_plan_adj", "nufft_plan_spec_fwd",
    "nufft_plan_spec_inv", "nufft_plan_fwd_ex", "nufft_plan_inv_ex",
    "nufft_plan_adj_ex", "nufft_execute",
    "nufft_execute_phase",
    "nufft_destroy", "nufft_plan_get_info", "nufft_plan_coeffs",
    "nufft_select_params",
    "nufft_fwd_batched", "nufft_plan_fwd_batched", "nufft_execute_batched",
    "nufft_destroy_batched", "nufft_autotune", "nufft_autotune_clear", "nufft_autotune_save", "nufft_autotune_load",
    "nufft_set_timing", "nufft_plan_get_timings",
    "nufft_lsq", "nufft_fwd_noalloc", "nufft_release_cache", "nufft_last_error",
)


class NufftError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class PlanInfo(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("M", ctypes.c_int64),
                ("kind", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("p", ctypes.c_int32), ("q", ctypes.c_int32),
                ("lmax", ctypes.c_int32), ("nterms", ctypes.c_int32),
                ("eps", ctypes.c_double), ("mterms", ctypes.c_int32),
                ("log_nterms", ctypes.c_int32), ("log_mterms", ctypes.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads libfmmnufft.so and declares the C signatures.  Raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it first "
            "(python -m paper_1611_09379_amd.build); there is no fallback path")
    # PyTorch ships its own HIP runtime under the same soname: import it
    # first, so that the library binds to the runtime that owns the tensors
    # and streams (loaded the other way round, the two stacks mix and the
    # runtime finds no device)
    _torch()
    lib = ctypes.CDLL(path)
    i64, i32, dbl, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
    pp = ctypes.POINTER(ctypes.c_void_p)
    pi32 = ctypes.POINTER(ctypes.c_int32)
    sig = {
        "nufft_fwd": [i64, i64, vp, vp, vp, dbl, ctypes.c_int, vp],
        "inufft": [i64, vp, vp, vp, dbl, ctypes.c_int, vp],
        "nufft_adj": [i64, i64, vp, vp, vp, dbl, ctypes.c_int, vp],
        "nufft_spec_fwd": [i64, i64, vp, vp, vp, dbl, ctypes.c_int, vp],
        "inufft_spec": [i64, vp, vp, vp, dbl, ctypes.c_int, vp],
        "nufft_plan_spec_fwd": [pp, i64, i64, vp, dbl, ctypes.c_int, vp],
        "nufft_plan_spec_inv": [pp, i64, vp, dbl, ctypes.c_int, vp],
        "nufft_plan_adj": [pp, i64, i64, vp, dbl, ctypes.c_int, vp],
        "nufft_plan_adj_ex": [pp, i64, i64, vp, dbl, ctypes.c_int, i32, i32, i32, vp],
        "nufft_plan_fwd": [pp, i64, i64, vp, dbl, ctypes.c_int, vp],
        "nufft_plan_inv": [pp, i64, vp, dbl, ctypes.c_int, vp],
        "nufft_plan_fwd_ex": [pp, i64, i64, vp, dbl, ctypes.c_int, i32, i32, i32, vp],
        "nufft_plan_inv_ex": [pp, i64, vp, dbl, ctypes.c_int, i32, i32, i32, vp],
        "nufft_execute": [vp, vp, vp, vp],
        "nufft_execute_phase": [vp, vp, vp, ctypes.c_int, vp],
        "nufft_destroy": [vp],
        "nufft_plan_get_info": [vp, ctypes.POINTER(PlanInfo)],
        "nufft_plan_coeffs": [vp, vp, vp, vp],
        "nufft_select_params": [i64, i64, dbl, ctypes.c_int, pi32, pi32, pi32],
        "nufft_fwd_batched": [i32, vp, vp, vp, vp, vp, dbl, ctypes.c_int, vp],
        "nufft_plan_fwd_batched": [pp, i32, vp, vp, vp, dbl, ctypes.c_int, vp],
        "nufft_execute_batched": [vp, vp, vp, vp],
        "nufft_destroy_batched": [vp],
        "nufft_autotune": [ctypes.c_int, i64, i64, dbl, ctypes.c_int, pi32, pi32, vp],
        "nufft_autotune_clear": [],
        "nufft_autotune_save": [ctypes.c_char_p],
        "nufft_autotune_load": [ctypes.c_char_p],
        "nufft_set_timing": [ctypes.c_int],
        "nufft_plan_get_timings": [vp, ctypes.POINTER(ctypes.c_float), pi32],
        "nufft_fwd_noalloc": [i64, i64, vp, vp, vp, dbl, ctypes.c_int, vp],
        "nufft_lsq": [i64, i64, vp, vp, vp, dbl, dbl, i32, ctypes.c_int, pi32,
                      ctypes.POINTER(ctypes.c_double), vp],
        "nufft_release_cache": [],
        "nufft_last_error": [],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name == "nufft_last_error" else ctypes.c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != FN_OK:
        msg = load_library().nufft_last_error().decode(errors="replace")
        raise NufftError(status, msg)


def _torch():
    import torch
    return torch


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.complex128:
        return FN_C128
    if t.dtype == torch.complex64:
        return FN_C64
    raise TypeError(f"data must be complex128 or complex64, got {t.dtype}")


def _dev_ptr(t, name):
    if not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _check_y(y):
    torch = _torch()
    if y.dtype != torch.float64 or y.dim() != 1:
        raise TypeError("y must be a 1-D float64 tensor (radians)")


def select_params(N: int, M: int, eps: float, dtype: int = FN_C128):
    """(p, q, lmax) the library chooses: Eq. (18.2) and Eq. (25)."""
    p, q, l = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(load_library().nufft_select_params(N, M, eps, dtype, ctypes.byref(p),
                                              ctypes.byref(q), ctypes.byref(l)))
    return p.value, q.value, l.value


class Plan:
    """A plan: the setup step (points only) of Section 3.3."""

    def __init__(self, handle, kind: int, N: int, M: int, dtype: int):
        self._h = handle
        self.kind, self.N, self.M, self.dtype = kind, N, M, dtype

    @classmethod
    def forward(cls, N: int, y, eps: float, dtype: int = FN_C128,
                p: int = 0, q: int = 0, lmax: int = 0):
        _check_y(y)
        h = ctypes.c_void_p()
        _check(load_library().nufft_plan_fwd_ex(
            ctypes.byref(h), N, y.shape[0], _dev_ptr(y, "y"), eps, dtype,
            p, q, lmax, _stream()))
        return cls(h, 0, N, y.shape[0], dtype)

    @classmethod
    def inverse(cls, y, eps: float, dtype: int = FN_C128, p: int = 0,
                q: int = 0, lmax: int = 0):
        _check_y(y)
        h = ctypes.c_void_p()
        N = y.shape[0]
        _check(load_library().nufft_plan_inv_ex(
            ctypes.byref(h), N, _dev_ptr(y, "y"), eps, dtype, p, q, lmax,
            _stream()))
        return cls(h, 1, N, N, dtype)

    @classmethod
    def adjoint(cls, N: int, y, eps: float, dtype: int = FN_C128, p: int = 0,
                q: int = 0, lmax: int = 0):
        """Adjoint plan: f = K^H g (M points y -> N grid values)."""
        _check_y(y)
        h = ctypes.c_void_p()
        _check(load_library().nufft_plan_adj_ex(
            ctypes.byref(h), N, y.shape[0], _dev_ptr(y, "y"), eps, dtype, p, q, lmax,
            _stream()))
        return cls(h, 2, N, y.shape[0], dtype)

    @classmethod
    def spectral_forward(cls, N: int, y, eps: float, dtype: int = FN_C128):
        """Spectral forward plan: coefficients c (N) -> values g_j = f(y_j)
        (Eq. p1), the uniform DFT by rocFFT, then the forward FMM."""
        _check_y(y)
        h = ctypes.c_void_p()
        _check(load_library().nufft_plan_spec_fwd(
            ctypes.byref(h), N, y.shape[0], _dev_ptr(y, "y"), eps, dtype, _stream()))
        return cls(h, 0, N, y.shape[0], dtype)

    @classmethod
    def spectral_inverse(cls, y, eps: float, dtype: int = FN_C128):
        """Spectral inverse plan (M = N): values g_j -> coefficients c."""
        _check_y(y)
        h = ctypes.c_void_p()
        N = y.shape[0]
        _check(load_library().nufft_plan_spec_inv(
            ctypes.byref(h), N, _dev_ptr(y, "y"), eps, dtype, _stream()))
        return cls(h, 1, N, N, dtype)

    def info(self) -> PlanInfo:
        out = PlanInfo()
        _check(load_library().nufft_plan_get_info(self._h, ctypes.byref(out)))
        return out

    def timings(self):
        """Plans created with timing on (set_timing): milliseconds of the sort
        and (inverse plans) of the log-sum FMM's upward pass, translations and
        evaluation, and its expansion length; -1 entries when not recorded."""
        ms = (ctypes.c_float * 4)()
        terms = ctypes.c_int32()
        _check(load_library().nufft_plan_get_timings(self._h, ms, ctypes.byref(terms)))
        return {"log_up_ms": ms[0], "log_trans_ms": ms[1], "log_eval_ms": ms[2],
                "sort_ms": ms[3], "log_terms": terms.value}

    def coeffs(self):
        """Inverse plans: (Chat, Dhat) of Eq. (p8), rescaled by 2^N and 2^-N
        (Dhat in the order of y), as complex128/float64 GPU tensors."""
        torch = _torch()
        chat = torch.empty(self.N, dtype=torch.float64, device="cuda")
        dhat = torch.empty(self.N, dtype=torch.complex128, device="cuda")
        _check(load_library().nufft_plan_coeffs(self._h, _dev_ptr(chat, "chat"),
                                                _dev_ptr(dhat, "dhat"), _stream()))
        return chat, dhat

    def execute(self, x, out=None):
        torch = _torch()
        if self._h is None:
            raise RuntimeError("plan was destroyed")
        if _dtype_code(x) != self.dtype:
            raise TypeError("input dtype does not match the plan")
        n_in = self.M if self.kind == 2 else self.N
        n_out = self.M if self.kind == 0 else self.N
        if x.shape != (n_in,):
            raise ValueError(f"input must have shape ({n_in},)")
        if out is None:
            out = torch.empty(n_out, dtype=x.dtype, device=x.device)
        elif out.shape != (n_out,) or out.dtype != x.dtype:
            raise ValueError("bad output tensor")
        _check(load_library().nufft_execute(self._h, _dev_ptr(x, "input"),
                                            _dev_ptr(out, "output"), _stream()))
        return out

    __call__ = execute

    def execute_phase(self, x, out, phase: int):
        """One part of execute (0: upward pass, 1: downward translations,
        2: evaluation); the three must be enqueued in order with the same x."""
        _check(load_library().nufft_execute_phase(
            self._h, _dev_ptr(x, "input"), _dev_ptr(out, "output"), phase,
            _stream()))
        return out

    def destroy(self):
        if self._h is not None:
            _check(load_library().nufft_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def nufft_fwd(y, f, eps: float, out=None):
    """g_j = sum_k K_jk f_k (Eq. p2) at the points y (radians), one shot."""
    torch = _torch()
    _check_y(y)
    dt = _dtype_code(f)
    N, M = f.shape[0], y.shape[0]
    if out is None:
        out = torch.empty(M, dtype=f.dtype, device=f.device)
    _check(load_library().nufft_fwd(N, M, _dev_ptr(y, "y"), _dev_ptr(f, "f"),
                                    _dev_ptr(out, "g"), eps, dt, _stream()))
    return out


def inufft(y, g, eps: float, out=None):
    """f = L g (Eq. p6), M = N, one shot."""
    torch = _torch()
    _check_y(y)
    dt = _dtype_code(g)
    N = y.shape[0]
    if g.shape != (N,):
        raise ValueError("g must have the shape of y (M = N)")
    if out is None:
        out = torch.empty(N, dtype=g.dtype, device=g.device)
    _check(load_library().inufft(N, _dev_ptr(y, "y"), _dev_ptr(g, "g"),
                                 _dev_ptr(out, "f"), eps, dt, _stream()))
    return out


def nufft_spec_fwd(y, c, eps: float, out=None):
    """g_j = sum_n c_n e^{i n y_j} (Eq. p1) from the coefficients c, one shot
    (rocFFT for the uniform DFT, then the forward FMM)."""
    torch = _torch()
    _check_y(y)
    dt = _dtype_code(c)
    N, M = c.shape[0], y.shape[0]
    if out is None:
        out = torch.empty(M, dtype=c.dtype, device=c.device)
    _check(load_library().nufft_spec_fwd(N, M, _dev_ptr(y, "y"), _dev_ptr(c, "c"),
                                         _dev_ptr(out, "g"), eps, dt, _stream()))
    return out


def inufft_spec(y, g, eps: float, out=None):
    """The coefficients c of the band-limited interpolant through the values
    g_j at the points y (M = N), one shot (inverse FMM, then rocFFT)."""
    torch = _torch()
    _check_y(y)
    dt = _dtype_code(g)
    N = y.shape[0]
    if g.shape != (N,):
        raise ValueError("g must have the shape of y (M = N)")
    if out is None:
        out = torch.empty(N, dtype=g.dtype, device=g.device)
    _check(load_library().inufft_spec(N, _dev_ptr(y, "y"), _dev_ptr(g, "g"),
                                      _dev_ptr(out, "c"), eps, dt, _stream()))
    return out


def nufft_adj(y, g, N: int, eps: float, out=None):
    """f_k = sum_j conj(K_jk) g_j (the adjoint of Eq. p2), k = 0..N-1, one
    shot."""
    torch = _torch()
    _check_y(y)
    dt = _dtype_code(g)
    M = y.shape[0]
    if g.shape != (M,):
        raise ValueError("g must have the shape of y")
    if out is None:
        out = torch.empty(N, dtype=g.dtype, device=g.device)
    _check(load_library().nufft_adj(N, M, _dev_ptr(y, "y"), _dev_ptr(g, "g"),
                                    _dev_ptr(out, "f"), eps, dt, _stream()))
    return out


def nufft_lsq(y, g, N: int, eps: float, tol: float = 1e-12, maxiter: int = 100, out=None):
    """f = argmin ||K f - g|| (K of Eq. p2, M = len(y) points) by conjugate
    gradients on the normal equations, each step a forward and an adjoint
    transform.  Returns (f, iterations, relative normal-equation residual)."""
    torch = _torch()
    _check_y(y)
    dt = _dtype_code(g)
    M = y.shape[0]
    if g.shape != (M,):
        raise ValueError("g must have the shape of y")
    if out is None:
        out = torch.empty(N, dtype=g.dtype, device=g.device)
    it = ctypes.c_int32()
    res = ctypes.c_double()
    _check(load_library().nufft_lsq(N, M, _dev_ptr(y, "y"), _dev_ptr(g, "g"),
                                    _dev_ptr(out, "f"), eps, tol, maxiter, dt,
                                    ctypes.byref(it), ctypes.byref(res), _stream()))
    return out, it.value, res.value


def _ptr_array(ts, name):
    arr = (ctypes.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = _dev_ptr(t, f"{name}[{i}]").value
    return arr


def _sizes(vals):
    arr = (ctypes.c_int64 * len(vals))()
    for i, v in enumerate(vals):
        arr[i] = int(v)
    return arr


def nufft_fwd_batched(ys, fs, eps: float, outs=None):
    """g_t = K_t f_t for every t (Eq. p2), one shot over a batch: ys and fs
    are sequences of tensors (one transform each, same dtype)."""
    torch = _torch()
    if len(ys) != len(fs) or not ys:
        raise ValueError("ys and fs must be non-empty and of equal length")
    for y in ys:
        _check_y(y)
    dt = _dtype_code(fs[0])
    if any(_dtype_code(f) != dt for f in fs):
        raise TypeError("every f must have the same dtype")
    if outs is None:
        outs = [torch.empty(y.shape[0], dtype=fs[0].dtype, device=fs[0].device) for y in ys]
    Ns = _sizes([f.shape[0] for f in fs])
    Ms = _sizes([y.shape[0] for y in ys])
    _check(load_library().nufft_fwd_batched(
        len(ys), Ns, Ms, _ptr_array(ys, "y"), _ptr_array(fs, "f"),
        _ptr_array(outs, "g"), eps, dt, _stream()))
    return outs


class Batch:
    """Setup of a batch of forward transforms, evaluated repeatedly
    (nufft_plan_fwd_batched / nufft_execute_batched)."""

    def __init__(self, handle, Ns, Ms, dtype):
        self._h = handle
        self.Ns, self.Ms, self.dtype = list(Ns), list(Ms), dtype

    @classmethod
    def forward(cls, ys, Ns, eps: float, dtype: int = FN_C128):
        for y in ys:
            _check_y(y)
        if len(ys) != len(Ns) or not ys:
            raise ValueError("ys and Ns must be non-empty and of equal length")
        h = ctypes.c_void_p()
        Ms = [y.shape[0] for y in ys]
        _check(load_library().nufft_plan_fwd_batched(
            ctypes.byref(h), len(ys), _sizes(Ns), _sizes(Ms), _ptr_array(ys, "y"),
            eps, dtype, _stream()))
        return cls(h, Ns, Ms, dtype)

    def execute(self, fs, outs=None):
        torch = _torch()
        if self._h is None:
            raise RuntimeError("batch was destroyed")
        if len(fs) != len(self.Ns):
            raise ValueError("one input per transform")
        for f, n in zip(fs, self.Ns):
            if _dtype_code(f) != self.dtype or f.shape != (n,):
                raise ValueError("input dtype or shape does not match the batch")
        if outs is None:
            outs = [torch.empty(m, dtype=fs[0].dtype, device=fs[0].device) for m in self.Ms]
        _check(load_library().nufft_execute_batched(
            self._h, _ptr_array(fs, "f"), _ptr_array(outs, "g"), _stream()))
        return outs

    __call__ = execute

    def destroy(self):
        if self._h is not None:
            _check(load_library().nufft_destroy_batched(self._h))
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def autotune(kind: str, N: int, M: int, eps: float, dtype: int = FN_C128):
    """Runs the library's autotuner for forward ("fwd"), inverse ("inv") or
    adjoint ("adj") transforms of sizes N, M; later plans of that size class use its
    choice.  Returns (lmax, nterms) (nterms 0: default length kept)."""
    l = ctypes.c_int32()
    p = ctypes.c_int32()
    _check(load_library().nufft_autotune({"fwd": 0, "inv": 1, "adj": 2}[kind], N, M, eps, dtype,
                                         ctypes.byref(l), ctypes.byref(p), _stream()))
    return l.value, p.value


def autotune_clear():
    """Forgets every choice recorded by autotune."""
    _check(load_library().nufft_autotune_clear())


def autotune_save(path: str):
    """Writes the recorded autotune choices to a text file."""
    _check(load_library().nufft_autotune_save(os.fsencode(path)))


def autotune_load(path: str):
    """Adds the autotune choices of a file written by autotune_save."""
    _check(load_library().nufft_autotune_load(os.fsencode(path)))


def set_timing(on: bool):
    """Process-wide: inverse plans created while on record event timings of
    their log-sum FMM (Plan.timings)."""
    _check(load_library().nufft_set_timing(1 if on else 0))


def release_cache():
    """Frees the device blocks the library keeps cached for later plans."""
    _check(load_library().nufft_release_cache())
