"""CPU oracle for the FMM-based NUFFT / INUFFT (test infrastructure).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It is independent of the GPU library:
it shares no source, table or constant with it, and computes every result
by direct summation of the paper's closed forms (oracle.c), plus numpy's FFT
as a library step for the spectral cross-check of Eq. (p1).

Functions (all arrays numpy; complex arrays are complex128):
  grid_units(N, y)            -> (m, theta): N y / 2 pi = m + theta, exact reduction
  fwd(N, y, f)                -> g, Eq. (p2) via its closed form (p4)-(p5)
  fwd_at(N, y, f, sel)        -> g[sel]
  adj(N, y, g, ks=None)       -> f_k = sum_j conj(K_jk) g_j (adjoint of Eq. p2), at ks
  kmatrix(N, y)               -> the M x N matrix K of Eq. (p2), closed form per entry
  lsq(N, y, g)                -> argmin ||K f - g||_2 (dense K, LAPACK least squares)
  fwd_spectral(N, y, f)       -> g, Eq. (p1): c = DFT(f)/N, g_j = sum_n c_n e^{i n y_j}
  eval_series(N, y, c)        -> g, Eq. (p1) from given coefficients
  logsums(N, y, ks, js)       -> (logC, negC, logD, negD) behind Eq. (p8)
  coeffs_at(N, y, ks, js)     -> (Chat[ks], Dhat[js]) of Eq. (p8), rescaled by 2^N
  inv(N, y, g)                -> f, Eq. (p6)/(p8) Lagrange form (M = N)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> None:
    """Compile oracle.c into liboracle.so (gcc, OpenMP, binary128 via libquadmath)."""
    subprocess.run(["sh", os.path.join(_HERE, "build.sh")], check=True)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    i64, dp, ip, vp = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), \
        ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p
    lib.or_grid_units.argtypes = [i64, i64, vp, vp, vp]
    lib.or_fwd_kernel.argtypes = [i64, i64, vp, vp, vp, ctypes.c_int]
    lib.or_fwd_kernel_at.argtypes = [i64, i64, vp, vp, i64, vp, vp, ctypes.c_int]
    lib.or_adj_at.argtypes = [i64, i64, vp, vp, i64, vp, vp, ctypes.c_int]
    lib.or_kmatrix.argtypes = [i64, i64, vp, vp, ctypes.c_int]
    lib.or_eval_series.argtypes = [i64, i64, vp, vp, vp, ctypes.c_int]
    lib.or_logsums_at.argtypes = [i64, vp, i64, vp, vp, vp, i64, vp, vp, vp,
                                  ctypes.c_int]
    lib.or_coeffs_at.argtypes = [i64, vp, i64, vp, vp, i64, vp, vp, ctypes.c_int]
    lib.or_inv.argtypes = [i64, vp, vp, vp, ctypes.c_int]
    lib.or_inv.restype = ctypes.c_int
    lib.or_max_threads.argtypes = [ctypes.c_int]
    lib.or_max_threads.restype = ctypes.c_int
    del dp, ip
    _lib = lib
    return lib


def _threads() -> int:
    return int(os.environ.get("ORACLE_THREADS", "0"))


def threads() -> int:
    """Threads the oracle's parallel loops use."""
    return int(_load().or_max_threads(_threads()))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def grid_units(N: int, y):
    """(m, theta) with N y_j / (2 pi) = m_j + theta_j (mod N), m_j in [0, N),
    theta_j in [-1/2, 1/2]; the product is formed in binary128."""
    y = _f64(y)
    m = np.empty(y.shape[0], dtype=np.int64)
    th = np.empty(y.shape[0], dtype=np.float64)
    _load().or_grid_units(N, y.shape[0], _ptr(y), _ptr(m), _ptr(th))
    return m, th


def fwd(N: int, y, f):
    """g_j = sum_k K_jk f_k, K of Eq. (p2) through the closed form (p4)-(p5)."""
    y, f = _f64(y), _c128(f)
    assert f.shape[0] == N
    g = np.empty(y.shape[0], dtype=np.complex128)
    _load().or_fwd_kernel(N, y.shape[0], _ptr(y), _ptr(f), _ptr(g), _threads())
    return g


def fwd_at(N: int, y, f, sel):
    """fwd(N, y, f)[sel] computed for the selected targets only."""
    y, f = _f64(y), _c128(f)
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    assert f.shape[0] == N and (sel.size == 0 or (sel.min() >= 0 and sel.max() < y.shape[0]))
    g = np.empty(sel.shape[0], dtype=np.complex128)
    _load().or_fwd_kernel_at(N, y.shape[0], _ptr(y), _ptr(f), sel.shape[0],
                             _ptr(sel), _ptr(g), _threads())
    return g


def adj(N: int, y, g, ks=None):
    """f_k = sum_j conj(K_jk) g_j (the adjoint of Eq. p2, K in its closed
    form p4-p5) for k in ks (default: k = 0..N-1)."""
    y, g = _f64(y), _c128(g)
    assert g.shape[0] == y.shape[0]
    ks_a = None if ks is None else np.ascontiguousarray(ks, dtype=np.int64)
    nk = N if ks_a is None else ks_a.shape[0]
    f = np.empty(nk, dtype=np.complex128)
    _load().or_adj_at(N, y.shape[0], _ptr(y), _ptr(g), nk,
                      None if ks_a is None else _ptr(ks_a), _ptr(f), _threads())
    return f


def kmatrix(N: int, y):
    """The M x N matrix K of Eq. (p2), every entry in the closed form
    (p4)-(p5) (a Kronecker delta row for a point on the grid)."""
    y = _f64(y)
    K = np.empty((y.shape[0], N), dtype=np.complex128)
    _load().or_kmatrix(N, y.shape[0], _ptr(y), _ptr(K), _threads())
    return K


def lsq(N: int, y, g):
    """argmin_f ||K f - g||_2 with the dense K of Eq. (p2) (numpy's LAPACK
    least squares, a library step; the minimum-norm solution when K has
    deficient rank).  For small N only."""
    return np.linalg.lstsq(kmatrix(N, y), _c128(g), rcond=None)[0]


def eval_series(N: int, y, c):
    """g_j = sum_{n=0}^{N-1} c_n e^{i n y_j} (Eq. p1), term by term."""
    y, c = _f64(y), _c128(c)
    assert c.shape[0] == N
    g = np.empty(y.shape[0], dtype=np.complex128)
    _load().or_eval_series(N, y.shape[0], _ptr(y), _ptr(c), _ptr(g), _threads())
    return g


def fwd_spectral(N: int, y, f):
    """Eq. (p1) route: c_n = (1/N) sum_k f_k e^{-i n x_k} by FFT, then the series."""
    f = _c128(f)
    return eval_series(N, y, np.fft.fft(f) / N)


def logsums(N: int, y, ks=None, js=None):
    """Log-sums behind Eq. (p8) (rescaled by 2^N):
    logC[k] = sum_j log|2 sin((x_k - y_j)/2)|, negC[k] = #{j: s'_j > k};
    logD[j] = -sum_{i!=j} log|2 sin((y_j - y_i)/2)|, negD[j] = #{i: s'_i > s'_j}.
    ks / js select the entries (default: all)."""
    y = _f64(y)
    assert y.shape[0] == N
    ks_a = None if ks is None else np.ascontiguousarray(ks, dtype=np.int64)
    js_a = None if js is None else np.ascontiguousarray(js, dtype=np.int64)
    nk = N if ks_a is None else ks_a.shape[0]
    nj = N if js_a is None else js_a.shape[0]
    logC = np.empty(nk)
    logD = np.empty(nj)
    negC = np.empty(nk, dtype=np.int64)
    negD = np.empty(nj, dtype=np.int64)
    _load().or_logsums_at(N, _ptr(y), nk, None if ks_a is None else _ptr(ks_a),
                          _ptr(logC), _ptr(negC), nj,
                          None if js_a is None else _ptr(js_a), _ptr(logD),
                          _ptr(negD), _threads())
    return logC, negC, logD, negD


def coeffs_at(N: int, y, ks, js):
    """Chat_k = (-1)^(k + #{j: s_j > k}) prod_j |2 sin((x_k - y_j)/2)| and
    Dhat_j = i e^{-i N y_j / 2} / prod_{i != j} 2 sin((y_j - y_i)/2) (Eq. p8,
    rescaled by 2^N and 2^-N) at the selected k and j, each from O(N) direct
    log-sums."""
    y = _f64(y)
    assert y.shape[0] == N
    ks_a = np.ascontiguousarray(ks, dtype=np.int64)
    js_a = np.ascontiguousarray(js, dtype=np.int64)
    chat = np.empty(ks_a.shape[0])
    dhat = np.empty(js_a.shape[0], dtype=np.complex128)
    _load().or_coeffs_at(N, _ptr(y), ks_a.shape[0], _ptr(ks_a), _ptr(chat),
                         js_a.shape[0], _ptr(js_a), _ptr(dhat), _threads())
    return chat, dhat


class OracleError(RuntimeError):
    pass


def inv(N: int, y, g):
    """f = L g, Eq. (p6) with C_k, D_j of Eq. (p8) (M = N)."""
    y, g = _f64(y), _c128(g)
    assert y.shape[0] == N and g.shape[0] == N
    f = np.empty(N, dtype=np.complex128)
    st = _load().or_inv(N, _ptr(y), _ptr(g), _ptr(f), _threads())
    if st == 4:
        raise OracleError("two points coincide: the interpolation problem is singular")
    if st == 5:
        raise OracleError("a coefficient of Eq. (p8) leaves the binary64 range")
    return f
