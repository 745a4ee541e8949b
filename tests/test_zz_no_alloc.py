"""The allocation-free forward call (nufft_fwd_noalloc) through the C ABI:
the same result as nufft_fwd on two calls in a row (the second smaller, so
the static scratch region holds the first call's contents), within the
oracle's tolerance; sizes beyond the region are rejected."""
import ctypes

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import dev, host, rel_l2, say

pytestmark = pytest.mark.gpu

fn = pytest.importorskip("paper_1611_09379_amd")


def noalloc(N, y, f, eps):
    import torch
    lib = fn.load_library()
    g = torch.empty(y.shape[0], dtype=f.dtype, device="cuda")
    dt = fn.FN_C128 if f.dtype == torch.complex128 else fn.FN_C64
    st = lib.nufft_fwd_noalloc(N, y.shape[0], ctypes.c_void_p(y.data_ptr()),
                               ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                               eps, dt, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, g


@pytest.mark.parametrize("dtype,eps", [(np.complex128, 1e-12), (np.complex64, 1e-6)])
def test_noalloc_matches_nufft_fwd(dtype, eps):
    for N, M, seed in ((1 << 20, 1 << 20, 1), (5000, 3001, 2)):
        say(f"noalloc N={N} M={M} {np.dtype(dtype).name}")
        y, f, c = workloads.forward_case(N, M, "uniform", seed=seed)
        f = f.astype(dtype)
        yd, fd = dev(y), dev(f)
        st, g = noalloc(N, yd, fd, eps)
        assert st == fn.FN_OK, fn.load_library().nufft_last_error()
        g = host(g)
        ref = host(fn.nufft_fwd(yd, fd, eps))
        err = rel_l2(g, ref)
        say(f"  vs nufft_fwd {err:.3e} (bitwise equal: {np.array_equal(g, ref)})")
        assert err < eps
        sel = np.random.default_rng(seed).choice(M, min(M, 512), replace=False)
        o = oracle.fwd_at(N, y, f.astype(np.complex128), sel)
        assert rel_l2(g[sel], o) < eps


def test_noalloc_rejects_beyond_scratch():
    N = M = 1 << 22
    y, f, c = workloads.forward_case(N, M, "uniform", seed=3)
    st, g = noalloc(N, dev(y), dev(f), 1e-12)
    assert st == fn.FN_EINVAL
    assert b"static scratch" in fn.load_library().nufft_last_error()
    # still usable afterwards
    y, f, c = workloads.forward_case(256, 100, "uniform", seed=4)
    st, g = noalloc(256, dev(y), dev(f), 1e-12)
    assert st == fn.FN_OK
    assert rel_l2(host(g), oracle.fwd(256, y, f)) < 1e-12
