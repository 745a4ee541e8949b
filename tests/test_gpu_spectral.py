"""Spectral transforms (Eq. p1, f(x) = sum_n c_n e^{inx}) with rocFFT for the
uniform DFT: the forward g_j = f(y_j) from the coefficients against the
oracle's term-by-term series, and the inverse (M = N) coefficients against
the oracle's Lagrange-form inverse followed by numpy's FFT (a library step),
and against the coefficients that generated the values.  Tolerances: 1e-12
(binary64), 1e-6 (mixed, against the oracle on the same rounded input)."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import dev, host, rel_l2, say

pytestmark = pytest.mark.gpu

fn = pytest.importorskip("paper_1611_09379_amd")

PATHS = [(np.complex128, 1e-12), (np.complex64, 1e-6)]


@pytest.mark.parametrize("dtype,eps", PATHS)
@pytest.mark.parametrize("N,M,dist", [(1, 3, "uniform"), (7, 40, "uniform"),
                                      (1000, 1777, "clustered"), (4096, 4096, "uniform"),
                                      (8192, 3000, "uniform"), (6000, 9000, "clustered")])
def test_spectral_forward_full(N, M, dist, dtype, eps):
    y, f, c = workloads.forward_case(N, M, dist, seed=N + M)
    c = c.astype(dtype)
    say(f"spec fwd N={N} M={M} {dist} {np.dtype(dtype).name}")
    g = host(fn.nufft_spec_fwd(dev(y), dev(c), eps))
    ref = oracle.eval_series(N, y, c.astype(np.complex128))
    err = rel_l2(g, ref)
    say(f"  rel l2 {err:.3e}")
    assert err < eps


@pytest.mark.parametrize("dtype,eps", PATHS)
@pytest.mark.parametrize("N,amp", [(64, 0.3), (1000, 0.4), (4096, 0.4), (8191, 0.2)])
def test_spectral_inverse_full(N, amp, dtype, eps):
    y, c = workloads.inverse_case(N, amp, seed=N)
    g = oracle.eval_series(N, y, c)            # values of the interpolant
    gx = g.astype(dtype)
    say(f"spec inv N={N} amp={amp} {np.dtype(dtype).name}")
    cg = host(fn.inufft_spec(dev(y), dev(gx), eps))
    ref = np.fft.fft(oracle.inv(N, y, gx.astype(np.complex128))) / N
    err = rel_l2(cg, ref)
    say(f"  rel l2 vs oracle {err:.3e}, vs generating c {rel_l2(cg, c):.3e}")
    assert err < eps
    if dtype == np.complex128:
        assert rel_l2(cg, c) < 1e-11   # the round trip, within the condition number


@pytest.mark.parametrize("dtype,eps", PATHS)
def test_spectral_plan_reuse(dtype, eps):
    """Section 3.3: one setup per point set, many coefficient vectors."""
    N, M = 3000, 5000
    y, f, c = workloads.forward_case(N, M, "uniform", seed=3)
    dt = fn.FN_C128 if dtype == np.complex128 else fn.FN_C64
    plan = fn.Plan.spectral_forward(N, dev(y), eps, dt)
    rng = np.random.default_rng(4)
    for r in range(3):
        cr = ((rng.standard_normal(N) + 1j * rng.standard_normal(N)) / np.sqrt(2)).astype(dtype)
        g = host(plan(dev(cr)))
        assert rel_l2(g, oracle.eval_series(N, y, cr.astype(np.complex128))) < eps
    plan.destroy()
    yi, ci = workloads.inverse_case(N, 0.4, seed=5)
    pi = fn.Plan.spectral_inverse(dev(yi), eps, dt)
    for r in range(2):
        cr = (rng.standard_normal(N) + 1j * rng.standard_normal(N)) / np.sqrt(2)
        gr = oracle.eval_series(N, yi, cr).astype(dtype)
        cc = host(pi(dev(gr)))
        ref = np.fft.fft(oracle.inv(N, yi, gr.astype(np.complex128))) / N
        assert rel_l2(cc, ref) < eps
    pi.destroy()


@pytest.mark.parametrize("dtype,eps", PATHS)
def test_spectral_2p20_sampled(dtype, eps):
    """N = M = 2^20: the forward on 256 sampled targets against the series,
    and the inverse of exact samples returning the coefficients."""
    N = M = 1 << 20
    y, f, c = workloads.forward_case(N, M, "uniform", seed=20)
    c = c.astype(dtype)
    g = host(fn.nufft_spec_fwd(dev(y), dev(c), eps))
    sel = np.random.default_rng(1).choice(M, 256, replace=False)
    ref = oracle.eval_series(N, y[sel], c.astype(np.complex128))
    err = rel_l2(g[sel], ref)
    say(f"spec fwd 2^20 {np.dtype(dtype).name}: {err:.3e}")
    assert err < eps
    yi, ci = workloads.inverse_case(N, 0.4, seed=21)
    # the values at the jittered points, from the forward FMM of the
    # grid samples (exact to the forward's tolerance, checked above)
    fi = workloads.samples_from_coefficients(ci)
    gi = host(fn.nufft_fwd(dev(yi), dev(fi), 1e-12))
    cc = host(fn.inufft_spec(dev(yi), dev(gi.astype(dtype)), eps))
    errc = rel_l2(cc, ci)
    say(f"spec inv 2^20 {np.dtype(dtype).name}: round trip {errc:.3e}")
    assert errc < (1e-11 if dtype == np.complex128 else 1e-5)
