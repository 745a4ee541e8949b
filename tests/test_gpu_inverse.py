"""Inverse transform (M = N) on the GPU against the CPU oracle (Eq. p6/p8)."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import dev, host, rel_l2, say

pytestmark = pytest.mark.gpu

fn = pytest.importorskip("paper_1611_09379_amd")


def run_inv(y, g, eps, dtype=np.complex128):
    say(f"inv N={y.shape[0]} eps={eps} dtype={np.dtype(dtype).name}")
    return host(fn.inufft(dev(y), dev(g.astype(dtype)), eps))


@pytest.mark.parametrize("N,amp", [(1024, 0.4), (1000, 0.3), (8192, 0.4),
                                   (4097, 0.1)])
def test_inv_fp64_full(N, amp):
    y, c = workloads.inverse_case(N, amp, seed=0)
    rng = np.random.default_rng(1)
    g = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    f = run_inv(y, g, 1e-12)
    ref = oracle.inv(N, y, g)
    err = rel_l2(f, ref)
    say("rel l2", err)
    assert err < 1e-12


@pytest.mark.parametrize("lmax", [6, 7, 8])
def test_inv_explicit_depths(lmax):
    """Shallow trees put more points in one sort key (a box of 16 leaves):
    4096 at depth 6, about 2048 at depth 7 (on both sides of the limit),
    1024 at depth 8.  Above 2048 points the leaf order goes through global
    memory instead of LDS, and the ranks it forms still have to give the
    oracle's f (Eq. p8 signs and self-exclusion)."""
    N = 1 << 14
    y, c = workloads.inverse_case(N, 0.35, seed=4)
    rng = np.random.default_rng(2)
    g = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    plan = fn.Plan.inverse(dev(y), 1e-12, fn.FN_C128, lmax=lmax)
    assert plan.info().lmax == lmax
    f = host(plan(dev(g)))
    plan.destroy()
    err = rel_l2(f, oracle.inv(N, y, g))
    say("lmax", lmax, "rel l2", err)
    assert err < 1e-12


@pytest.mark.parametrize("N", [1, 2, 3, 5, 16, 100])
def test_inv_tiny(N):
    y, c = workloads.inverse_case(N, 0.3, seed=N)
    rng = np.random.default_rng(N)
    g = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    assert rel_l2(run_inv(y, g, 1e-12), oracle.inv(N, y, g)) < 1e-12


def test_inv_uniform_shift():
    """y_j = x_j + 2 pi delta / N: the inverse undoes the fractional shift.
    g_j = f(y_j) is evaluated from the coefficients at the binary64 points
    (Eq. p1), so the inverse must return the samples f_k themselves."""
    N, delta = 4096, 0.37
    y = 2 * np.pi * (np.arange(N) + delta) / N
    rng = np.random.default_rng(2)
    c = workloads.coefficients(N, rng)
    f = workloads.samples_from_coefficients(c)
    g = oracle.eval_series(N, y, c)
    f2 = run_inv(y, g, 1e-12)
    err = rel_l2(f2, f)
    say("shift rel l2", err)
    assert err < 1e-12


def test_inv_hits_and_errors():
    N = 512
    y, c = workloads.inverse_case(N, 0.3, seed=4)
    y[0] = 0.0
    rng = np.random.default_rng(3)
    g = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    f = run_inv(y, g, 1e-12)
    assert f[0] == g[0]
    assert rel_l2(f, oracle.inv(N, y, g)) < 1e-12
    y2 = y.copy()
    y2[5] = y2[9]
    with pytest.raises(fn.NufftError) as e:
        run_inv(y2, g, 1e-12)
    assert e.value.status == fn.FN_ESINGULAR


@pytest.mark.parametrize("N,amp,dtype,eps", [(1 << 16, 0.4, np.complex128, 1e-12),
                                             (1 << 16, 0.4, np.complex64, 1e-6),
                                             (1 << 20, 0.4, np.complex128, 1e-12),
                                             (1 << 20, 0.4, np.complex64, 1e-6)])
def test_round_trip(N, amp, dtype, eps):
    """INUFFT(NUFFT(f)) = f (Eq. p6 inverts Eq. p2), within cond * eps."""
    y, c = workloads.inverse_case(N, amp, seed=0)
    f = workloads.samples_from_coefficients(c).astype(dtype)
    fd, yd = dev(f), dev(y)
    say(f"round trip N={N} dtype={np.dtype(dtype).name}")
    g = fn.nufft_fwd(yd, fd, eps)
    f2 = host(fn.inufft(yd, g, eps))
    err = rel_l2(f2, f)
    say("round trip rel l2", err)
    assert err < 10 * eps


def test_inv_mixed():
    N = 8192
    y, c = workloads.inverse_case(N, 0.4, seed=6)
    rng = np.random.default_rng(6)
    g = (rng.standard_normal(N) + 1j * rng.standard_normal(N)).astype(np.complex64)
    f = run_inv(y, g, 1e-6, dtype=np.complex64)
    ref = oracle.inv(N, y, g.astype(np.complex128))
    err = rel_l2(f, ref)
    say("mixed inv rel l2", err)
    assert err < 1e-6


def test_inv_clustered_rejected():
    """A clustered point set makes the inverse ill-posed (Eq. p8: the
    products of sines leave any floating-point range): FN_ERANGE, from the
    one-shot call and from the plan, without running the near field of the
    dense leaves."""
    N = 8192
    rng = np.random.default_rng(9)
    g = dev((rng.standard_normal(N) + 1j * rng.standard_normal(N)))
    # every point in one leaf: far above the dense-leaf limit
    y_one = np.pi + 1e-3 * np.sort(rng.random(N))
    # a mixture of 8 narrow Gaussians: |D_j| overflows
    y_mix = workloads.points_clustered(N, rng)
    for y in (y_one, y_mix):
        say("clustered inverse", y.min(), y.max())
        with pytest.raises(fn.NufftError) as e:
            fn.inufft(dev(y), g, 1e-12)
        assert e.value.status == fn.FN_ERANGE
        with pytest.raises(fn.NufftError) as e:
            fn.Plan.inverse(dev(y), 1e-12)
        assert e.value.status == fn.FN_ERANGE
    # still usable afterwards
    y, c = workloads.inverse_case(1024, 0.4, seed=3)
    g1 = np.random.default_rng(4).standard_normal(1024) + 0j
    assert rel_l2(run_inv(y, g1, 1e-12), oracle.inv(1024, y, g1)) < 1e-12


@pytest.mark.parametrize("N,amp,dtype", [(1 << 20, 0.4, fn.FN_C128), (1 << 20, 0.4, fn.FN_C64),
                                         (1 << 16, 0.4, fn.FN_C128), (4097, 0.1, fn.FN_C128)])
def test_coeffs_sampled(N, amp, dtype):
    """Chat_k and Dhat_j of Eq. (p8) (log-kernel FMM) against the oracle's
    direct log-sums at sampled indices, at full size."""
    y, c = workloads.inverse_case(N, amp, seed=0)
    plan = fn.Plan.inverse(dev(y), 1e-12 if dtype == fn.FN_C128 else 1e-6, dtype)
    chat, dhat = (host(t) for t in plan.coeffs())
    plan.destroy()
    rng = np.random.default_rng(11)
    ks = rng.choice(N, min(N, 384), replace=False)
    js = rng.choice(N, min(N, 384), replace=False)
    rc, rd = oracle.coeffs_at(N, y, ks, js)
    ec, ed = rel_l2(chat[ks], rc), rel_l2(dhat[js], rd)
    say(f"coeffs N={N}: Chat {ec:.2e} Dhat {ed:.2e}")
    # the log-sums are binary64 on both paths, truncated for a tenth of eps
    tol = 1e-12 if dtype == fn.FN_C128 else 1e-6
    assert ec < tol and ed < tol


def test_setup_timings():
    """Event timings of the log-sum FMM: recorded only while timing is on,
    and leaving the coefficients unchanged."""
    N = 1 << 14
    y, c = workloads.inverse_case(N, 0.4, seed=3)
    yd = dev(y)
    say(f"timings N={N}")
    p0 = fn.Plan.inverse(yd, 1e-12, fn.FN_C128)
    t0 = p0.timings()
    ch0, dh0 = (host(x) for x in p0.coeffs())
    p0.destroy()
    assert t0["log_up_ms"] == -1 and t0["log_trans_ms"] == -1 and t0["log_eval_ms"] == -1
    assert t0["log_terms"] > 0
    fn.set_timing(True)
    try:
        p1 = fn.Plan.inverse(yd, 1e-12, fn.FN_C128)
    finally:
        fn.set_timing(False)
    t1 = p1.timings()
    ch1, dh1 = (host(x) for x in p1.coeffs())
    p1.destroy()
    say("timings", t1)
    assert t1["log_up_ms"] > 0 and t1["log_trans_ms"] > 0 and t1["log_eval_ms"] > 0
    assert t1["sort_ms"] > 0 and t0["sort_ms"] == -1
    assert np.array_equal(ch0, ch1) and np.array_equal(dh0, dh1)
    pf = fn.Plan.forward(N, yd, 1e-12, fn.FN_C128)
    assert pf.timings()["log_terms"] == 0 and pf.timings()["sort_ms"] == -1
    pf.destroy()
    fn.set_timing(True)
    try:
        pf = fn.Plan.forward(N, yd, 1e-12, fn.FN_C128)
    finally:
        fn.set_timing(False)
    tf = pf.timings()
    pf.destroy()
    assert tf["sort_ms"] > 0 and tf["log_up_ms"] == -1


def test_inv_mixed_range():
    """A grid compressed into 95% of the circle (N = 1024): log|Dhat_j|
    reaches about -120 (oracle), beyond what the mixed path's binary32
    weights Dhat_j g_j hold (and the problem's condition number is about
    7e15).  FN_C64 reports FN_ERANGE instead of a wrong result; FN_C128
    (range exp(+-700)) accepts it, with Chat_k and Dhat_j equal to the
    oracle's log-sums."""
    N = 1024
    y = 2 * np.pi * np.arange(N) / N * 0.95 + 1e-3
    lC, _, lD, _ = oracle.logsums(N, y)
    assert np.abs(lD).max() > 100 and np.abs(lD).max() < 700
    rng = np.random.default_rng(5)
    g = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    with pytest.raises(fn.NufftError) as e:
        fn.inufft(dev(y), dev(g.astype(np.complex64)), 1e-6)
    assert e.value.status == fn.FN_ERANGE
    with pytest.raises(fn.NufftError) as e:
        fn.Plan.inverse(dev(y), 1e-6, fn.FN_C64)
    assert e.value.status == fn.FN_ERANGE
    plan = fn.Plan.inverse(dev(y), 1e-12, fn.FN_C128)
    chat, dhat = (host(t) for t in plan.coeffs())
    assert np.all(np.isfinite(host(plan(dev(g)))))
    plan.destroy()
    ks = np.arange(1, N, 7)
    js = np.arange(0, N, 5)
    rc, rd = oracle.coeffs_at(N, y, ks, js)
    ec, ed = rel_l2(chat[ks], rc), rel_l2(dhat[js], rd)
    say(f"compressed grid, binary64 coefficients: Chat {ec:.2e} Dhat {ed:.2e}")
    assert ec < 1e-12 and ed < 1e-12


@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
def test_tiny_fractions_are_hits(dtype):
    """Points within 2^-100 grid units of a grid point (|theta| as small as
    1e-42 and subnormal) are exact hits: no overflowing reciprocal, and the
    result matches the oracle's exact sums (which differ from f_m by a term
    of order theta)."""
    N, M = 256, 64
    y, f, c = workloads.forward_case(N, M, "uniform", seed=6)
    y[:4] = [1e-42, -1e-42, 2 * np.pi * 5 / N, 5e-324]
    f = f.astype(dtype)
    eps = 1e-12 if dtype == np.complex128 else 1e-6
    g = host(fn.nufft_fwd(dev(y), dev(f), eps))
    assert np.all(np.isfinite(g))
    ref = oracle.fwd(N, y, f.astype(np.complex128))
    assert rel_l2(g, ref) < eps
    yi, ci = workloads.inverse_case(N, 0.3, seed=6)
    yi[0] = 1e-42
    gi = (np.random.default_rng(6).standard_normal(N) + 0j).astype(dtype)
    fi = host(fn.inufft(dev(yi), dev(gi), eps))
    assert np.all(np.isfinite(fi))
    assert rel_l2(fi, oracle.inv(N, yi, gi.astype(np.complex128))) < eps
