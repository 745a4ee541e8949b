"""Large transforms: the 2^24 forward and the 2^22 inverse (deep trees, key
ranges beyond the LDS histogram of the sort), checked on sampled targets
against the oracle and by the round trip."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import dev, host, rel_l2, say

pytestmark = pytest.mark.gpu

fn = pytest.importorskip("paper_1611_09379_amd")


@pytest.mark.parametrize("dtype,eps", [(np.complex128, 1e-10), (np.complex64, 1e-6)])
def test_fwd_2p24_sampled(dtype, eps):
    N = M = 1 << 24
    y, f, c = workloads.forward_case(N, M, "uniform", seed=0)
    fq = f.astype(dtype)
    say(f"fwd 2^24 {np.dtype(dtype).name} eps={eps}")
    g = host(fn.nufft_fwd(dev(y), dev(fq), eps))
    sel = np.random.default_rng(5).choice(M, 48, replace=False)
    ref = oracle.fwd_at(N, y, fq.astype(np.complex128), sel)
    err = rel_l2(g[sel], ref)
    say("sampled rel l2", err)
    assert err < eps


def test_fwd_deep_tree_small_leaves():
    """2^17 leaves holding two sources each: the sort takes its global-atomic
    path and the multi-pass scan."""
    N, M = 1 << 18, 1 << 16
    y, f, c = workloads.forward_case(N, M, "uniform", seed=2)
    plan = fn.Plan.forward(N, dev(y), 1e-12, lmax=17)
    assert plan.info().lmax == 17
    g = host(plan(dev(f)))
    plan.destroy()
    sel = np.random.default_rng(6).choice(M, 256, replace=False)
    err = rel_l2(g[sel], oracle.fwd_at(N, y, f, sel))
    say("deep tree rel l2", err)
    assert err < 1e-12


@pytest.mark.parametrize("dtype,eps", [(np.complex128, 1e-10), (np.complex64, 1e-6)])
def test_inv_2p22_round_trip(dtype, eps):
    N = 1 << 22
    y, c = workloads.inverse_case(N, 0.3, seed=0)
    f = workloads.samples_from_coefficients(c).astype(dtype)
    yd, fd = dev(y), dev(f)
    say(f"round trip 2^22 {np.dtype(dtype).name}")
    g = fn.nufft_fwd(yd, fd, eps)
    f2 = host(fn.inufft(yd, g, eps))
    err = rel_l2(f2, f)
    say("round trip rel l2", err)
    assert err < 10 * eps


@pytest.mark.parametrize("dtype,eps", [(np.complex128, 1e-12), (np.complex64, 1e-6)])
def test_fwd_prime_sizes_sampled(dtype, eps):
    """N and M prime near 2^20: leaves of unequal grid counts (the vector
    P2M in place of the matrix-core one, ragged leaf boundaries) at full
    scale, on sampled targets."""
    N, M = 1000003, 999983
    y, f, c = workloads.forward_case(N, M, "uniform", seed=3)
    fq = f.astype(dtype)
    say(f"fwd N={N} M={M} {np.dtype(dtype).name} eps={eps}")
    g = host(fn.nufft_fwd(dev(y), dev(fq), eps))
    sel = np.random.default_rng(7).choice(M, 256, replace=False)
    err = rel_l2(g[sel], oracle.fwd_at(N, y, fq.astype(np.complex128), sel))
    say("sampled rel l2", err)
    assert err < eps


@pytest.mark.parametrize("dtype,eps", [(np.complex128, 1e-12), (np.complex64, 1e-6)])
def test_inv_prime_size_round_trip(dtype, eps):
    """The inverse at N = 1000003 (prime) on a jittered grid: its coefficients
    Chat_k, Dhat_j against the oracle's direct log-sums at sampled indices,
    and the round trip forward then inverse."""
    N = 1000003
    y, c = workloads.inverse_case(N, 0.4, seed=4)
    f = workloads.samples_from_coefficients(c).astype(dtype)
    yd, fd = dev(y), dev(f)
    say(f"inverse N={N} {np.dtype(dtype).name}")
    plan = fn.Plan.inverse(yd, eps, fn.FN_C128 if dtype == np.complex128 else fn.FN_C64)
    chat, dhat = plan.coeffs()
    rng = np.random.default_rng(8)
    ks = rng.choice(N, 64, replace=False)
    js = rng.choice(N, 64, replace=False)
    rc, rd = oracle.coeffs_at(N, y, ks, js)
    ec = rel_l2(host(chat)[ks], rc)
    ed = rel_l2(host(dhat)[js], rd)
    plan.destroy()
    say("coefficients rel l2", ec, ed)
    tol = 1e-12 if dtype == np.complex128 else 1e-6
    assert ec < tol and ed < tol
    g = fn.nufft_fwd(yd, fd, eps)
    f2 = host(fn.inufft(yd, g, eps))
    err = rel_l2(f2, f)
    say("round trip rel l2", err)
    assert err < 10 * eps
