"""Batches of forward transforms of uneven sizes in shared launches, against
the oracle and against the single-transform path."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import dev, host, rel_l2, say

pytestmark = pytest.mark.gpu

fn = pytest.importorskip("paper_1611_09379_amd")


def make_batch(count, seed, lo, hi):
    Ns, Ms = workloads.batched_sizes(count, seed=seed, lo=lo, hi=hi)
    cases = []
    for t, (N, M) in enumerate(zip(Ns, Ms)):
        y, f, c = workloads.forward_case(int(N), int(M), "uniform", seed=1000 * seed + t)
        cases.append((int(N), y, f))
    return cases


@pytest.mark.parametrize("dtype,eps", [(np.complex128, 1e-12), (np.complex64, 1e-6)])
def test_batch_full_parity(dtype, eps):
    cases = make_batch(24, seed=1, lo=3.0, hi=11.0)
    say(f"batch of {len(cases)}, sizes {[c[0] for c in cases]}")
    ys = [dev(y) for _, y, _ in cases]
    fs = [dev(f.astype(dtype)) for _, _, f in cases]
    gs = fn.nufft_fwd_batched(ys, fs, eps)
    for (N, y, f), g in zip(cases, gs):
        ref = oracle.fwd(N, y, f.astype(dtype).astype(np.complex128))
        err = rel_l2(host(g), ref)
        assert err < eps, (N, y.shape[0], err)


def test_batch_equals_single_and_graph_replay():
    """The shared launches compute what single transforms compute, bit for
    bit; a batch plan replays its graph with new inputs and outputs."""
    cases = make_batch(40, seed=2, lo=6.0, hi=13.0)
    ys = [dev(y) for _, y, _ in cases]
    fs = [dev(f) for _, _, f in cases]
    singles = [host(fn.nufft_fwd(y, f, 1e-12)) for y, f in zip(ys, fs)]
    gs = fn.nufft_fwd_batched(ys, fs, 1e-12)
    for a, b in zip(gs, singles):
        assert np.array_equal(host(a), b)
    batch = fn.Batch.forward(ys, [c[0] for c in cases], 1e-12)
    rng = np.random.default_rng(3)
    for rep in range(2):
        f2 = [f * complex(rng.standard_normal(), rng.standard_normal()) for f in fs]
        g2 = batch(f2)
        g2b = batch(f2) if rep else g2  # replays the same graph again
        for (N, y, f), fx, g, gb in zip(cases, f2, g2, g2b):
            want = host(fn.nufft_fwd(dev(y), fx, 1e-12))
            assert np.array_equal(host(g), want)
            assert np.array_equal(host(gb), want)
    batch.destroy()


def test_batch_with_a_large_transform():
    """A transform whose tree exceeds the shared sort runs with its own
    launches inside the same call."""
    cases = make_batch(6, seed=4, lo=8.0, hi=12.0)
    N = M = 1 << 22
    y, f, c = workloads.forward_case(N, M, "uniform", seed=44)
    cases.insert(3, (N, y, f))
    ys = [dev(y) for _, y, _ in cases]
    fs = [dev(f) for _, _, f in cases]
    gs = fn.nufft_fwd_batched(ys, fs, 1e-10)
    for (Nt, yt, ft), g in zip(cases, gs):
        if Nt == N:
            sel = np.random.default_rng(5).choice(M, 64, replace=False)
            err = rel_l2(host(g)[sel], oracle.fwd_at(Nt, yt, ft, sel))
        else:
            err = rel_l2(host(g), oracle.fwd(Nt, yt, ft))
        assert err < 1e-10, (Nt, err)


@pytest.mark.parametrize("dtype,eps", [(np.complex128, 1e-12), (np.complex64, 1e-6)])
def test_batch_512_sampled(dtype, eps):
    """512 transforms, N log-uniform in [2^8, 2^16], M = N U(0.5, 2)."""
    cases = make_batch(512, seed=0, lo=8.0, hi=16.0)
    ys = [dev(y) for _, y, _ in cases]
    fs = [dev(f.astype(dtype)) for _, _, f in cases]
    say("batch 512", sum(c[0] for c in cases), sum(c[1].shape[0] for c in cases))
    gs = fn.nufft_fwd_batched(ys, fs, eps)
    rng = np.random.default_rng(6)
    num = den = 0.0
    for (N, y, f), g in zip(cases, gs):
        sel = rng.choice(y.shape[0], min(16, y.shape[0]), replace=False)
        ref = oracle.fwd_at(N, y, f.astype(dtype).astype(np.complex128), sel)
        num += np.sum(np.abs(host(g)[sel] - ref) ** 2)
        den += np.sum(np.abs(ref) ** 2)
    err = np.sqrt(num / den)
    say("batch 512 sampled rel l2", err)
    assert err < eps


def test_batch_errors():
    cases = make_batch(5, seed=7, lo=6.0, hi=9.0)
    ys = [dev(y) for _, y, _ in cases]
    fs = [dev(f) for _, _, f in cases]
    bad = cases[2][1].copy()
    bad[1] = np.nan
    ys[2] = dev(bad)
    with pytest.raises(fn.NufftError) as e:
        fn.nufft_fwd_batched(ys, fs, 1e-12)
    assert e.value.status == fn.FN_EINVAL and "transform 2" in str(e.value)
    with pytest.raises(fn.NufftError) as e:
        fn.Batch.forward(ys, [c[0] for c in cases], 1e-12)
    assert e.value.status == fn.FN_EINVAL
    with pytest.raises(fn.NufftError) as e:
        fn.nufft_fwd_batched(ys[:1], fs[:1], 1e-20)
    assert e.value.status == fn.FN_EPREC
