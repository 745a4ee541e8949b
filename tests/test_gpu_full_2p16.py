"""The N = M = 2^16 configuration in full, element by element against the
oracle: the forward transform (Eq. p2) and the inverse (Eq. p6, p8) on a
jittered grid y_j = 2 pi (j + u_j) / N, u_j ~ U(-0.4, 0.4), seed 0, with
c_n iid complex normal.  Every output is compared, not a sample: the
oracle's direct sums (O(N^2), a few tens of seconds on the host cores)
check the inverse's final output at this size, beyond the round trip.

Tolerances: rel-l2 1e-12 on the binary64 path, 1e-6 on the mixed path
(against the oracle on the same binary32-rounded input)."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import dev, host, rel_l2, say

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

fn = pytest.importorskip("paper_1611_09379_amd")

N = 1 << 16


@pytest.fixture(scope="module")
def case():
    y, c = workloads.inverse_case(N, 0.4, seed=0)
    f = workloads.samples_from_coefficients(c)
    say("oracle forward at 2^16 ...")
    g = oracle.fwd(N, y, f)       # exact samples f(y_j): the inverse's input
    return y, f, g


def test_forward_full(case):
    y, f, g_ref = case
    g = host(fn.nufft_fwd(dev(y), dev(f), 1e-12))
    err = rel_l2(g, g_ref)
    say(f"forward 2^16, all {N} targets: {err:.3e}")
    assert err < 1e-12
    f32 = f.astype(np.complex64)
    g32 = host(fn.nufft_fwd(dev(y), dev(f32), 1e-6))
    ref32 = oracle.fwd(N, y, f32.astype(np.complex128))
    err32 = rel_l2(g32, ref32)
    say(f"forward 2^16 mixed: {err32:.3e}")
    assert err32 < 1e-6


def test_inverse_full(case):
    y, f, g = case
    say("oracle inverse at 2^16 ...")
    ref = oracle.inv(N, y, g)
    out = host(fn.inufft(dev(y), dev(g), 1e-12))
    err = rel_l2(out, ref)
    # the oracle's inverse of exact samples returns the samples of the
    # band-limited function: a pin of this input independent of the GPU
    say(f"inverse 2^16, all {N} outputs: {err:.3e}; oracle round trip "
        f"{rel_l2(ref, f):.3e}")
    assert err < 1e-12
    assert rel_l2(ref, f) < 1e-12


def test_inverse_full_mixed(case):
    y, f, g = case
    g32 = g.astype(np.complex64)
    ref = oracle.inv(N, y, g32.astype(np.complex128))
    out = host(fn.inufft(dev(y), dev(g32), 1e-6))
    err = rel_l2(out, ref)
    say(f"inverse 2^16 mixed, all {N} outputs: {err:.3e}")
    assert err < 1e-6
