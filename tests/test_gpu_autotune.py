"""The autotuner: its choice is used by later plans, which still meet the
accuracy target against the oracle."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import dev, host, rel_l2, say

pytestmark = pytest.mark.gpu

fn = pytest.importorskip("paper_1611_09379_amd")


@pytest.fixture(autouse=True)
def clear_tuning():
    fn.autotune_clear()
    yield
    fn.autotune_clear()


@pytest.mark.parametrize("dtype,eps", [(fn.FN_C128, 1e-12), (fn.FN_C64, 1e-6)])
def test_autotune_forward(dtype, eps):
    N, M = 4096, 6000
    y, f, c = workloads.forward_case(N, M, "uniform", seed=8)
    cdt = np.complex128 if dtype == fn.FN_C128 else np.complex64
    plain = fn.Plan.forward(N, dev(y), eps, dtype).info()
    l, p = fn.autotune("fwd", N, M, eps, dtype)
    say("tuned", l, p, "default", plain.lmax, plain.nterms)
    assert 2 <= l <= 24 and p in (0, 16, 32, 48)
    plan = fn.Plan.forward(N, dev(y), eps, dtype)
    info = plan.info()
    assert info.lmax == l and (p == 0 or info.nterms == p)
    g = host(plan(dev(f.astype(cdt))))
    plan.destroy()
    err = rel_l2(g, oracle.fwd(N, y, f.astype(cdt).astype(np.complex128)))
    say("tuned rel l2", err)
    assert err < eps
    # the record covers batches of that size class too
    gs = fn.nufft_fwd_batched([dev(y)], [dev(f.astype(cdt))], eps)
    assert np.array_equal(host(gs[0]), g)
    fn.autotune_clear()
    assert fn.Plan.forward(N, dev(y), eps, dtype).info().lmax == plain.lmax


def test_autotune_mixed_skewed():
    """A depth tuned on the mixed path at N = M is reused for a skewed
    N >> M of the same size class (round(log2 sqrt(N M)) = 12): the plan
    still keeps at most 128 sources per leaf and meets 1e-6."""
    l, p = fn.autotune("fwd", 4096, 4096, 1e-6, fn.FN_C64)
    N, M = 1 << 16, 1 << 8
    y, f, c = workloads.forward_case(N, M, "uniform", seed=12)
    f = f.astype(np.complex64)
    plan = fn.Plan.forward(N, dev(y), 1e-6, fn.FN_C64)
    info = plan.info()
    say("tuned", l, p, "skewed plan depth", info.lmax)
    assert (N >> info.lmax) <= 128
    g = host(plan(dev(f)))
    plan.destroy()
    err = rel_l2(g, oracle.fwd(N, y, f.astype(np.complex128)))
    say("skewed rel l2", err)
    assert err < 1e-6


def test_autotune_inverse():
    N = 4096
    y, c = workloads.inverse_case(N, 0.4, seed=9)
    l, p = fn.autotune("inv", N, N, 1e-12)
    say("tuned inverse", l, p)
    plan = fn.Plan.inverse(dev(y), 1e-12)
    assert plan.info().lmax == l
    rng = np.random.default_rng(9)
    g = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    f = host(plan(dev(g)))
    plan.destroy()
    assert rel_l2(f, oracle.inv(N, y, g)) < 1e-12


def test_autotune_errors():
    with pytest.raises(fn.NufftError) as e:
        fn.autotune("fwd", 0, 10, 1e-12)
    assert e.value.status == fn.FN_EINVAL
    with pytest.raises(fn.NufftError) as e:
        fn.autotune("fwd", 100, 100, 1e-20)
    assert e.value.status == fn.FN_EPREC


def test_autotune_records_survive_a_file(tmp_path):
    """A tuned record saved, cleared and loaded again sets the depth of
    later plans."""
    N, M = 4096, 4096
    l, p = fn.autotune("fwd", N, M, 1e-12)
    path = str(tmp_path / "tune.txt")
    fn.autotune_save(path)
    fn.autotune_clear()
    fn.autotune_load(path)
    y, f, c = workloads.forward_case(N, M, "uniform", seed=13)
    info = fn.Plan.forward(N, dev(y), 1e-12).info()
    say("tuned", l, p, "after reload", info.lmax, info.nterms)
    assert info.lmax == l and (p == 0 or info.nterms == p)
