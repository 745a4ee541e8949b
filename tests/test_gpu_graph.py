"""nufft_execute under HIP graph capture: a plan's execute captured once
(torch.cuda.graph) and replayed on new inputs, with eager work and
synchronisations between the replays, equals the eager execute bit for
bit every time (Section 3.3: a plan set up once serves many inputs)."""
import numpy as np
import pytest

import workloads
from gpu_util import dev, host, say

pytestmark = pytest.mark.gpu

fn = pytest.importorskip("paper_1611_09379_amd")


def replay_check(plan, n_in, n_out, cdt, seed):
    import torch
    tdt = torch.complex128 if cdt == np.complex128 else torch.complex64
    rng = np.random.default_rng(seed)

    def data():
        return (rng.standard_normal(n_in) + 1j * rng.standard_normal(n_in)).astype(cdt)

    x = dev(data())
    out = torch.empty(n_out, dtype=tdt, device="cuda")
    plan.execute(x, out=out)          # eager run before capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.execute(x, out=out)
    for rep in range(4):
        xin = data()
        x.copy_(dev(xin))
        graph.replay()
        got = host(out).copy()
        ref = host(plan.execute(dev(xin)))   # eager, on a fresh output
        say("replay", rep, "max diff", float(np.abs(got - ref).max()))
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("dtype,eps", [(np.complex128, 1e-12), (np.complex64, 1e-6)])
def test_forward_plan_graph(dtype, eps):
    N, M = 4096, 5000
    y, f, c = workloads.forward_case(N, M, "uniform", seed=31)
    plan = fn.Plan.forward(N, dev(y), eps, fn.FN_C128 if dtype == np.complex128 else fn.FN_C64)
    replay_check(plan, N, M, dtype, 31)
    plan.destroy()


def test_inverse_plan_graph():
    N = 4096
    y, c = workloads.inverse_case(N, 0.4, seed=32)
    plan = fn.Plan.inverse(dev(y), 1e-12)
    replay_check(plan, N, N, np.complex128, 32)
    plan.destroy()
