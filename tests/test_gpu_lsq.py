"""Least-squares inverse (nufft_lsq: CG on the normal equations of Eq. p2,
one forward and one adjoint transform per iteration) against the oracle's
dense least squares: oversampled uniform points (M > N), noisy data, the
square jittered case (where it must agree with the Lagrange inverse), and
clustered points that the square inverse rejects.  Tolerances are stated
per case from the condition number of K (measured with numpy)."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import dev, host, rel_l2, say

pytestmark = pytest.mark.gpu

fn = pytest.importorskip("paper_1611_09379_amd")


def cond(N, y):
    return float(np.linalg.cond(oracle.kmatrix(N, y)))


@pytest.mark.parametrize("dtype,eps,tol", [(np.complex128, 1e-12, 1e-12),
                                           (np.complex64, 1e-6, 1e-6)])
@pytest.mark.parametrize("N,M,noise", [(256, 512, 0.0), (1000, 3000, 0.0),
                                       (512, 2048, 0.1), (97, 300, 0.05)])
def test_lsq_oversampled(N, M, noise, dtype, eps, tol):
    rng = np.random.default_rng(N + M)
    y = workloads.points_uniform(M, rng)
    c = workloads.coefficients(N, rng)
    f = workloads.samples_from_coefficients(c)
    g = oracle.fwd(N, y, f)
    if noise:
        g = g + noise * np.linalg.norm(g) / np.sqrt(M) * (
            rng.standard_normal(M) + 1j * rng.standard_normal(M)) / np.sqrt(2)
    gx = g.astype(dtype)
    ref = oracle.lsq(N, y, gx.astype(np.complex128))
    k = cond(N, y)
    out, it, res = fn.nufft_lsq(dev(y), dev(gx), N, eps, tol=tol, maxiter=500)
    err = rel_l2(host(out), ref)
    say(f"lsq N={N} M={M} noise={noise} {np.dtype(dtype).name}: cond {k:.1f}, "
        f"{it} iterations, residual {res:.2e}, rel l2 vs oracle {err:.2e}")
    assert res <= tol
    # CG stops at a normal-equation residual tol: the error is at most
    # cond(K)^2 tol, plus cond(K) times the transforms' own error
    assert err < k * k * tol + 10 * k * eps


def test_lsq_square_matches_inverse():
    """M = N on a jittered grid: the least-squares solution is the inverse
    (Eq. p6), against the oracle's Lagrange form."""
    N = 2048
    y, c = workloads.inverse_case(N, 0.3, seed=5)
    g = oracle.eval_series(N, y, c)
    out, it, res = fn.nufft_lsq(dev(y), dev(g), N, 1e-12, tol=1e-13, maxiter=300)
    ref = oracle.inv(N, y, g)
    err = rel_l2(host(out), ref)
    say(f"lsq square N={N}: {it} iterations, residual {res:.2e}, vs inverse {err:.2e}")
    assert err < 1e-10


def test_lsq_where_the_square_inverse_fails():
    """Points squeezed into 95% of the circle (N = 512, M = N): the square
    inverse is out of range on the mixed path and ill-conditioned; with
    M = 4N points on the same arc K has a condition number near 1e17 (a
    band-limited function is nearly free on the empty arc), yet CG fits the
    data: its relative misfit ||K f - g|| / ||g|| falls to 1.2e-6 at a
    normal-equation residual of 1e-10 (measured), where the solution itself
    is not determined."""
    N, M = 512, 2048
    rng = np.random.default_rng(11)
    y = 2 * np.pi * 0.95 * np.sort(rng.random(M))
    f = workloads.samples_from_coefficients(workloads.coefficients(N, rng))
    g = oracle.fwd(N, y, f)
    with pytest.raises(fn.NufftError):
        fn.inufft(dev(y[:N]), dev(g[:N].astype(np.complex64)), 1e-6)
    out, it, res = fn.nufft_lsq(dev(y), dev(g), N, 1e-12, tol=1e-10, maxiter=2000)
    fo = host(out)
    ref = oracle.lsq(N, y, g)
    K = oracle.kmatrix(N, y)
    fit = np.linalg.norm(K @ fo - g) / np.linalg.norm(g)
    fit_ref = np.linalg.norm(K @ ref - g) / np.linalg.norm(g)
    say(f"lsq gap: cond {cond(N, y):.2e}, {it} iterations, residual {res:.2e}, "
        f"data misfit {fit:.2e} (oracle {fit_ref:.2e})")
    assert res <= 1e-10 and fit < 1e-5
