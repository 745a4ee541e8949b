"""Pins of the CPU oracle against things other than itself: brute force of
Eq. (p2) in mpmath, closed forms of the paper (f = 1 gives g = 1, Section 3.1;
exact band-limited interpolation, Eq. p1), the exact-hit limit of Eq. (p2),
the Lagrange-form inverse (Eq. p6/p8) against a dense linear solve, and the
uniform-shift closed forms of the products of Eq. (p8)."""
import mpmath
import numpy as np
import pytest

import oracle
import workloads

mpmath.mp.dps = 40


def mp_grid(N, y):
    s = mpmath.mpf(y) * N / (2 * mpmath.pi)
    n = mpmath.floor(s + mpmath.mpf(1) / 2)
    return int(n) % N, s - n


@pytest.mark.parametrize("N", [1, 2, 7, 64, 1000, 1 << 20])
def test_grid_units_exact(N):
    rng = np.random.default_rng(N)
    y = np.concatenate([rng.random(40) * 2 * np.pi, [0.0, -1e-300, 2 * np.pi,
                        -3.5, 17.25, np.nextafter(2 * np.pi, 0)]])
    m, th = oracle.grid_units(N, y)
    for j in range(y.size):
        mm, tt = mp_grid(N, y[j])
        assert m[j] == mm
        assert abs(th[j] - float(tt)) <= 1e-16 * max(1.0, abs(float(tt)))
        assert -0.5 <= th[j] <= 0.5


def mp_K(N, y, k):
    """K_jk of Eq. (p2) summed literally over n in 40-digit arithmetic."""
    x = 2 * mpmath.pi * k / N
    yy = mpmath.mpf(y)
    return sum(mpmath.exp(1j * n * (yy - x)) for n in range(N)) / N


@pytest.mark.parametrize("N", [1, 2, 3, 8, 13])
def test_fwd_brute_force_eq_p2(N):
    rng = np.random.default_rng(100 + N)
    f = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    y = np.concatenate([rng.random(6) * 2 * np.pi, [0.0, 2 * np.pi * 1 / N,
                        np.pi, 6.0]])
    g = oracle.fwd(N, y, f)
    for j in range(y.size):
        ref = sum(mp_K(N, y[j], k) * mpmath.mpc(f[k]) for k in range(N))
        assert abs(complex(ref) - g[j]) <= 1e-14 * (1 + abs(complex(ref)))


@pytest.mark.parametrize("N,dist", [(1000, "uniform"), (1024, "clustered"),
                                    (1024, "uniform")])
def test_fwd_matches_spectral_route(N, dist):
    y, f, c = workloads.forward_case(N, 777, dist, seed=3)
    g1 = oracle.fwd(N, y, f)
    g2 = oracle.fwd_spectral(N, y, f)
    g3 = oracle.eval_series(N, y, c)
    assert np.linalg.norm(g1 - g2) / np.linalg.norm(g2) < 1e-14
    assert np.linalg.norm(g1 - g3) / np.linalg.norm(g3) < 1e-14


@pytest.mark.parametrize("N", [5, 1000, 4096])
def test_constant_function(N):
    """Section 3.1: f = 1 is interpolated exactly, g_j = 1."""
    rng = np.random.default_rng(N)
    y = workloads.points_uniform(997, rng)
    g = oracle.fwd(N, y, np.ones(N))
    assert np.abs(g - 1).max() < 1e-14


@pytest.mark.parametrize("N,n0", [(64, 0), (64, 1), (64, 63), (999, 500),
                                  (1024, 17)])
def test_single_frequency(N, n0):
    """c = e_{n0} (Eq. p1): f_k = e^{i n0 x_k} and g_j = e^{i n0 y_j}."""
    rng = np.random.default_rng(n0)
    y = workloads.points_uniform(50, rng)
    f = np.array([complex(mpmath.expjpi(mpmath.mpf(2 * ((n0 * k) % N)) / N))
                  for k in range(N)])
    g = oracle.fwd(N, y, f)
    ref = np.array([complex(mpmath.exp(1j * n0 * mpmath.mpf(v))) for v in y])
    assert np.abs(g - ref).max() < 2e-14


def test_exact_and_near_hits():
    N = 256
    rng = np.random.default_rng(5)
    f = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    y = np.array([0.0, 2 * np.pi * 5 / N, 2 * np.pi * 100 / N, np.pi])
    g = oracle.fwd(N, y, f)
    assert g[0] == f[0]                     # exact hit: K_jk = delta
    # fl(x_k) is within one ulp of x_k: g = f_k up to N * u
    assert abs(g[1] - f[5]) < 1e-12 * np.abs(f).max()
    assert abs(g[2] - f[100]) < 1e-12 * np.abs(f).max()
    assert abs(g[3] - f[128]) < 1e-12 * np.abs(f).max()
    ref = [complex(sum(mp_K(N, y[j], k) * mpmath.mpc(f[k]) for k in range(N)))
           for j in (1, 3)]
    assert abs(g[1] - ref[0]) < 1e-13 * abs(ref[0])
    assert abs(g[3] - ref[1]) < 1e-13 * abs(ref[1])


def dense_K(N, y):
    """K_jk of Eq. (p2) as an explicit matrix, summed over n in numpy."""
    n = np.arange(N)
    Ey = np.exp(1j * np.outer(y, n))
    Ex = np.exp(1j * np.outer(2 * np.pi * np.arange(N) / N, n))
    return Ey @ Ex.conj().T / N


@pytest.mark.parametrize("N,amp", [(64, 0.4), (127, 0.3), (256, 0.1)])
def test_inverse_matches_dense_solve(N, amp):
    y, c = workloads.inverse_case(N, amp, seed=N)
    rng = np.random.default_rng(1)
    g = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    f = oracle.inv(N, y, g)
    ref = np.linalg.solve(dense_K(N, y), g)
    assert np.linalg.norm(f - ref) / np.linalg.norm(ref) < 1e-12


@pytest.mark.parametrize("N,amp", [(257, 0.4), (1024, 0.3), (2048, 0.4)])
def test_round_trip(N, amp):
    """Eq. (p6) inverts Eq. (p2): INUFFT(NUFFT(f)) = f for M = N."""
    y, c = workloads.inverse_case(N, amp, seed=7)
    f = workloads.samples_from_coefficients(c)
    g = oracle.fwd(N, y, f)
    f2 = oracle.inv(N, y, g)
    assert np.linalg.norm(f2 - f) / np.linalg.norm(f) < 1e-13


@pytest.mark.parametrize("N,delta", [(16, 0.25), (1000, 0.37), (1024, -0.2)])
def test_uniform_shift_closed_forms(N, delta):
    """y_j = x_j + 2 pi delta / N: prod_j 2 sin(pi (k - j - delta)/N) has modulus
    2|sin(pi delta)| and prod_{k!=j} |2 sin(pi (j - k)/N)| = N, so
    logC = log(2|sin pi delta|) and logD = -log N (Eq. p8 rescaled by 2^N);
    the inverse is the exact fractional shift of a band-limited function."""
    y = 2 * np.pi * (np.arange(N) + delta) / N
    # y_j is rounded to binary64, which moves s_j by up to N 2^-52 grid units;
    # d logC / d s_j = (pi/N) cot(pi (k - s_j)/N) sums to about 2 (1 + ln N)
    # in modulus, so the closed form holds to that input perturbation.
    tol = 4.0 * N * 2.0 ** -52 * (1.0 + np.log(N)) + 1e-14
    logC, negC, logD, negD = oracle.logsums(N, y)
    assert np.abs(logC - np.log(2 * abs(np.sin(np.pi * delta)))).max() < tol
    assert np.abs(logD + np.log(N)).max() < tol
    assert sorted(negD.tolist()) == list(range(N))   # ranks are a permutation
    rng = np.random.default_rng(2)
    c = workloads.coefficients(N, rng)
    f = workloads.samples_from_coefficients(c)
    g = oracle.eval_series(N, y, c)
    f2 = oracle.inv(N, y, g)
    assert np.linalg.norm(f2 - f) / np.linalg.norm(f) < 1e-13


def test_logsums_brute_force():
    N = 12
    rng = np.random.default_rng(9)
    y = np.sort(rng.random(N) * 2 * np.pi)
    y[3] = 0.0 + 1e-3
    logC, negC, logD, negD = oracle.logsums(N, y)
    for k in range(N):
        xk = 2 * mpmath.pi * k / N
        prod = mpmath.mpf(1)
        for v in y:
            prod *= 2 * mpmath.sin((xk - mpmath.mpf(v)) / 2)
        assert abs(float(mpmath.log(abs(prod))) - logC[k]) < 1e-14
        assert (prod < 0) == bool(negC[k] % 2)
    for j in range(N):
        prod = mpmath.mpf(1)
        for i in range(N):
            if i != j:
                prod *= 2 * mpmath.sin((mpmath.mpf(y[j]) - mpmath.mpf(y[i])) / 2)
        assert abs(-float(mpmath.log(abs(prod))) - logD[j]) < 1e-14
        assert (prod < 0) == bool(negD[j] % 2)


def test_inverse_hits_and_singular():
    N = 64
    y, c = workloads.inverse_case(N, 0.3, seed=4)
    y[0] = 0.0                                   # exact hit at x_0
    rng = np.random.default_rng(3)
    g = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    f = oracle.inv(N, y, g)
    assert f[0] == g[0]
    ref = np.linalg.solve(dense_K(N, y), g)
    assert np.linalg.norm(f - ref) / np.linalg.norm(ref) < 1e-12
    y2 = y.copy()
    y2[5] = y2[9]
    with pytest.raises(oracle.OracleError):
        oracle.inv(N, y2, g)


@pytest.mark.parametrize("N,amp", [(16, 0.3), (23, 0.45)])
def test_coeffs_brute_force_eq_p8(N, amp):
    """Chat_k = 2^N C_k and Dhat_j = 2^-N D_j of Eq. (p8), written as the
    products of sines they are, in 40-digit arithmetic."""
    y, c = workloads.inverse_case(N, amp, seed=N)
    ks = np.arange(N)
    chat, dhat = oracle.coeffs_at(N, y, ks, ks)
    for k in range(N):
        xk = 2 * mpmath.pi * k / N
        prod = mpmath.mpf(1)
        for v in y:
            prod *= 2 * mpmath.sin((xk - mpmath.mpf(v)) / 2)
        ref = (-1) ** k * prod
        assert abs(chat[k] - float(ref)) <= 1e-13 * abs(float(ref))
    for j in range(N):
        yj = mpmath.mpf(y[j])
        prod = mpmath.mpf(1)
        for i in range(N):
            if i != j:
                prod *= 2 * mpmath.sin((yj - mpmath.mpf(y[i])) / 2)
        ref = 1j * mpmath.exp(-1j * N * yj / 2) / prod
        assert abs(dhat[j] - complex(ref)) <= 1e-13 * abs(complex(ref))


def test_logsums_large_n_mpmath():
    """Log-sums of Eq. (p8) at N = 2^16 against 30-digit sums.  Per-term
    errors of about 5e-17 (random) allow some 1e-14 here; a bias common to
    all N terms shows far above that (a rounded pi in the sine's argument:
    3.9e-17 N ln 2 = 1.8e-12; rounding the whole logarithm of each term:
    about 4e-13)."""
    N = 1 << 16
    y, c = workloads.inverse_case(N, 0.4, seed=21)
    ks = np.array([7, 40000])
    js = np.array([3, 51234])
    logC, negC, logD, negD = oracle.logsums(N, y, ks, js)
    with mpmath.workdps(30):
        ym = [mpmath.mpf(v) for v in y]
        for i, k in enumerate(ks):
            xk = 2 * mpmath.pi * int(k) / N
            ref = mpmath.fsum(mpmath.log(abs(2 * mpmath.sin((xk - v) / 2))) for v in ym)
            assert abs(float(ref) - logC[i]) < 2e-13, (k, float(ref) - logC[i])
        for t, j in enumerate(js):
            yj = ym[int(j)]
            ref = -mpmath.fsum(mpmath.log(abs(2 * mpmath.sin((yj - v) / 2)))
                               for i, v in enumerate(ym) if i != int(j))
            assert abs(float(ref) - logD[t]) < 2e-13, (j, float(ref) - logD[t])


@pytest.mark.parametrize("N", [1, 7, 1000, 4096])
def test_fwd_at_selects_fwd(N):
    """fwd_at(N, y, f, sel) is fwd(N, y, f)[sel] bit for bit (Eq. p2 through
    p4): the selection keeps duplicates and order, and exact hits (y = 0,
    y = 2 pi, y = -2 pi) go through the same per-target sum."""
    rng = np.random.default_rng(31 + N)
    M = 300
    y = workloads.points_uniform(M, rng)
    y[:3] = [0.0, 2 * np.pi, -2 * np.pi]
    y[3] = 2 * np.pi * (N // 2) / N
    f = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    g = oracle.fwd(N, y, f)
    sel = np.concatenate([[M - 1, 0, 5, 5, 1, 2, 3, 0], rng.permutation(M)[:50],
                          rng.integers(0, M, 20)])
    gs = oracle.fwd_at(N, y, f, sel)
    assert gs.shape == sel.shape
    assert np.array_equal(gs.view(np.float64), g[sel].view(np.float64))
    assert np.array_equal(oracle.fwd_at(N, y, f, sel[:0]), g[:0])


@pytest.mark.parametrize("N", [5, 13])
def test_fwd_at_brute_force_eq_p2(N):
    """fwd_at against Eq. (p2) summed literally over n in 40 digits, at
    targets picked out of order."""
    rng = np.random.default_rng(200 + N)
    f = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    y = np.concatenate([rng.random(5) * 2 * np.pi, [0.0, 2 * np.pi * 3 / N]])
    sel = np.array([4, 6, 0, 5, 2, 2])
    g = oracle.fwd_at(N, y, f, sel)
    for i, j in enumerate(sel):
        ref = sum(mp_K(N, y[j], k) * mpmath.mpc(f[k]) for k in range(N))
        assert abs(complex(ref) - g[i]) <= 1e-14 * (1 + abs(complex(ref)))


@pytest.mark.parametrize("N,M", [(64, 100), (127, 50), (256, 256)])
def test_adj_matches_dense_conjugate_transpose(N, M):
    """adj is K^H g with K of Eq. (p2) as an explicit matrix (numpy sum over
    n), including points on the grid and repeated points."""
    rng = np.random.default_rng(N + M)
    y = workloads.points_uniform(M, rng)
    y[:4] = [0.0, 2 * np.pi * 5 / N, y[10], 0.0]     # hits, repeats
    g = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    f = oracle.adj(N, y, g)
    ref = dense_K(N, y).conj().T @ g
    assert np.linalg.norm(f - ref) / np.linalg.norm(ref) < 1e-12


@pytest.mark.parametrize("N,M,dist", [(1000, 1500, "uniform"), (1024, 700, "clustered"),
                                      (4097, 4097, "uniform")])
def test_adj_inner_product_identity(N, M, dist):
    """<K f, g> = <f, K^H g> with the oracle's forward sum (Eq. p2-p5): a
    dropped conjugate, a sign of the cot term or a swapped index fails it."""
    y, f, c = workloads.forward_case(N, M, dist, seed=11)
    rng = np.random.default_rng(12)
    g = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    lhs = np.vdot(g, oracle.fwd(N, y, f))
    rhs = np.vdot(oracle.adj(N, y, g), f)
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(f) * np.linalg.norm(g) * np.sqrt(N)


@pytest.mark.parametrize("N", [1, 3, 8, 13])
def test_adj_brute_force_eq_p2(N):
    """f_k = sum_j conj(K_jk) g_j with K_jk of Eq. (p2) summed literally over
    n in 40 digits; points on the grid and a repeated point included, and a
    selection of k out of order."""
    rng = np.random.default_rng(300 + N)
    y = np.concatenate([rng.random(5) * 2 * np.pi, [0.0, 2 * np.pi * (N - 1) / N, 0.0]])
    M = y.size
    g = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    ks = np.array([N - 1, 0, N // 2, 0])
    f = oracle.adj(N, y, g, ks)
    for i, k in enumerate(ks):
        ref = sum(mpmath.conj(mp_K(N, y[j], int(k))) * mpmath.mpc(g[j]) for j in range(M))
        assert abs(complex(ref) - f[i]) <= 1e-14 * (1 + abs(complex(ref)))
    assert np.array_equal(oracle.adj(N, y, g)[ks], f)


def test_fwd_tiny_fractions_brute_force_eq_p2():
    """Points a subnormal or tiny distance from a grid point: the oracle's
    value is finite and equals the literal sum of Eq. (p2) (40 digits), i.e.
    f_m up to a term of order theta."""
    N = 13
    rng = np.random.default_rng(77)
    f = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    y = np.array([5e-324, -5e-324, 1e-250, -1e-210, 1e-190, 2 * np.pi * 3 / N + 1e-300])
    g = oracle.fwd(N, y, f)
    assert np.all(np.isfinite(g))
    for j in range(y.size):
        ref = sum(mp_K(N, y[j], k) * mpmath.mpc(f[k]) for k in range(N))
        assert abs(complex(ref) - g[j]) <= 1e-14 * (1 + abs(complex(ref)))
    gi = oracle.inv(N, np.concatenate([[1e-250], 2 * np.pi * (np.arange(1, N) + 0.3) / N]), f)
    assert np.all(np.isfinite(gi)) and gi[0] == f[0]


@pytest.mark.parametrize("N,M", [(1, 3), (8, 5), (64, 100), (257, 300)])
def test_kmatrix_matches_eq_p2_and_forward(N, M):
    """The closed-form matrix equals Eq. (p2) summed over n (numpy), and its
    product with f is the oracle's forward sum; a grid point gives a delta
    row."""
    rng = np.random.default_rng(N + M)
    y = rng.random(M) * 2 * np.pi
    y[0] = 2 * np.pi * (N // 2) / N if N > 1 else 0.0
    y[-1] = 0.0
    K = oracle.kmatrix(N, y)
    Kd = dense_K(N, y)
    assert np.abs(K - Kd).max() < 1e-13 * max(1, N)
    assert np.array_equal(K[-1], np.eye(N)[0])
    f = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    assert np.linalg.norm(K @ f - oracle.fwd(N, y, f)) <= 1e-13 * np.linalg.norm(K @ f)


def test_lsq_normal_equations_and_consistent_data():
    """oracle.lsq: for consistent data g = K f it returns f (K has full
    column rank for M = 2N uniform points); for inconsistent data its
    residual is orthogonal to the range of K (the normal equations)."""
    rng = np.random.default_rng(9)
    N, M = 64, 128
    y = rng.random(M) * 2 * np.pi
    f = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    K = oracle.kmatrix(N, y)
    assert np.linalg.norm(oracle.lsq(N, y, K @ f) - f) < 1e-9 * np.linalg.norm(f)
    g = K @ f + 0.1 * (rng.standard_normal(M) + 1j * rng.standard_normal(M))
    fl = oracle.lsq(N, y, g)
    assert np.linalg.norm(K.conj().T @ (K @ fl - g)) < 1e-10 * np.linalg.norm(K.conj().T @ g)
