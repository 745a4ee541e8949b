"""Seeded synthetic inputs for the FMM-based NUFFT / INUFFT.

This module only draws random numbers and arranges them into the shapes of
the paper's experiments (Section 3: N = M up to 2^20, uniformly random
targets for the forward transform, a perturbed uniform grid for the inverse).
It holds none of the transform's arithmetic, so both the CPU oracle and the
GPU path may take their inputs from it.

Conventions (Eq. p1): f(x) = sum_{n=0}^{N-1} c_n e^{inx}, f_k = f(2 pi k / N).
The coefficients c_n are iid complex normal with E|c_n|^2 = 1, drawn before
the points, and f is their inverse DFT scaled so that f_k = sum_n c_n
e^{2 pi i n k / N}.
"""
from __future__ import annotations

import numpy as np

TWO_PI = 2.0 * np.pi


def coefficients(N: int, rng: np.random.Generator) -> np.ndarray:
    """c_n, n = 0..N-1: iid complex normal with unit variance."""
    z = rng.standard_normal((N, 2))
    return (z[:, 0] + 1j * z[:, 1]) / np.sqrt(2.0)


def samples_from_coefficients(c: np.ndarray) -> np.ndarray:
    """f_k = sum_n c_n e^{2 pi i n k / N} (band-limited samples, Eq. p1)."""
    return np.fft.ifft(c) * c.shape[0]


def points_uniform(M: int, rng: np.random.Generator) -> np.ndarray:
    """y_j iid uniform on [0, 2 pi)."""
    y = rng.random(M) * TWO_PI
    return np.where(y >= TWO_PI, 0.0, y)


def points_jittered(N: int, amp: float, rng: np.random.Generator) -> np.ndarray:
    """y_j = 2 pi (j + u_j) / N with u_j iid U(-amp, amp), reduced to [0, 2 pi)."""
    u = rng.uniform(-amp, amp, N)
    y = TWO_PI * (np.arange(N) + u) / N
    y = np.mod(y, TWO_PI)
    return np.where(y >= TWO_PI, 0.0, y)


def points_clustered(M: int, rng: np.random.Generator, centres: int = 8,
                     sigma: float = 0.01) -> np.ndarray:
    """Wrapped mixture of `centres` equal-weight Gaussians of width sigma."""
    mu = rng.random(centres) * TWO_PI
    which = rng.integers(0, centres, M)
    y = np.mod(mu[which] + sigma * rng.standard_normal(M), TWO_PI)
    return np.where(y >= TWO_PI, 0.0, y)


def forward_case(N: int, M: int, dist: str = "uniform", seed: int = 0,
                 jitter: float = 0.4):
    """(y, f, c) for a forward transform; c is drawn before y."""
    rng = np.random.default_rng(seed)
    c = coefficients(N, rng)
    f = samples_from_coefficients(c)
    if dist == "uniform":
        y = points_uniform(M, rng)
    elif dist == "clustered":
        y = points_clustered(M, rng)
    elif dist == "jittered":
        if M != N:
            raise ValueError("jittered points need M == N")
        y = points_jittered(N, jitter, rng)
    else:
        raise ValueError(f"unknown distribution {dist!r}")
    return y, f, c


def inverse_case(N: int, jitter: float = 0.4, seed: int = 0):
    """(y, c) for an inverse transform on a jittered grid (M = N)."""
    rng = np.random.default_rng(seed)
    c = coefficients(N, rng)
    y = points_jittered(N, jitter, rng)
    return y, c


def batched_sizes(count: int = 512, seed: int = 0, lo: float = 8.0,
                  hi: float = 16.0):
    """N_i = rint(2^U(lo, hi)), M_i = rint(N_i U(0.5, 2)) for `count` transforms."""
    rng = np.random.default_rng(seed)
    Ns = np.rint(2.0 ** rng.uniform(lo, hi, count)).astype(np.int64)
    Ms = np.maximum(1, np.rint(Ns * rng.uniform(0.5, 2.0, count))).astype(np.int64)
    return Ns, Ms
