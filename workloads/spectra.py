"""Seeded singular spectra for training and judging the learned coefficients.

Each sample draws h ~ U{64..1024}, w = round(h * U(1, 4)), and a spectrum from one of three
families with equal weight (chosen by the sample index modulo 3):
  log-uniform   sigma_i = 10^(-d u_i), d ~ U(2, 4)           (log-uniform on [10^-d, 1])
  power law     sigma_i = i^(-alpha), alpha ~ U(0.5, 2)
  near 1        sigma_i = clip(1 - |N(0, tau^2)|, 1e-6, 1), tau ~ U(0.01, 0.2)
Every random number comes from the counter generator (stream = 1000 + sample index).
"""
from __future__ import annotations

import numpy as np

from .gen import normal_np, uniform_np

__all__ = ["spectral_sample", "spectral_mixture", "pad_spectra"]


def spectral_sample(seed: int, index: int, hmin: int = 64, hmax: int = 1024):
    stream = 1000 + index
    u = uniform_np(seed, stream, 3)
    h = hmin + int(u[0] * (hmax - hmin + 1))
    w = int(round(h * (1.0 + 3.0 * u[1])))
    kind = index % 3
    if kind == 0:
        d = 2.0 + 2.0 * u[2]
        sig = 10.0 ** (-d * uniform_np(seed, stream + 10_000_000, h))
    elif kind == 1:
        alpha = 0.5 + 1.5 * u[2]
        sig = np.arange(1, h + 1, dtype=np.float64) ** -alpha
    else:
        tau = 0.01 + 0.19 * u[2]
        sig = np.clip(1.0 - np.abs(tau * normal_np(seed, stream + 10_000_000, h)), 1e-6, 1.0)
    return h, w, np.sort(sig)[::-1].copy()


def spectral_mixture(n: int, seed: int = 5, start: int = 0, hmin: int = 64, hmax: int = 1024):
    return [spectral_sample(seed, start + i, hmin, hmax) for i in range(n)]


def pad_spectra(samples, smax: int = 1024):
    """(sig[n][smax] float32 zero-padded, nsig[n] int32)."""
    n = len(samples)
    sig = np.zeros((n, smax), dtype=np.float32)
    nsig = np.zeros(n, dtype=np.int32)
    for i, (h, _, s) in enumerate(samples):
        sig[i, :h] = s
        nsig[i] = h
    return sig, nsig
