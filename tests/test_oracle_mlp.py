"""Pins of the learned-coefficient oracle: central finite differences for the backward pass,
the spectral loss against the matrix definition ||Y - U V^T||_F^2 / h, and the spectral
features against traces of explicit Gram powers."""
import math

import numpy as np
import pytest

import oracle as O
from workloads import gen, spectra


def test_parameter_count():
    assert O.MLP_NUM_PARAMS == 5126


def test_backward_matches_finite_differences():
    theta = O.mlp_init(3)
    samples = spectra.spectral_mixture(4, seed=9, hmax=96)
    batch = [(O.features_from_spectrum(s), s) for _, _, s in samples]
    loss, grad = O.mlp_loss_and_grad(theta, batch)
    idx = [0, 7, 300, 511, 512, 600, 2000, 4100, 4672, 4700, 4736, 5000, 5120, 5125]
    eps = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (O.mlp_loss_and_grad(tp, batch)[0] - O.mlp_loss_and_grad(tm, batch)[0]) / (2 * eps)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, grad[i])


def test_projection_sums_to_one():
    theta = O.mlp_init(4)
    c, _ = O.mlp_forward(theta, np.linspace(-1, 0, 8))
    assert abs(c.sum() - 1.0) < 1e-12


def test_spectral_loss_is_polar_distance():
    """(1/h) sum (f(s~) - 1)^2 equals ||Y - U V^T||_F^2 / h for the matrix polynomial."""
    rows, cols = 24, 40
    sig = np.sort(0.05 + gen.uniform_np(2, 3, rows))[::-1]
    M, U, V = gen.spectral_np(rows, cols, sig, seed=2)
    c = np.array([1.7, -0.8, 0.3, 0.1, -0.2, -0.1])
    loss, _ = O.spectral_loss(c, sig)
    Y = O.ifnso(M, O.LEARNED_EXPONENTS, c)
    d = Y - U @ V.T
    assert abs(loss - float(np.sum(d * d)) / rows) < 1e-12 * max(1.0, loss)


def test_features_are_traces_of_gram_powers():
    rows, cols = 16, 30
    sig = 10.0 ** (-2 * gen.uniform_np(7, 3, rows))
    M, U, V = gen.spectral_np(rows, cols, sig, seed=7)
    parts = O.ifnso_parts(M, [0, 1, 2, 4, 8, 16, 32, 64, 128], [1] * 9)
    phi = O.features_from_spectrum(sig)
    for j in range(8):
        tr = float(np.trace(parts["powers"][2 ** j]))
        if tr > 1e-280:
            assert abs(phi[j] - math.log2(tr / rows) / (8 * 2 ** j)) < 1e-9, j


def test_feature_log_space_does_not_underflow():
    sig = np.full(500, 1.0)  # lambda = 1/500; lambda^128 underflows float64 directly
    phi = O.features_from_spectrum(sig)
    for j in range(8):
        assert abs(phi[j] - (2 ** j) * math.log2(1 / 500) / (8 * 2 ** j)) < 1e-9


def test_spectral_mixture_families():
    s = spectra.spectral_mixture(9, seed=5)
    for i, (h, w, sig) in enumerate(s):
        assert 64 <= h <= 1024 and h <= w <= 4 * h + 1 and sig.shape == (h,)
        assert np.all(sig > 0) and np.all(sig <= 1.0) and np.all(np.diff(sig) <= 0)
    assert s[2][2].min() >= 1e-6  # clustered near 1
