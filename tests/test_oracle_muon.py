"""Pins of the Muon-step oracle against closed forms and invariants (no GPU).

* Prescribed spectra: for G = U diag(sigma) V^T the orthogonalised update is
  U diag(f(sigma~)) V^T with the polynomial's scalar map f, so the weight change is known in
  closed form without calling the oracle's polynomial.
* The momentum recursion unrolls to a geometric sum of the gradients.
* Nesterov's input (1 + mu) G (zero initial momentum) orthogonalises like G itself: the
  Frobenius-normalised method is invariant under positive scaling of its input.
* Zero gradient and zero momentum: the weight only decays, by exactly (1 - lr wd).
* The shape factor sqrt(max(1, rows / cols)) gives tall and wide updates the same RMS per entry
  when the update is exactly orthogonal (a polynomial that is the identity on sigma~ = 1).
"""
import math

import numpy as np

import oracle
from oracle import muon as MU
from workloads import configs, gen


def _spectral(rows, cols, seed):
    r = min(rows, cols)
    U = gen.haar_np(rows, r, seed, 1)
    V = gen.haar_np(cols, r, seed, 2)
    sig = 0.1 + 0.9 * gen.uniform_np(seed, 3, r)
    return U, sig, V


def test_update_matches_closed_form():
    exps, c = configs.load_coeffs("gform_v1")
    for rows, cols in [(24, 40), (40, 24)]:
        U, sig, V = _spectral(rows, cols, 5)
        G = (U * sig) @ V.T
        W = gen.gaussian_np(rows, cols, 6)
        lr, wd = 0.02, 0.1
        W1, B1, _ = MU.muon_step(W, G, np.zeros_like(G), exps, c, lr, momentum=0.0, weight_decay=wd, nesterov=False)
        O = oracle.closed_form(U, sig, V, exps, c)
        want = (1 - lr * wd) * W - lr * math.sqrt(max(1.0, rows / cols)) * O
        assert np.allclose(W1, want, rtol=0, atol=1e-12)
        assert np.array_equal(B1, G)


def test_momentum_is_a_geometric_sum():
    exps, c = configs.load_coeffs("gform_v1")
    mu = 0.9
    Gs = [gen.gaussian_np(16, 32, 10 + k) for k in range(4)]
    B = np.zeros((16, 32))
    W = np.zeros((16, 32))
    for G in Gs:
        W, B, _ = MU.muon_step(W, G, B, exps, c, lr=0.01, momentum=mu, nesterov=False)
    want = sum(mu ** (3 - k) * Gs[k] for k in range(4))
    assert np.allclose(B, want, rtol=1e-14, atol=1e-14)


def test_nesterov_input_is_a_positive_multiple_at_zero_momentum():
    exps, c = configs.load_coeffs("gform_v1")
    G = gen.gaussian_np(20, 36, 21)
    W = gen.gaussian_np(20, 36, 22)
    a = MU.muon_step(W, G, np.zeros_like(G), exps, c, lr=0.05, momentum=0.95, nesterov=True)
    b = MU.muon_step(W, G, np.zeros_like(G), exps, c, lr=0.05, momentum=0.0, nesterov=False)
    assert np.allclose(a[0], b[0], rtol=0, atol=1e-12)
    assert np.allclose(a[1], G) and np.allclose(b[1], G)


def test_zero_gradient_only_decays():
    exps, c = configs.load_coeffs("gform_v1")
    W = gen.gaussian_np(12, 30, 31)
    W1, B1, O = MU.muon_step(W, np.zeros_like(W), np.zeros_like(W), exps, c, lr=0.1, momentum=0.9,
                             weight_decay=0.25)
    assert np.array_equal(O, np.zeros_like(W))
    assert np.array_equal(W1, (1 - 0.1 * 0.25) * W) and not B1.any()


def test_shape_factor_equalises_update_rms():
    """An input with all singular values equal (G = 3 U V^T) and the constant polynomial
    c_0 = sqrt(r) (r = min(rows, cols)) orthogonalise exactly to U V^T. Its RMS per entry is
    1/sqrt(cols) when wide and 1/sqrt(rows) when tall; after the shape factor the update's RMS is
    1/sqrt(cols) either way."""
    for rows, cols in [(16, 48), (48, 16), (48, 48)]:
        r = min(rows, cols)
        U = gen.haar_np(rows, r, 41, 1)
        V = gen.haar_np(cols, r, 41, 2)
        G = U @ V.T * 3.0
        W1, _, O = MU.muon_step(np.zeros((rows, cols)), G, np.zeros((rows, cols)), (0,), (math.sqrt(r),),
                                lr=1.0, momentum=0.0, nesterov=False)
        # Frobenius normalisation gives X = U V^T / sqrt(r); c_0 = sqrt(r) restores U V^T
        assert np.allclose(O, U @ V.T, atol=1e-12)
        rms = np.sqrt(np.mean(W1 * W1))
        assert abs(rms - 1.0 / math.sqrt(cols)) < 1e-12
        assert abs(MU.muon_scale(rows, cols) - math.sqrt(max(1.0, rows / cols))) < 1e-15
