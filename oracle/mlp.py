"""FP64 oracle of the learned-coefficient network (test infrastructure only).

The paper names "dynamic coefficients" as future work (Sec. 4, Conclusion). The learned mode
predicts, per matrix, the coefficients of the Gram-basis polynomial with exponents
{0, 1, 2, 4, 8, 16} from spectral moments of the Gram matrix G = X X^T, X = A / ||A||_F:

  m_j = tr(G^(2^j)) / h,   j = 0..7            (traces of the powers the method forms)
  phi_j = log2(m_j) / (8 * 2^j)                (scale-free input features)
  a1 = W1 phi + b1,  h1 = gelu(a1)             (64)
  a2 = W2 h1 + b2,   h2 = gelu(a2)             (64)
  z  = W3 h2 + b3                              (6)
  c  = z + (1 - sum z) / 6                     (projection onto sum c = 1)

gelu(x) = x * Phi(x) with the exact normal CDF. Training minimises, per matrix with
singular values sigma (of A) and sigma~ = sigma / ||sigma||_2 (those of X),

  loss = (1/h) sum_i (f(sigma~_i) - 1)^2,   f(x) = x * sum_k c_k x^(2 e_k),

which equals ||Y - U V^T||_F^2 / h for Y = sum_k c_k G^(e_k) X and the polar factor U V^T:
the polynomial acts on each singular value independently (the SVD argument of Sec. 1), so
the loss needs the singular values only.

Parameter vector layout (float): W1[64][8], b1[64], W2[64][64], b2[64], W3[6][64], b3[6].
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "MLP_IN", "MLP_HIDDEN", "MLP_OUT", "MLP_NUM_PARAMS", "LEARNED_EXPONENTS", "unpack_params", "mlp_init",
    "features_from_spectrum", "mlp_forward", "spectral_loss", "mlp_loss_and_grad", "gelu", "gelu_grad",
]

MLP_IN, MLP_HIDDEN, MLP_OUT = 8, 64, 6
LEARNED_EXPONENTS = (0, 1, 2, 4, 8, 16)
_SHAPES = [("W1", (64, 8)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (6, 64)), ("b3", (6,))]
MLP_NUM_PARAMS = sum(int(np.prod(s)) for _, s in _SHAPES)


def unpack_params(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shape in _SHAPES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def mlp_init(seed: int = 0) -> np.ndarray:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases (float64), from the
    seeded input generators."""
    from workloads.gen import fan_in_uniform_np
    return fan_in_uniform_np(seed, _SHAPES)


def features_from_spectrum(sigma) -> np.ndarray:
    """phi_j = log2(m_j) / (8 * 2^j) with m_j = (1/h) sum_i lambda_i^(2^j), lambda = sigma~^2,
    evaluated in log space so that no power underflows."""
    s = np.asarray(sigma, dtype=np.float64)
    h = s.size
    st = s / math.sqrt(float(np.sum(s * s)))
    nz = st[st > 0]
    l2lam = 2.0 * np.log2(nz)
    phi = np.empty(MLP_IN)
    for j in range(MLP_IN):
        t = (2.0 ** j) * l2lam
        mx = float(np.max(t))
        log2_sum = mx + math.log2(float(np.sum(np.exp2(t - mx))))
        phi[j] = (log2_sum - math.log2(h)) / (8.0 * 2.0 ** j)
    return phi


def gelu(x):
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * x * (1.0 + np.vectorize(math.erf)(x / math.sqrt(2.0)))


def gelu_grad(x):
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * (1.0 + np.vectorize(math.erf)(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2 * math.pi)


def mlp_forward(theta, phi):
    """Returns (c, cache) for one feature vector."""
    P = unpack_params(theta)
    phi = np.asarray(phi, dtype=np.float64)
    a1 = P["W1"] @ phi + P["b1"]
    h1 = gelu(a1)
    a2 = P["W2"] @ h1 + P["b2"]
    h2 = gelu(a2)
    z = P["W3"] @ h2 + P["b3"]
    c = z + (1.0 - np.sum(z)) / MLP_OUT
    return c, dict(phi=phi, a1=a1, h1=h1, a2=a2, h2=h2, z=z)


def spectral_loss(c, sigma):
    """(loss, dloss/dc) for one matrix; sigma are the singular values of A."""
    s = np.asarray(sigma, dtype=np.float64)
    h = s.size
    st = s / math.sqrt(float(np.sum(s * s)))
    e = np.asarray(LEARNED_EXPONENTS)
    pw = st[:, None] ** (2 * e[None, :] + 1)        # sigma~^(2e+1)
    f = pw @ np.asarray(c, dtype=np.float64)
    r = f - 1.0
    loss = float(np.sum(r * r)) / h
    dc = 2.0 * (pw.T @ r) / h
    return loss, dc


def mlp_loss_and_grad(theta, batch):
    """Mean spectral loss over a batch [(phi, sigma), ...] and its gradient w.r.t. theta."""
    P = unpack_params(theta)
    g = {k: np.zeros_like(v) for k, v in P.items()}
    total = 0.0
    for phi, sigma in batch:
        c, cache = mlp_forward(theta, phi)
        loss, dc = spectral_loss(c, sigma)
        total += loss
        dz = dc - np.mean(dc)                       # c = z + (1 - sum z)/6
        g["W3"] += np.outer(dz, cache["h2"])
        g["b3"] += dz
        dh2 = P["W3"].T @ dz
        da2 = dh2 * gelu_grad(cache["a2"])
        g["W2"] += np.outer(da2, cache["h1"])
        g["b2"] += da2
        dh1 = P["W2"].T @ da2
        da1 = dh1 * gelu_grad(cache["a1"])
        g["W1"] += np.outer(da1, cache["phi"])
        g["b1"] += da1
    n = len(batch)
    grad = np.concatenate([g[name].reshape(-1) for name, _ in _SHAPES]) / n
    return total / n, grad
