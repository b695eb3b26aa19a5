"""Coefficient fits of the paper's polynomials, in float64 / mpmath (test infrastructure).

Paper mode (complement basis, exponents n_0 = 0, n_l = 2^(l-1)):
    f(x) = x + sum_{l=1}^{L} w_l x (1 - x^2)^(2^(l-1))                       Eq. (sum_equation)
with w_L tied to the others by Eq. (b_approximation), which gives the training
polynomial of Eq. (overall_polynomial); the w_1..w_{L-1} minimise sum_j (f(x_j) - 1)^2
over points x_j in (0, 1).

Because f is affine in w, the expected loss over x ~ U(0, 1) is a quadratic whose
Gram entries are Beta integrals:
    int_0^1 x^2 (1 - x^2)^n dx = B(3/2, n + 1) / 2,   int_0^1 x (1 - x^2)^n dx = 1 / (2 (n + 1)),
so its minimiser is a closed-form least-squares solution (evaluated in mpmath).
The paper's own optimiser (Adam, lr 0.1 halved every 10000 iterations, 20000
iterations, 1000 fresh U(0,1) points per iteration; Sec. 3.1.1) is replicated by
:func:`tform_adam_fit`. Reading of the unstated details: PyTorch's default Adam
(beta = (0.9, 0.999), eps = 1e-8), w initialised to 0, one iteration per "epoch".

Gram-basis ("G-form") fixed coefficients: the same objective for
f(x) = sum_k c_k x^(2 e_k + 1) with the constraint sum_k c_k = 1 (so f(1) = 1, the
role the constraint plays in Eq. (our_scalar_formula)).
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np

__all__ = [
    "tform_exponents", "tform_f", "tform_basis", "tform_w_last_exact", "tform_w_last_approx",
    "tform_full_w", "tform_ls_fit", "tform_expected_loss", "tform_adam_fit",
    "tform_term_grad", "tform_extreme_point", "gform_ls_fit", "gform_f", "gform_expected_loss",
    "first_reach_one",
]


def tform_exponents(L: int):
    """n_0 = 0, n_l = 2^(l-1) for l = 1..L (exponential schedule of Sec. 2.2)."""
    return [0] + [2 ** (l - 1) for l in range(1, L + 1)]


def tform_basis(x: np.ndarray, L: int) -> np.ndarray:
    """phi_l(x) = x (1 - x^2)^(2^(l-1)), l = 1..L, as columns (Eq. (final_polynomial_term))."""
    x = np.asarray(x, dtype=np.float64)
    t = 1.0 - x * x
    cols = []
    for _ in range(L):
        cols.append(x * t)
        t = t * t
    return np.stack(cols, axis=-1)


def tform_f(x: np.ndarray, w: Sequence[float]) -> np.ndarray:
    """Eq. (sum_equation) with all L coefficients given."""
    w = np.asarray(w, dtype=np.float64)
    return np.asarray(x, dtype=np.float64) + tform_basis(x, len(w)) @ w


def tform_w_last_approx(w_head: Sequence[float], L: int) -> float:
    """Eq. (b_approximation)."""
    return math.exp(0.5) * (2.0 ** (L / 2.0) - 1.0) - float(np.sum(w_head))


def tform_w_last_exact(w_head: Sequence[float], L: int) -> float:
    """The exact solution of the peak constraint Eq. (peak), f(1/sqrt(2^L + 1)) = 1."""
    q = 2.0 ** L
    s = sum(wk * (q / (q + 1.0)) ** (2 ** (k - 1)) for k, wk in enumerate(w_head, start=1))
    return (math.sqrt(q + 1.0) - 1.0 - s) * ((q + 1.0) / q) ** (2 ** (L - 1))


def tform_full_w(w_head: Sequence[float], L: int, exact: bool = False) -> np.ndarray:
    last = tform_w_last_exact(w_head, L) if exact else tform_w_last_approx(w_head, L)
    return np.concatenate([np.asarray(w_head, dtype=np.float64), [last]])


def tform_term_grad(x: np.ndarray, l: int) -> np.ndarray:
    """Eq. (eq_gradient): f_l'(x) = (1 - x^2)^(2^(l-1) - 1) [1 - (2^l + 1) x^2], l >= 1."""
    x = np.asarray(x, dtype=np.float64)
    return (1.0 - x * x) ** (2 ** (l - 1) - 1) * (1.0 - (2 ** l + 1) * x * x)


def tform_extreme_point(l: int):
    """Extreme point of f_l (Sec. 2.2): x* = 1/sqrt(2^l + 1),
    y* = x* (2^l / (2^l + 1))^(2^(l-1)); also the printed approximation x* e^(-1/2)."""
    q = 2.0 ** l
    xs = 1.0 / math.sqrt(q + 1.0)
    ys = xs * (q / (q + 1.0)) ** (2 ** (l - 1))
    return xs, ys, xs * math.exp(-0.5)


def _mp():
    import mpmath
    return mpmath


def tform_ls_fit(L: int, dps: int = 60) -> np.ndarray:
    """Minimiser over w_1..w_{L-1} of E_{x~U(0,1)} (f(x) - 1)^2 for Eq. (overall_polynomial),
    returned as all L coefficients (w_L from Eq. (b_approximation))."""
    mp = _mp()
    mp.mp.dps = dps
    n = [2 ** (l - 1) for l in range(1, L + 1)]
    C = mp.e ** mp.mpf("0.5") * (mp.mpf(2) ** (mp.mpf(L) / 2) - 1)

    def I2(k):  # int x^2 (1-x^2)^k
        return mp.beta(mp.mpf(3) / 2, k + 1) / 2

    def I1(k):  # int x (1-x^2)^k
        return mp.mpf(1) / (2 * (k + 1))

    def Epp(a, b):
        return I2(n[a] + n[b])

    def Exp(a):
        return I2(n[a])

    def Ep(a):
        return I1(n[a])

    Li = L - 1  # free parameters index 0..L-2 ; phi index L-1 is the tied term
    # r0 = x + C phi_L - 1 ; psi_a = phi_a - phi_L
    H = mp.matrix(Li, Li)
    g = mp.matrix(Li, 1)
    last = L - 1
    for a in range(Li):
        for b in range(Li):
            H[a, b] = Epp(a, b) - Epp(a, last) - Epp(last, b) + Epp(last, last)
        e_psi_r0 = (Exp(a) + C * Epp(a, last) - Ep(a)) - (Exp(last) + C * Epp(last, last) - Ep(last))
        g[a] = -e_psi_r0
    w = mp.lu_solve(H, g)
    head = [float(w[i]) for i in range(Li)]
    return tform_full_w(head, L)


def tform_expected_loss(w: Sequence[float], nodes: int = 20000) -> float:
    """E_{x~U(0,1)} (f(x) - 1)^2 by composite Gauss-Legendre quadrature (numerical,
    independent of the Beta closed forms)."""
    gx, gw = np.polynomial.legendre.leggauss(64)
    edges = np.linspace(0.0, 1.0, nodes // 64 + 1)
    tot = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        x = 0.5 * (b - a) * gx + 0.5 * (a + b)
        tot += 0.5 * (b - a) * float(np.sum(gw * (tform_f(x, w) - 1.0) ** 2))
    return tot


def tform_adam_fit(L: int, iters: int = 20000, lr: float = 0.1, step: int = 10000, gamma: float = 0.5,
                   points: int = 1000, seed: int = 11, betas=(0.9, 0.999), eps: float = 1e-8) -> np.ndarray:
    """Replica of the paper's coefficient optimisation (Sec. 3.1.1): Adam on
    sum_j (f(x_j) - 1)^2 with fresh U(0,1) points each iteration and a step decay."""
    from workloads.gen import uniform_np  # seeded points only; no method arithmetic there

    Li = L - 1
    w = np.zeros(Li)
    m = np.zeros(Li)
    v = np.zeros(Li)
    C = math.exp(0.5) * (2.0 ** (L / 2.0) - 1.0)
    for t in range(1, iters + 1):
        x = uniform_np(seed, t, points)
        phi = tform_basis(x, L)
        psi = phi[:, :Li] - phi[:, Li:]
        f = x + C * phi[:, Li] + psi @ w
        grad = 2.0 * psi.T @ (f - 1.0)
        m = betas[0] * m + (1 - betas[0]) * grad
        v = betas[1] * v + (1 - betas[1]) * grad * grad
        mh = m / (1 - betas[0] ** t)
        vh = v / (1 - betas[1] ** t)
        cur_lr = lr * gamma ** ((t - 1) // step)
        w = w - cur_lr * mh / (np.sqrt(vh) + eps)
    return tform_full_w(w, L)


def gform_f(x: np.ndarray, exponents: Sequence[int], c: Sequence[float]) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    for e, ck in zip(exponents, c):
        out = out + ck * x ** (2 * e + 1)
    return out


def gform_expected_loss(exponents, c, nodes: int = 20000) -> float:
    gx, gw = np.polynomial.legendre.leggauss(64)
    edges = np.linspace(0.0, 1.0, nodes // 64 + 1)
    tot = 0.0
    for a, b in zip(edges[:-1], edges[1:]):
        x = 0.5 * (b - a) * gx + 0.5 * (a + b)
        tot += 0.5 * (b - a) * float(np.sum(gw * (gform_f(x, exponents, c) - 1.0) ** 2))
    return tot


def gform_ls_fit(exponents: Sequence[int], dps: int = 60) -> np.ndarray:
    """argmin_c E_{x~U(0,1)} (sum_k c_k x^(2 e_k + 1) - 1)^2 subject to sum_k c_k = 1,
    via the KKT system with moments int x^(2a+2b+2) = 1/(2a+2b+3), int x^(2a+1) = 1/(2a+2)."""
    mp = _mp()
    mp.mp.dps = dps
    e = [int(x) for x in exponents]
    K = len(e)
    Mx = mp.matrix(K + 1, K + 1)
    rhs = mp.matrix(K + 1, 1)
    for i in range(K):
        for j in range(K):
            Mx[i, j] = mp.mpf(1) / (2 * e[i] + 2 * e[j] + 3)
        Mx[i, K] = 1
        Mx[K, i] = 1
        rhs[i] = mp.mpf(1) / (2 * e[i] + 2)
    rhs[K] = 1
    sol = mp.lu_solve(Mx, rhs)
    return np.array([float(sol[i]) for i in range(K)])


def first_reach_one(w: Sequence[float], lo: float = 1e-6, n: int = 2_000_001) -> float:
    """Smallest grid x in (0, 1) with f(x) >= 1 (the curve comparison of Sec. 3.4.1)."""
    x = np.linspace(lo, 1.0, n)
    f = tform_f(x, w)
    idx = np.nonzero(f >= 1.0)[0]
    return float(x[idx[0]]) if idx.size else float("nan")
