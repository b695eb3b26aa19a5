"""FP64 oracle of the Newton-Schulz variants the paper compares against (test infrastructure only).

Sec. 2 names, besides Muon's fixed quintic of Eq. (iteration_jordan):

* Cesista's iteration: one odd quintic per step, reparameterised by three numbers
  (gamma, r, u) as x -> gamma (x - f_1) ... (x - f_5) + x with the five roots
  f = (-(1 + r), -(1 - u), 0, 1 - u, 1 + r);
* CANS: odd polynomials chosen with the Chebyshev alternation theorem, applied to the input
  scaled by Gelfand's bound, Eq. (gelfand_formula) and Eq. (scale_formula_function):
  X_0 = A / ||(A A^T)^q||_F^(1/(2q)), which puts every singular value in (0, 1].

The paper prints neither Cesista's fitted (gamma, r, u) nor the CANS polynomials. The
readings used here:

* Cesista: five steps, one (gamma_k, r_k, u_k) per step, fitted jointly to minimise
  E_{x ~ U(0,1)} (phi(x) - 1)^2 of the composed scalar map phi (the objective the paper uses
  for its own coefficients, experiment section), the expectation taken by Gauss-Legendre
  quadrature, by BFGS (exact gradient) started from Muon's quintic on every step.
* CANS: step k applies the odd polynomial of degree 3 or 5 that minimises max |1 - p(x)| over
  the interval [lo_k, hi_k] known to hold the singular values (Remez exchange), widened at the
  top by a 2 % margin for rounding; the interval starts at [delta, 1] and becomes
  [1 - E_k, 1 + E_k] after a step with minimax error E_k.

Matrix iterations: X_{k+1} = a_k X_k + b_k (X_k X_k^T) X_k + c_k (X_k X_k^T)^2 X_k with
numpy's matmul as the only library step. Only the tests, the smoke check and the
benchmark's CPU-baseline leg may use this module.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np

from .ifnso import orient

__all__ = [
    "cesista_to_abc", "abc_to_cesista", "compose_scalar", "cesista_objective", "cesista_objective_grad",
    "cesista_fit",
    "minimax_odd", "cans_schedule", "gelfand_scale", "ns_schedule",
]


# ---------------------------------------------------------------------------------------------
# Cesista's reparameterised quintic
# ---------------------------------------------------------------------------------------------
def cesista_to_abc(gamma: float, r: float, u: float) -> Tuple[float, float, float]:
    """Coefficients of x -> a x + b x^3 + c x^5 equal to gamma prod_i (x - f_i) + x.

    With alpha = 1 - u and beta = 1 + r the roots pair up as +-alpha, +-beta and 0, so
    prod_i (x - f_i) = x (x^2 - alpha^2)(x^2 - beta^2)
                     = x^5 - (alpha^2 + beta^2) x^3 + alpha^2 beta^2 x."""
    al2, be2 = (1.0 - u) ** 2, (1.0 + r) ** 2
    return 1.0 + gamma * al2 * be2, -gamma * (al2 + be2), gamma


def abc_to_cesista(a: float, b: float, c: float) -> Tuple[float, float, float]:
    """Inverse of :func:`cesista_to_abc` where it exists (c != 0 and alpha^2, beta^2 real
    and positive): gamma = c; alpha^2 and beta^2 are the roots of t^2 + (b/c) t + (a-1)/c,
    the smaller one alpha^2."""
    if c == 0.0:
        raise ValueError("a cubic has no (gamma, r, u) form")
    s, p = -b / c, (a - 1.0) / c
    disc = s * s - 4.0 * p
    if disc < 0.0 or p <= 0.0:
        raise ValueError("roots not real and positive")
    t1, t2 = (s - math.sqrt(disc)) / 2.0, (s + math.sqrt(disc)) / 2.0
    return c, math.sqrt(t2) - 1.0, 1.0 - math.sqrt(t1)


def compose_scalar(x, schedule: Sequence[Sequence[float]]) -> np.ndarray:
    """phi(x): the scalar maps x <- a x + b x^3 + c x^5 of the schedule applied in order
    (what the matrix iteration does to every singular value)."""
    x = np.asarray(x, dtype=np.float64).copy()
    for a, b, c in schedule:
        x2 = x * x
        x = x * (a + x2 * (b + c * x2))
    return x


def _gauss_legendre_unit(n: int):
    t, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (t + 1.0), 0.5 * w


def cesista_objective(schedule, nodes: int = 400) -> float:
    """E_{x ~ U(0,1)} (phi(x) - 1)^2 by n-point Gauss-Legendre quadrature on (0, 1)."""
    x, w = _gauss_legendre_unit(nodes)
    return float(np.sum(w * (compose_scalar(x, schedule) - 1.0) ** 2))


def cesista_objective_grad(params, nodes: int = 400):
    """The objective of :func:`cesista_objective` for the schedule of (gamma_k, r_k, u_k) and its
    gradient with respect to those parameters (reverse accumulation through the composed map:
    g_k = g_{k+1} p_k'(x_k) with p_k' = a + 3 b x^2 + 5 c x^4, then the chain rule through
    a = 1 + gamma alpha^2 beta^2, b = -gamma (alpha^2 + beta^2), c = gamma, alpha = 1 - u,
    beta = 1 + r)."""
    x, w = _gauss_legendre_unit(nodes)
    params = [tuple(float(v) for v in p) for p in params]
    abc = [cesista_to_abc(*p) for p in params]
    xs = [np.asarray(x, dtype=np.float64)]
    for a, b, c in abc:
        t = xs[-1]
        t2 = t * t
        xs.append(t * (a + t2 * (b + c * t2)))
    d = xs[-1] - 1.0
    loss = float(np.sum(w * d * d))
    g = 2.0 * w * d
    grad = np.zeros((len(params), 3))
    for k in range(len(params) - 1, -1, -1):
        a, b, c = abc[k]
        t = xs[k]
        t2 = t * t
        da, db, dc = float(np.sum(g * t)), float(np.sum(g * t * t2)), float(np.sum(g * t * t2 * t2))
        gamma, r, u = params[k]
        al, be = 1.0 - u, 1.0 + r
        grad[k, 0] = da * al * al * be * be - db * (al * al + be * be) + dc
        grad[k, 1] = da * gamma * al * al * 2.0 * be - db * gamma * 2.0 * be
        grad[k, 2] = -da * gamma * be * be * 2.0 * al + db * gamma * 2.0 * al
        g = g * (a + t2 * (3.0 * b + 5.0 * c * t2))
    return loss, grad


def cesista_fit(steps: int = 5, nodes: int = 400, start=(3.4445, -4.7750, 2.0315)):
    """Fits (gamma_k, r_k, u_k), k = 0..steps-1, to the objective of
    :func:`cesista_objective` by BFGS with the gradient of :func:`cesista_objective_grad`, to a
    stationary point (gradient below 1e-10); starts every step at the (gamma, r, u) of the
    `start` quintic.
    Returns (params [steps][3], schedule [steps][3] of (a, b, c))."""
    from scipy.optimize import minimize

    theta0 = np.array(list(abc_to_cesista(*start)) * steps, dtype=np.float64)

    def fun(theta):
        with np.errstate(over="ignore", invalid="ignore"):  # trial points of the line search may diverge
            v, g = cesista_objective_grad(theta.reshape(steps, 3), nodes)
        if not (math.isfinite(v) and np.all(np.isfinite(g))):
            return 1e300, np.zeros_like(theta)
        return v, g.reshape(-1)

    res = minimize(fun, theta0, jac=True, method="BFGS", options={"maxiter": 20000, "gtol": 1e-10})
    sched = [cesista_to_abc(*(float(v) for v in res.x[3 * k:3 * k + 3])) for k in range(steps)]
    # (r, u) and (-u, -r) give the same polynomial: report the form with 1 - u <= 1 + r
    return [abc_to_cesista(*abc) for abc in sched], sched


# ---------------------------------------------------------------------------------------------
# CANS: minimax odd polynomials (Chebyshev alternation) and their interval schedule
# ---------------------------------------------------------------------------------------------
def minimax_odd(lo: float, hi: float, degree: int = 5, iters: int = 100, tol: float = 1e-15):
    """Odd polynomial p(x) = sum_j c_j x^(2j+1) of the given degree (3 or 5) minimising
    max_{x in [lo, hi]} |1 - p(x)|, by the Remez exchange: on a reference of d + 1 points
    (d = (degree + 1) / 2 coefficients) solve 1 - p(x_i) = (-1)^i E, move the reference to the
    endpoints and the interior extrema of 1 - p, repeat until the levels agree.
    Returns (coefficients padded to (a, b, c), E >= 0)."""
    if degree not in (3, 5) or not (0.0 < lo < hi):
        raise ValueError("degree 3 or 5 on 0 < lo < hi")
    d = (degree + 1) // 2
    k = np.arange(d + 1)
    ref = 0.5 * (lo + hi) - 0.5 * (hi - lo) * np.cos(np.pi * k / d)  # Chebyshev extrema
    powers = 2 * np.arange(d) + 1
    c = np.zeros(d)
    E = 0.0
    for _ in range(iters):
        Amat = np.zeros((d + 1, d + 1))
        Amat[:, :d] = ref[:, None] ** powers[None, :]
        Amat[:, d] = (-1.0) ** k
        sol = np.linalg.solve(Amat, np.ones(d + 1))
        c, E = sol[:d], sol[d]
        # interior critical points: p'(x) = sum_j (2j+1) c_j t^j with t = x^2
        dcoef = (powers * c)[::-1]  # highest power of t first
        roots = np.roots(dcoef) if d > 1 else np.array([])
        crit = sorted(math.sqrt(t.real) for t in roots
                      if abs(t.imag) < 1e-12 and lo * lo < t.real < hi * hi)
        new = np.array([lo] + crit + [hi])
        if len(new) != d + 1:
            break
        err = 1.0 - new[:, None] ** powers[None, :] @ c
        done = abs(np.max(np.abs(err)) - abs(E)) <= tol * max(1.0, abs(E)) and np.allclose(new, ref, rtol=0, atol=1e-15)
        ref = new
        if done:
            break
    out = [0.0, 0.0, 0.0]
    out[:d] = [float(v) for v in c]
    return tuple(out), float(abs(E))


def cans_schedule(steps: int, delta: float, degree: int = 5, margin: float = 0.02):
    """Per-step minimax polynomials for singular values starting in [delta, 1]; returns
    (schedule [steps][3], intervals [steps + 1][2]). Step k's polynomial is the minimax one
    on [lo_k, (1 + margin) hi_k] and maps it onto [lo_{k+1}, hi_{k+1}] = [1 - E, 1 + E]. The
    margin keeps a singular value that rounding has pushed just past hi_k inside the range
    the polynomial was built for: each polynomial rises steeply at the top of its interval,
    and without the margin the next one would amplify such an excess at every step."""
    lo, hi = float(delta), 1.0
    sched: List[Tuple[float, float, float]] = []
    iv = [(lo, hi)]
    for _ in range(steps):
        abc, E = minimax_odd(lo, hi * (1.0 + margin), degree)
        sched.append(abc)
        lo, hi = 1.0 - E, 1.0 + E
        iv.append((lo, hi))
    return sched, iv


# ---------------------------------------------------------------------------------------------
# Gelfand scaling and the matrix iteration
# ---------------------------------------------------------------------------------------------
def gelfand_scale(A: np.ndarray, q: int) -> float:
    """s = ||(A A^T)^q||_F^(1/(2q)), Eq. (scale_formula_function); an upper bound of the
    largest singular value of A by Eq. (gelfand_formula)."""
    if q < 1:
        raise ValueError("q >= 1")
    A = np.asarray(A, dtype=np.float64)
    G = A @ A.T
    P = G
    for _ in range(q - 1):
        P = P @ G
    return float(np.sqrt(np.sum(P * P)) ** (1.0 / (2 * q)))


def ns_schedule(M: np.ndarray, schedule: Sequence[Sequence[float]], gelfand_q: int = 0) -> np.ndarray:
    """The matrix iteration of a schedule: A oriented as in Sec. 1 (h <= w), X_0 = A / s with
    s = ||A||_F (gelfand_q = 0, Eq. (constraint)) or s = ||(A A^T)^q||_F^(1/(2q)) (q >= 1),
    then X_{k+1} = a_k X_k + b_k G_k X_k + c_k G_k^2 X_k, G_k = X_k X_k^T. Returned in M's
    orientation; a zero input gives zero."""
    A, trans = orient(M)
    s = float(np.sqrt(np.sum(A * A))) if gelfand_q == 0 else gelfand_scale(A, gelfand_q)
    X = np.zeros_like(A) if s == 0.0 else A / s
    for a, b, c in schedule:
        G = X @ X.T
        X = a * X + b * (G @ X) + c * (G @ (G @ X))
    return X.T if trans else X

