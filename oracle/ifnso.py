"""FP64 oracle of IFNSO and of classical Newton-Schulz (test infrastructure only).

Plain numpy in float64; matrix products use numpy's matmul as a library step and
nothing is blocked, fused or reordered. Every function states the passage of the
paper (Hu et al., "IFNSO: Iteration-Free Newton-Schulz Orthogonalization",
arXiv 2602.02500) it follows. Readings of silent or ambiguous passages:

* The output is returned in the orientation of the input M (the paper's
  Algorithm 1 returns Y in the orientation of A); Y_M = Y^T when M was transposed.
* No epsilon is added to any normalisation; a zero input gives a zero output.
* "I - XX^T" is read for the "(1 - XX^T)" printed in Eq. (newnew_formula).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this module.
"""
from __future__ import annotations

import math
from typing import Dict, Sequence, Tuple

import numpy as np

__all__ = [
    "orient", "normalise", "ifnso", "ifnso_parts", "paper_form", "classical_ns",
    "orth_error", "singular_value_map", "closed_form", "flops_ifnso", "flops_ns",
    "paper_w_last_approx", "paper_coeffs_to_terms", "BASES", "NORMS",
]

BASES = ("gram", "complement")
NORMS = ("frobenius", "gram_frobenius", "none")


def orient(M: np.ndarray) -> Tuple[np.ndarray, bool]:
    """Transposition rule of Sec. 1 (first equation) and Algorithm 1, initialisation:
    A = M if h_input <= w_input, else M^T, so that A A^T is the smaller h x h Gram."""
    M = np.asarray(M, dtype=np.float64)
    trans = M.shape[0] > M.shape[1]
    return (M.T if trans else M), trans


def normalise(A: np.ndarray, norm: str) -> Tuple[np.ndarray, float]:
    """Returns (X, s) with X = A / s.

    * ``frobenius``: s = ||A||_F, Eq. (constraint).
    * ``gram_frobenius``: s = ||A A^T||_F^(1/2), Eq. (new_scale_formula), i.e. the
      Gelfand scaling of Eq. (scale_formula_function) with q = 1.
    * ``none``: s = 1.
    A zero norm gives s = 0 and X = 0 (no epsilon is added)."""
    if norm == "frobenius":
        s = float(np.sqrt(np.sum(A * A)))
    elif norm == "gram_frobenius":
        T0 = A @ A.T
        s = float(np.sqrt(np.sqrt(np.sum(T0 * T0))))
    elif norm == "none":
        s = 1.0
    else:
        raise ValueError(norm)
    if s == 0.0:
        return np.zeros_like(A), 0.0
    return A / s, s


def _check_terms(exponents: Sequence[int], coeffs: Sequence[float]):
    e = [int(x) for x in exponents]
    if len(e) != len(coeffs) or not e:
        raise ValueError("exponents and coefficients must have the same nonzero length")
    for x in e:
        if x != 0 and (x & (x - 1)) != 0:
            raise ValueError("exponents must be 0 or powers of two")
    if any(b <= a for a, b in zip(e, e[1:])):
        raise ValueError("exponents must be strictly increasing")
    return e, [float(c) for c in coeffs]


def ifnso_parts(M: np.ndarray, exponents: Sequence[int], coeffs: Sequence[float],
                basis: str = "gram", norm: str = "frobenius") -> Dict[str, object]:
    """The polynomial Y = sum_k c_k B^{e_k} X, with its intermediates.

    * basis ``gram``: B = X X^T -- the learnable unified polynomial of
      Eq. (new_unified_formula_0) restricted to the sparse exponent set {0} u {2^j}
      of the term-selection section.
    * basis ``complement``: B = I - X X^T -- the constrained polynomial of
      Eq. (after_matrix_formula) / Eq. (generalized_matrix_formula); with the
      ``gram_frobenius`` norm, B is T_1 of the T_l sequence (Sec. 2.4).
    * powers B^{2^j} by repeated squaring, (B^{2^(j-1)})^2 (Sec. 2.4, squaring property).
    * Y = P X with P = sum_k c_k B^{e_k} and B^0 = I (Algorithm 1, aggregation)."""
    e, c = _check_terms(exponents, coeffs)
    if basis not in BASES:
        raise ValueError(basis)
    A, trans = orient(M)
    h = A.shape[0]
    X, s = normalise(A, norm)
    XXt = X @ X.T
    B = XXt if basis == "gram" else np.eye(h) - XXt
    powers = {0: np.eye(h), 1: B}
    p = 1
    while p < e[-1]:
        powers[2 * p] = powers[p] @ powers[p]
        p *= 2
    P = np.zeros((h, h))
    for ek, ck in zip(e, c):
        P = P + ck * powers[ek]
    Y = P @ X
    return {"A": A, "trans": trans, "X": X, "scale": s, "B": B, "powers": powers,
            "P": P, "Y": Y.T if trans else Y}


def ifnso(M: np.ndarray, exponents: Sequence[int], coeffs: Sequence[float],
          basis: str = "gram", norm: str = "frobenius") -> np.ndarray:
    """Y in M's orientation; see :func:`ifnso_parts`."""
    return ifnso_parts(M, exponents, coeffs, basis, norm)["Y"]


def paper_form(M: np.ndarray, w: Sequence[float]) -> np.ndarray:
    """The paper's own form of the method (Sec. 2.2, Eq. newnew_formula with the scale of
    Eq. new_scale_formula; Algorithm 1 computes it), evaluated spectrally instead of by repeated
    squaring: with A A^T = Q diag(lambda) Q^T and o = ||A A^T||_F, the polynomial in
    T_1 = I - A A^T / o acts on each eigenvalue, so
        Y = Q diag(1 + sum_l w_l (1 - lambda / o)^(2^(l-1))) Q^T A / sqrt(o).
    Returned in M's orientation; a zero input gives zero. The squaring route is
    :func:`ifnso` with :func:`paper_coeffs_to_terms` and the complement basis."""
    A, trans = orient(M)
    lam, Q = np.linalg.eigh(A @ A.T)
    o = float(np.sqrt(np.sum(lam * lam)))
    if o == 0.0:
        return np.zeros_like(np.asarray(M, dtype=np.float64))
    t = 1.0 - lam / o
    d = np.ones_like(t)
    for l, wl in enumerate(w, start=1):
        d = d + float(wl) * t ** (2 ** (l - 1))
    Y = (Q * d) @ (Q.T @ A) / math.sqrt(o)
    return Y.T if trans else Y


def paper_w_last_approx(w_head: Sequence[float], L: int) -> float:
    """Eq. (b_approximation) as used in Eq. (overall_polynomial):
    w_L = e^(1/2) (2^(L/2) - 1) - sum_{l<L} w_l."""
    return math.exp(0.5) * (2.0 ** (L / 2.0) - 1.0) - float(np.sum(w_head))


def paper_coeffs_to_terms(w: Sequence[float]):
    """Eq. (newnew_formula): Y = X + sum_{l=1}^{L} w_l (I - X X^T)^{2^(l-1)} X, as the
    (exponents, coefficients) of a complement-basis polynomial."""
    L = len(w)
    exps = [0] + [2 ** (l - 1) for l in range(1, L + 1)]
    return exps, [1.0] + [float(x) for x in w]


def classical_ns(M: np.ndarray, steps: int, abc: Sequence[float], normalise_input: bool = True) -> np.ndarray:
    """Newton-Schulz iteration with one odd quintic per step, Eq. (iteration_jordan):
    X_{k+1} = a X_k + b (X_k X_k^T) X_k + c (X_k X_k^T)^2 X_k, from X_0 = A / ||A||_F
    (Eq. (constraint)). (a, b, c) = (1.5, -0.5, 0) is the cubic of
    Eq. (one_iteration_matrix). Returned in M's orientation."""
    a, b, c = (float(x) for x in abc)
    A, trans = orient(M)
    X = normalise(A, "frobenius")[0] if normalise_input else A.copy()
    for _ in range(steps):
        G = X @ X.T
        X = a * X + b * (G @ X) + c * (G @ (G @ X))
    return X.T if trans else X


def orth_error(Y: np.ndarray) -> float:
    """Error metric of the experiment section: ||Y Y^T - I||_F, with Y taken in the h <= w
    orientation (so the identity is h x h)."""
    Z, _ = orient(Y)
    E = Z @ Z.T - np.eye(Z.shape[0])
    return float(np.sqrt(np.sum(E * E)))


def singular_value_map(sig_tilde: np.ndarray, exponents, coeffs, basis: str = "gram") -> np.ndarray:
    """Scalar form of the polynomial acting on each singular value of X:
    gram:       f(x) = sum_k c_k x^(2 e_k) x           (Eq. (new_unified_formula))
    complement: f(x) = sum_k c_k (1 - x^2)^(e_k) x     (Eq. (our_scalar_formula))."""
    x = np.asarray(sig_tilde, dtype=np.float64)
    e, c = _check_terms(exponents, coeffs)
    base = x * x if basis == "gram" else 1.0 - x * x
    out = np.zeros_like(x)
    for ek, ck in zip(e, c):
        out = out + ck * base ** ek
    return out * x


def closed_form(U: np.ndarray, sigma: np.ndarray, V: np.ndarray, exponents, coeffs,
                basis: str = "gram", norm: str = "frobenius") -> np.ndarray:
    """Exact result for M = U diag(sigma) V^T (U, V with orthonormal columns): the method
    acts on singular values only (the SVD argument of Eq. (N_fold) and what follows), so
    Y = U diag(f(sigma~)) V^T with sigma~ the singular values after normalisation."""
    s = np.asarray(sigma, dtype=np.float64)
    if norm == "frobenius":
        d = math.sqrt(float(np.sum(s * s)))
    elif norm == "gram_frobenius":
        d = math.sqrt(math.sqrt(float(np.sum(s ** 4))))
    else:
        d = 1.0
    st = s / d
    f = singular_value_map(st, exponents, coeffs, basis)
    return (U * f) @ V.T


def flops_ifnso(h: int, w: int, L: int) -> float:
    """Dense FLOP count of Algorithm 1: A A^T and Y' A (2 h^2 w each) plus L-1 squarings
    (2 h^3 each); aggregation is not counted."""
    return 4.0 * h * h * w + 2.0 * (L - 1) * h ** 3


def flops_ns(h: int, w: int, steps: int, long_products: int) -> float:
    """Dense FLOP count of ``steps`` NS steps, each with ``long_products`` products of an
    h x h by h x w (or h x w by w x h) shape (2 h^2 w each)."""
    return steps * long_products * 2.0 * h * h * w
