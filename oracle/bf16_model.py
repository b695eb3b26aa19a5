"""Float64 models of the bfloat16 storage points of the library's bf16 paths (test
infrastructure only).

Each model runs one path of the method in float64 and rounds to bfloat16 exactly where that
path stores a bfloat16 value, and nowhere else. Its distance to the exact polynomial
(:func:`oracle.ifnso`, :func:`oracle.baselines.ns_schedule`, the closed forms) is the error that
the storage points alone introduce; the tolerances of the bf16 parity tests are set from it,
and ``tests/test_oracle_bounds.py`` recomputes every one of them. The float32 accumulation of
the device adds a far smaller error (2^-24 per addition, against 2^-9 per stored value), except
where very large coefficients amplify it: the split model therefore offers float32 products
too (``accum=np.float32``).

What is stored where (the paths of the method, Sec. 1 orientation and normalisation, Sec. 2.4
repeated squaring, Algorithm 1 aggregation and product):

* Gram basis, level layout (bf16 plans, :func:`gram_levels`): the input A (bf16), each stored
  power L_1 = A A^T, L_{l+1} = L_l L_l (bf16; a power-of-two rescaling of a level does not
  change its rounding), the weighted sum P (bf16) and the output. The last squaring's own
  product enters P before any rounding (its aggregation is folded into it). With J = 0 the
  product reads the stored Gram itself.
* Newton-Schulz steps on the generic kernels (:func:`ns_generic`): per step the Gram G_k of
  the iterate (kept in float32 and stored as a bf16 operand), B_k = b G_k + c G_k^2 with G_k^2
  formed from the bf16 operand (stored bf16), and the iterate X_{k+1} = a X_k + B_k X_k
  (stored bf16).
* Newton-Schulz steps as chained Gram-basis plans (:func:`ns_chained`): each step is one
  level-layout evaluation with exponents {0, 1, 2} (or {0, 1}), the first one normalised, and
  its output (the next iterate) stored in bf16.
* Complement basis with split operands (:func:`complement_split`): every squaring operand and
  P are stored as a pair hi = bf16(x), lo = bf16(x - hi); a squaring forms
  hi hi + hi lo + lo hi (lo lo dropped); D_l = T^(2^(l-1)) - I is carried in that pair.
* Vectors (h = 1): the scalar Gram is exact, the polynomial is evaluated in float64 and only
  the output (or each chained iterate) is rounded.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use this module.
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np

from .fp8 import bf16_round
from .ifnso import _check_terms, orient

__all__ = ["gram_levels", "gram_traces", "ns_generic", "ns_chained", "complement_split", "split_pair"]


def _identity(x):
    return np.asarray(x, dtype=np.float64)


def _scale(A: np.ndarray, G: np.ndarray, norm: str) -> float:
    if norm == "frobenius":
        return math.sqrt(float(np.sum(A * A)))
    if norm == "gram_frobenius":
        return math.sqrt(math.sqrt(float(np.sum(G * G))))
    if norm == "none":
        return 1.0
    raise ValueError(norm)


def gram_levels(M, exponents: Sequence[int], coeffs: Sequence[float], norm: str = "frobenius",
                out_bf16: bool = True, store=bf16_round, split_p: bool = False) -> np.ndarray:
    """Gram-basis polynomial Y = sum_k c_k (X X^T)^(e_k) X with the bf16 plans' storage points
    (module docstring). M holds the input values as the device reads them. ``split_p``: P is
    stored as a split pair hi + lo (IFNSO_FLAG_SPLIT_P) instead of one bf16 value. Returns Y in
    M's orientation."""
    e, c = _check_terms(exponents, coeffs)
    r_out = store if out_bf16 else _identity
    A, trans = orient(M)
    h = A.shape[0]
    G = A @ A.T
    n = _scale(A, G, norm)
    if n == 0.0:
        Y = np.zeros_like(A)
        return Y.T if trans else Y
    J = 0
    while (1 << J) < e[-1]:
        J += 1
    if h == 1:  # the scalar Gram is exact; the polynomial is evaluated in float64
        g = float(G[0, 0]) / (n * n)
        v = sum(ck * g ** ek for ek, ck in zip(e, c))
        Y = r_out(v * A / n)
        return Y.T if trans else Y
    # levels: B^(2^(l-1)) = L_l / n^(2^l); only the powers the polynomial uses enter P
    L = {1: store(G)}
    last = None
    for l in range(1, J + 1):
        prod = L[l] @ L[l]
        if l < J:
            L[l + 1] = store(prod)
        else:
            last = prod  # the last squaring's product enters P unrounded
    c0 = 0.0
    P = np.zeros((h, h))
    for ek, ck in zip(e, c):
        if ek == 0:
            c0 = ck
            continue
        l = ek.bit_length()
        lev = last if (l == J + 1 and J >= 1) else L[l]
        P = P + ck * lev / n ** (2 ** l)
    if J >= 1:
        P = sum(split_pair(P, store)) if split_p else store(P)
    # J = 0: the product reads the stored Gram (already rounded)
    Y = r_out((c0 * A + P @ A) / n)
    return Y.T if trans else Y


def ns_generic(M, schedule: Sequence[Sequence[float]], gelfand_q: int = 0, store=bf16_round) -> np.ndarray:
    """Newton-Schulz with one (a, b, c) per step on the generic kernels, with their bf16 storage
    points (module docstring). X_0 = A / s, s from Eq. (constraint) (q = 0) or Gelfand's bound
    (q = 1: from the float32 Gram; q = 2: from the square of its bf16 operand)."""
    A, trans = orient(M)
    h = A.shape[0]
    G = A @ A.T
    if gelfand_q == 0:
        s = math.sqrt(float(np.sum(A * A)))
    elif gelfand_q == 1:
        s = math.sqrt(math.sqrt(float(np.sum(G * G))))
    elif gelfand_q == 2:
        G2 = store(G) @ store(G)
        s = float(np.sum(G2 * G2)) ** 0.125
    else:
        raise ValueError("gelfand_q in {0, 1, 2}")
    if s == 0.0:
        Y = np.zeros_like(A)
        return Y.T if trans else Y
    if h == 1:  # scalar recursion in float64 over the whole schedule, one rounding at the end
        x = math.sqrt(float(G[0, 0])) / s
        for a, b, c in schedule:
            x = x * (a + x * x * (b + c * x * x))
        Y = store(A * (x / math.sqrt(float(G[0, 0]))))
        return Y.T if trans else Y
    X = A / s
    for k, (a, b, c) in enumerate(schedule):
        Gk = G / (s * s) if k == 0 else X @ X.T
        Gop = store(Gk)
        B = store(b * Gk + c * (Gop @ Gop))
        X = store(a * X + B @ X)
    return X.T if trans else X


def ns_chained(M, schedule: Sequence[Sequence[float]], gelfand_q: int = 0, store=bf16_round) -> np.ndarray:
    """Newton-Schulz steps as chained Gram-basis plans on the batched path: step k is
    :func:`gram_levels` with exponents {0, 1, 2} (or {0, 1} when c = 0), normalised by
    ||A||_F (q = 0) or ||A A^T||_F^(1/2) (q = 1) at the first step and not at all later; every
    iterate is stored in bf16."""
    if gelfand_q not in (0, 1):
        raise ValueError("chained schedules scale with q = 0 or 1")
    X = np.asarray(M, dtype=np.float64)
    for k, (a, b, c) in enumerate(schedule):
        norm = ("frobenius" if gelfand_q == 0 else "gram_frobenius") if k == 0 else "none"
        exps, co = ((0, 1), (a, b)) if c == 0.0 else ((0, 1, 2), (a, b, c))
        X = gram_levels(X, exps, co, norm=norm, out_bf16=True, store=store)
    return X


def split_pair(x, store=bf16_round):
    """(hi, lo) with hi = bf16(x) and lo = bf16(x - hi)."""
    hi = store(x)
    return hi, store(np.asarray(x, dtype=np.float64) - hi)


def complement_split(M, exponents: Sequence[int], coeffs: Sequence[float], norm: str = "gram_frobenius",
                     accum=np.float64, store=bf16_round) -> np.ndarray:
    """Complement-basis polynomial Y = sum_k c_k (I - X X^T)^(e_k) X with split bf16 operands
    (module docstring): D_1 = -X X^T, D_{l+1} = 2 D_l + D_l^2 (T = I + D), P = sum_{k>=1} c_k
    D_{e_k} carried as a split pair, Y = (sum_k c_k) X + P X. ``accum=np.float32`` evaluates the
    matrix products in float32 (the device's accumulation type; the operands are exact in it).
    ``accum="f32seq"`` also rounds every value the kernels keep in float32 (the Gram, D_l, the
    running sum P) and sums each product in float32 along K, one rounding per 16 products into
    one accumulator over the concatenated K (hi hi, then hi lo, then lo hi), as a matrix-core
    accumulator does; the order inside a step is not modelled.
    Returns Y in M's orientation (float32 output)."""
    e, c = _check_terms(exponents, coeffs)
    A, trans = orient(M)
    h = A.shape[0]
    seq = isinstance(accum, str) and accum == "f32seq"

    def r32(x):  # a float32 store (f32seq only; the other modes keep float64)
        return np.asarray(x, dtype=np.float32).astype(np.float64) if seq else x

    def mm(*pairs):
        """sum of x @ y over the pairs: one accumulation over the concatenated K"""
        if seq:
            acc = np.zeros((pairs[0][0].shape[0], pairs[0][1].shape[1]))
            for x, y in pairs:
                for k0 in range(0, x.shape[1], 16):
                    acc = r32(acc + x[:, k0:k0 + 16] @ y[k0:k0 + 16, :])
            return acc
        return sum((x.astype(accum) @ y.astype(accum)).astype(np.float64) for x, y in pairs)

    G = mm((A, A.T)) if seq else A @ A.T
    n = _scale(A, G, norm)
    if n == 0.0:
        Y = np.zeros_like(A)
        return Y.T if trans else Y
    csum = float(sum(c))
    if h == 1:
        g = 1.0 - float(G[0, 0]) / (n * n)
        v = sum(ck * g ** ek for ek, ck in zip(e, c))
        Y = v * A / n
        return Y.T if trans else Y
    J = 0
    while (1 << J) < e[-1]:
        J += 1
    coef = {ek: ck for ek, ck in zip(e, c)}
    D = r32(-G / (n * n))                      # D_1 from the float32 Gram
    P = r32(coef.get(1, 0.0) * D)
    op = split_pair(G, store)                  # the Gram operand, split
    for l in range(1, J + 1):
        hi, lo = op
        sq = mm((hi, hi), (hi, lo), (lo, hi))
        if l == 1:
            sq = sq / (n * n) ** 2
            Dl = D
        else:
            Dl = hi + lo                       # D_l read back from its split operand
        D = r32(2.0 * Dl + sq)
        P = r32(P + coef.get(1 << l, 0.0) * D)
        op = split_pair(D, store)
    if J >= 1:
        ph, pl = split_pair(P, store)
    else:  # no squaring: the product reads c_1 D_1 from the split Gram operand
        w1 = -coef.get(1, 0.0) / (n * n)
        ph, pl = w1 * op[0], w1 * op[1]
    Y = (csum * A + mm((ph, A), (pl, A))) / n
    return Y.T if trans else Y


def gram_traces(M, levels: int = 8, store=bf16_round) -> np.ndarray:
    """log2 of the normalised traces m_j = tr(G^(2^j)) / h, j = 0..levels-1, of G = X X^T with
    X = A / ||A||_F, as the learned bf16 plans obtain them: each level is squared from its bf16
    operand, the trace of a level is taken from its product before rounding, and the last value
    is the sum of squares of the last level (tr(G^(2^(k+1))) = ||G^(2^k)||_F^2). A level is
    rescaled by 2^-round(log2 of its sum of squares) before it is stored, which leaves its
    rounding unchanged and keeps every value in range; the scales are carried in log2."""
    A, _ = orient(M)
    h = A.shape[0]
    out = np.empty(levels)
    cur = A @ A.T                                 # level 1 = ||A||_F^2 G
    l2s = -math.log2(float(np.sum(A * A)))        # log2 of (power / level)
    for j in range(levels - 1):
        out[j] = l2s + math.log2(float(np.trace(cur))) - math.log2(h)
        ss = float(np.sum(cur * cur))
        if j == levels - 2:
            out[j + 1] = 2.0 * l2s + math.log2(ss) - math.log2(h)
            break
        e = round(math.log2(ss))
        op = store(cur)
        cur = (op @ op) * 2.0 ** (-e)
        l2s = 2.0 * l2s + e
    return out
