"""FP64 oracle of the e4m3 compute mode (test infrastructure only).

The paper computes in full precision; the e4m3 mode is a production variant of its
method (Sec. 2.4's repeated squaring and Algorithm 1's aggregation, with low-precision
operands for the Gram and the squarings). This module states that variant exactly:

* OCP FP8 e4m3 ("e4m3fn"): 1 sign bit, 4 exponent bits with bias 7, 3 mantissa bits; no
  infinities; 0x7F / 0xFF are NaN; largest finite value 448 = 1.75 * 2^8; smallest normal
  2^-6; subnormals k * 2^-9. Rounding is to nearest, ties to even; magnitudes beyond 448
  saturate to 448.
* Per-tensor scale of an operand T from a maximum m: s = 2^e, e = floor(log2(448 / m))
  clamped to [-63, 63] (s = 1 for m = 0 or non-finite); the operand is e4m3(s T) / s. For A,
  m = max|A|. A stored power L = store(X X^T) (X = Q(A) for the Gram, X = Q(L_prev) for a
  squaring; L_prev is symmetric) is positive semi-definite before its bfloat16 rounding, so
  the largest magnitude of X X^T is its largest diagonal entry, the largest squared row norm
  of X; m is that value, known from X alone, so the power is quantised where it is formed.
  The rounding to bfloat16 can lift a stored value above m by at most 2^-8 relative, which
  the scaled maximum (at most 448 (1 + 2^-8)) absorbs: it still rounds to 448.
* Stored powers, their weighted sum P and the operands of the final product are bfloat16
  (8 significant bits, ties to even). Rounding is applied scale-free (on the significand),
  which is what the GPU's power-of-two rescaled levels see.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use this module.
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np

from .ifnso import _check_terms, orient

__all__ = [
    "E4M3_MAX", "e4m3_round", "e4m3_encode", "e4m3_decode", "e4m3_scale", "e4m3_quantize",
    "e4m3_quantize_with", "gram_row_max", "bf16_round", "ifnso_e4m3",
]

E4M3_MAX = 448.0


def e4m3_decode(codes) -> np.ndarray:
    """Values of e4m3 bit patterns (uint8): (-1)^s 2^(E-7) (1 + m/8) for E >= 1,
    (-1)^s 2^-6 (m/8) for E = 0; 0x7F and 0xFF are NaN."""
    c = np.asarray(codes, dtype=np.uint8).astype(np.int64)
    sign = np.where(c & 0x80, -1.0, 1.0)
    E = (c >> 3) & 0xF
    m = c & 0x7
    val = np.where(E == 0, np.ldexp(m / 8.0, -6), np.ldexp(1.0 + m / 8.0, E - 7))
    val = sign * val
    return np.where((c & 0x7F) == 0x7F, np.nan, val)


def e4m3_round(x) -> np.ndarray:
    """Nearest e4m3 value (ties to even), saturating at +-448; keeps the sign of zero."""
    x = np.asarray(x, dtype=np.float64)
    a = np.abs(x)
    m, e = np.frexp(a)                       # a = m 2^e, m in [0.5, 1)
    normal = np.ldexp(np.round(m * 16.0), e - 4)   # 4 significant bits
    sub = np.round(a * 512.0) / 512.0              # quantum 2^-9 below 2^-6
    r = np.where(a < 2.0 ** -6, sub, normal)
    r = np.minimum(r, E4M3_MAX)
    return np.copysign(r, x)


def e4m3_encode(x) -> np.ndarray:
    """Bit patterns (uint8) of e4m3_round(x)."""
    r = e4m3_round(x)
    a = np.abs(r)
    sign = np.signbit(r).astype(np.int64) << 7
    m, e = np.frexp(a)                       # a = m 2^e
    E = e + 6                                # biased exponent of a normal value (2m)(2^(e-1))
    mant_n = np.round((2.0 * m - 1.0) * 8.0).astype(np.int64)
    code_n = (E.astype(np.int64) << 3) | mant_n
    code_s = np.round(a * 512.0).astype(np.int64)   # subnormal: m/8 2^-6 = m 2^-9
    code = np.where(a < 2.0 ** -6, code_s, code_n)
    return (sign | code).astype(np.uint8)


def e4m3_scale(amax: float) -> float:
    """s = 2^floor(log2(448 / amax)), exponent clamped to [-63, 63]; 1 for amax <= 0 or non-finite."""
    amax = float(amax)
    if not (amax > 0.0) or not math.isfinite(amax):
        return 1.0
    e = math.floor(math.log2(E4M3_MAX / amax))
    # guard the floor against log2 rounding at exact powers of two
    while E4M3_MAX / amax < 2.0 ** e:
        e -= 1
    while E4M3_MAX / amax >= 2.0 ** (e + 1):
        e += 1
    return 2.0 ** max(-63, min(63, e))


def e4m3_quantize(T):
    """(e4m3(s T) / s, s) with the per-tensor scale of T."""
    T = np.asarray(T, dtype=np.float64)
    s = e4m3_scale(float(np.max(np.abs(T))) if T.size else 0.0)
    return e4m3_round(T * s) / s, s


def e4m3_quantize_with(T, m: float):
    """(e4m3(s T) / s, s) with the scale of the maximum m (e4m3_scale(m))."""
    T = np.asarray(T, dtype=np.float64)
    s = e4m3_scale(m)
    return e4m3_round(T * s) / s, s


def gram_row_max(X) -> float:
    """max_i sum_k X[i][k]^2: the largest diagonal entry of X X^T, which for this positive
    semi-definite product is also its largest magnitude."""
    X = np.asarray(X, dtype=np.float64)
    return float(np.max(np.sum(X * X, axis=1))) if X.size else 0.0


def bf16_round(x) -> np.ndarray:
    """Nearest value with 8 significant bits (ties to even), on the significand."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)
    return np.ldexp(np.round(m * 256.0) / 256.0, e)


def _identity(x):
    return np.asarray(x, dtype=np.float64)


def ifnso_e4m3(M, exponents: Sequence[int], coeffs: Sequence[float], norm: str = "frobenius",
               quantize=None, store=None) -> np.ndarray:
    """Gram-basis IFNSO with e4m3 operands for the Gram and the squarings.

    In the order of the method (Sec. 1 transposition, Sec. 2.4 squaring, Algorithm 1):
      A  = M or M^T (h <= w);  s_A = ||A||_F from the unquantised A (float64)
      X_1 = Q(A, max|A|);            L1 = store(X_1 X_1^T)        the Gram, unnormalised
      X_{l+1} = Q(L_l, rowmax(X_l)); L_{l+1} = store(X_{l+1} X_{l+1})   repeated squaring
      B^(2^(l-1)) = L_l / n^(2^l)                n = s_A (Frobenius), ||L1||_F^(1/2)
                                                 (Gram-Frobenius) or 1 (none)
      P  = store(sum_{e_k >= 1} c_k B^(e_k));  Y = (c_0 A + P A) / n
    Q(T, m) is the per-tensor e4m3 quantiser with the scale of the maximum m (e4m3_quantize_with),
    rowmax(X) = gram_row_max(X) the largest magnitude of X X^T (L_l = store(X_l X_l^T) with X_l
    symmetric for l >= 2), `store` the bfloat16 rounding of stored matrices. Both can be replaced
    (identity: the plain float64 polynomial); a replacement quantiser takes (T, m). Returns Y in
    M's orientation."""
    e, c = _check_terms(exponents, coeffs)
    Q = quantize if quantize is not None else (lambda T, m: e4m3_quantize_with(T, m)[0])
    store = store if store is not None else bf16_round
    A, trans = orient(M)
    h = A.shape[0]
    X = Q(A, float(np.max(np.abs(A))) if A.size else 0.0)
    levels = {1: store(X @ X.T)}
    J = 0
    while (1 << J) < e[-1]:
        J += 1
    for l in range(1, J + 1):
        X = Q(levels[l], gram_row_max(X))
        levels[l + 1] = store(X @ X)
    if norm == "frobenius":
        n = math.sqrt(float(np.sum(A * A)))
    elif norm == "gram_frobenius":
        n = math.sqrt(math.sqrt(float(np.sum(levels[1] * levels[1]))))
    elif norm == "none":
        n = 1.0
    else:
        raise ValueError(norm)
    if n == 0.0:
        Y = np.zeros_like(A)
        return Y.T if trans else Y
    P = np.zeros((h, h))
    c0 = 0.0
    for ek, ck in zip(e, c):
        if ek == 0:
            c0 = ck
            continue
        l = ek.bit_length()                   # e_k = 2^(l-1) lives in level l
        P = P + ck * (levels[l] / n ** (2 ** l))
    P = store(P)
    Y = (c0 * A + P @ A) / n
    return Y.T if trans else Y
