"""Counter-based random inputs with a host (numpy) and a device (torch) twin.

Generator definition (the same on both sides):

* ``mix64`` is the SplitMix64 output function (Steele, Lea and Flood, 2014):
  ``z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27; z *= 0x94D049BB133111EB;
  z ^= z >> 31`` on 64-bit unsigned integers (wrapping arithmetic).
* ``key(seed, stream) = mix64(seed ^ mix64(stream + GAMMA))``.
* the i-th 64-bit word of a stream is ``mix64(key + (i + 1) * GAMMA)``.
* a uniform is ``(word >> 11) * 2**-53`` in [0, 1).
* normals come from Box-Muller over consecutive pairs:
  ``r = sqrt(-2 ln(1 - u[2j]))``, ``z[2j] = r cos(2 pi u[2j+1])``,
  ``z[2j+1] = r sin(2 pi u[2j+1])``, computed in float64.

Storage rounding is round-to-nearest-even from float64, done on the bit
pattern so that float64 -> bfloat16 rounds once (no float32 double rounding).

The integer stream is bit-identical on both sides. The transcendental steps
(log, cos, sin) may differ by an ulp between numpy and the device, so a test
that compares device results with the oracle hands the oracle the very bytes
the device consumed.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_MASK64 = (1 << 64) - 1

__all__ = [
    "mix64_np", "stream_key", "uniform_np", "normal_np", "round_to_bf16_np",
    "bf16_bits_to_f32_np", "f32_to_bf16_bits_np", "gaussian_np", "haar_np",
    "spectral_np", "uniform_torch", "normal_torch", "round_to_bf16_torch",
    "gaussian_torch", "haar_torch", "spectral_torch", "lowrank_plus_noise_torch",
    "lowrank_plus_noise_np", "fan_in_uniform_np",
]


# ----------------------------------------------------------------------------------------------
# host (numpy)
# ----------------------------------------------------------------------------------------------
def mix64_np(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(_M1)
        z ^= z >> np.uint64(27)
        z *= np.uint64(_M2)
        z ^= z >> np.uint64(31)
    return z


def _mix64_int(z: int) -> int:
    z &= _MASK64
    z ^= z >> 30
    z = (z * _M1) & _MASK64
    z ^= z >> 27
    z = (z * _M2) & _MASK64
    z ^= z >> 31
    return z


def stream_key(seed: int, stream: int) -> int:
    return _mix64_int((seed & _MASK64) ^ _mix64_int((stream + GAMMA) & _MASK64))


def _words_np(seed: int, stream: int, n: int, offset: int = 0) -> np.ndarray:
    key = np.uint64(stream_key(seed, stream))
    idx = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        ctr = key + idx * np.uint64(GAMMA)
    return mix64_np(ctr)


def uniform_np(seed: int, stream: int, n: int, offset: int = 0) -> np.ndarray:
    w = _words_np(seed, stream, n, offset)
    return (w >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal_np(seed: int, stream: int, n: int) -> np.ndarray:
    m = (n + 1) // 2
    u = uniform_np(seed, stream, 2 * m)
    r = np.sqrt(-2.0 * np.log1p(-u[0::2]))
    t = 2.0 * math.pi * u[1::2]
    z = np.empty(2 * m, dtype=np.float64)
    z[0::2] = r * np.cos(t)
    z[1::2] = r * np.sin(t)
    return z[:n]


def round_to_bf16_np(x: np.ndarray) -> np.ndarray:
    """float64 -> nearest-even bfloat16 value, returned as float64 (exact)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    b = x.view(np.uint64).copy()
    lsb = (b >> np.uint64(45)) & np.uint64(1)
    with np.errstate(over="ignore"):
        b += np.uint64((1 << 44) - 1) + lsb
    b &= np.uint64(~((1 << 45) - 1) & _MASK64)
    return b.view(np.float64)


def f32_to_bf16_bits_np(x32: np.ndarray) -> np.ndarray:
    """float32 values that are already bfloat16-representable -> uint16 bit patterns."""
    return (np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32) >> np.uint32(16)).astype(np.uint16)


def bf16_bits_to_f32_np(bits: np.ndarray) -> np.ndarray:
    return (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


def gaussian_np(rows: int, cols: int, seed: int, stream: int = 0, std: float = 1.0) -> np.ndarray:
    return (std * normal_np(seed, stream, rows * cols)).reshape(rows, cols)


def haar_np(n: int, k: int, seed: int, stream: int) -> np.ndarray:
    """n x k matrix with orthonormal columns: QR of a Gaussian matrix with the sign of
    diag(R) folded into Q (Mezzadri's correction), so Q is Haar distributed."""
    z = gaussian_np(n, k, seed, stream)
    q, r = np.linalg.qr(z)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d


def spectral_np(rows: int, cols: int, sigma: np.ndarray, seed: int):
    """M = U diag(sigma) V^T with Haar U (rows x r), V (cols x r), r = min(rows, cols).
    Returns (M, U, V) in float64."""
    r = min(rows, cols)
    assert sigma.shape == (r,)
    u = haar_np(rows, r, seed, 1)
    v = haar_np(cols, r, seed, 2)
    return (u * sigma) @ v.T, u, v


def lowrank_plus_noise_np(rows: int, cols: int, seed: int, std: float = 0.02,
                          rank: int = 16, lr_norm: float = 0.5) -> np.ndarray:
    """std * N(0,1) noise plus Z1 Z2 scaled to Frobenius norm ``lr_norm`` (float64)."""
    noise = gaussian_np(rows, cols, seed, 0, std)
    z1 = gaussian_np(rows, rank, seed, 1)
    z2 = gaussian_np(rank, cols, seed, 2)
    r = z1 @ z2
    return noise + r * (lr_norm / np.linalg.norm(r))


# ----------------------------------------------------------------------------------------------
# device twin (torch); imported lazily so that the CPU-only paths never need torch
# ----------------------------------------------------------------------------------------------
def _s64(c: int) -> int:
    """unsigned 64-bit constant -> the int64 with the same bit pattern."""
    c &= _MASK64
    return c - (1 << 64) if c >= (1 << 63) else c


def _lshr(t, k: int):
    import torch
    return (t >> k) & torch.tensor((1 << (64 - k)) - 1, dtype=torch.int64, device=t.device)


def _mix64_torch(z):
    z = z ^ _lshr(z, 30)
    z = z * _s64(_M1)
    z = z ^ _lshr(z, 27)
    z = z * _s64(_M2)
    z = z ^ _lshr(z, 31)
    return z


def uniform_torch(seed: int, stream: int, n: int, device, offset: int = 0):
    import torch
    key = _s64(stream_key(seed, stream))
    idx = torch.arange(offset + 1, offset + n + 1, dtype=torch.int64, device=device)
    ctr = idx * _s64(GAMMA) + key
    w = _mix64_torch(ctr)
    return _lshr(w, 11).to(torch.float64) * (2.0 ** -53)


def normal_torch(seed: int, stream: int, n: int, device):
    import torch
    m = (n + 1) // 2
    u = uniform_torch(seed, stream, 2 * m, device).view(m, 2)
    r = torch.sqrt(-2.0 * torch.log1p(-u[:, 0]))
    t = (2.0 * math.pi) * u[:, 1]
    z = torch.stack((r * torch.cos(t), r * torch.sin(t)), dim=1).reshape(-1)
    return z[:n]


def round_to_bf16_torch(x):
    """float64 tensor -> bfloat16 tensor, rounding once to nearest-even."""
    import torch
    b = x.contiguous().view(torch.int64)
    lsb = (b >> 45) & 1
    b = (b + ((1 << 44) - 1) + lsb) & _s64(~((1 << 45) - 1))
    f32 = b.view(torch.float64).to(torch.float32)  # exact
    hi = (f32.view(torch.int32) >> 16).to(torch.int16)
    return hi.view(torch.bfloat16)


def gaussian_torch(rows: int, cols: int, seed: int, stream: int = 0, std: float = 1.0, device="cuda"):
    return (std * normal_torch(seed, stream, rows * cols, device)).view(rows, cols)


def haar_torch(n: int, k: int, seed: int, stream: int, device="cuda"):
    import torch
    z = gaussian_torch(n, k, seed, stream, device=device)
    q, r = torch.linalg.qr(z)
    d = torch.sign(torch.diagonal(r))
    d[d == 0] = 1.0
    return q * d


def spectral_torch(rows: int, cols: int, sigma, seed: int, device="cuda"):
    import torch
    r = min(rows, cols)
    sigma = torch.as_tensor(sigma, dtype=torch.float64, device=device)
    u = haar_torch(rows, r, seed, 1, device)
    v = haar_torch(cols, r, seed, 2, device)
    return (u * sigma) @ v.T.contiguous(), u, v


def lowrank_plus_noise_torch(rows: int, cols: int, seed: int, std: float = 0.02, rank: int = 16,
                             lr_norm: float = 0.5, device="cuda"):
    import torch
    noise = gaussian_torch(rows, cols, seed, 0, std, device)
    z1 = gaussian_torch(rows, rank, seed, 1, device=device)
    z2 = gaussian_torch(rank, cols, seed, 2, device=device)
    r = z1 @ z2
    return noise + r * (lr_norm / torch.linalg.norm(r))


def fan_in_uniform_np(seed: int, layout) -> np.ndarray:
    """Initial parameters of a layered network, flattened in `layout` order (a list of
    (name, shape)): a weight (name starting with "W", shape (out, in)) is drawn
    U(-1/sqrt(in), 1/sqrt(in)) from stream 100 + its position in `layout`; a bias is zero.
    float64."""
    parts = []
    for i, (name, shape) in enumerate(layout):
        n = int(np.prod(shape))
        if name.startswith("W"):
            bound = 1.0 / math.sqrt(shape[1])
            parts.append((2.0 * uniform_np(seed, 100 + i, n) - 1.0) * bound)
        else:
            parts.append(np.zeros(n))
    return np.concatenate(parts)
