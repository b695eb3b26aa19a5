"""The named synthetic workloads (shapes, seeds, value distributions).

D0  the paper's Table 1 shapes: N(0,1) 128x128, 128x512, 128x1024, seed 0.
D1  one 256x512 float32 N(0,1) matrix, seed 0; exponents {0,1,2,4,8} with a seeded
    coefficient vector normalised to sum 1; classical quintic NS, 5 steps.
D2  4096x4096 (seed 1) and 14336x4096 (seed 2) built as U diag(sigma) V^T from Haar
    factors with sigma log-uniform on [1e-3, 1]; exponents {0,1,2,4,8,16}.
D3  the weight-gradient set of a synthetic 32-layer transformer (hidden 4096, GQA,
    SwiGLU): per layer Wq, Wo 4096x4096, Wk, Wv 1024x4096, gate, up 14336x4096,
    down 4096x14336; bfloat16 N(0, 0.02^2) plus a rank-16 part of Frobenius norm 0.5;
    seed 1000 + 7*layer + index.
D4  64 matrices 2048x8192, U diag(sigma) V^T with sigma_i = i^-1.5 (max 1), seed 3.
"""
from __future__ import annotations

import json
import os

import numpy as np

from .gen import uniform_np

__all__ = [
    "MUON_ABC", "CUBIC_ABC", "D1_EXPONENTS", "D2_EXPONENTS", "d1_coeffs", "LAYER_SHAPES",
    "d3_shapes", "d3_seed", "load_coeffs", "D4_SHAPE", "D4_BATCH", "d4_seed", "d4_sigma", "d2_sigma_np",
    "PAPER_L", "load_schedule",
]

# Muon's quintic coefficients, Eq. (iteration_jordan).
MUON_ABC = (3.4445, -4.7750, 2.0315)
# Classical cubic Newton-Schulz, Eq. (one_iteration_matrix): X <- 1.5 X - 0.5 (X X^T) X.
CUBIC_ABC = (1.5, -0.5, 0.0)

D1_EXPONENTS = (0, 1, 2, 4, 8)
D2_EXPONENTS = (0, 1, 2, 4, 8, 16)
PAPER_L = 14  # default polynomial depth of the ablation study

# (name, rows, cols) of one synthetic transformer layer's weight gradients
LAYER_SHAPES = (
    ("wq", 4096, 4096), ("wk", 1024, 4096), ("wv", 1024, 4096), ("wo", 4096, 4096),
    ("gate", 14336, 4096), ("up", 14336, 4096), ("down", 4096, 14336),
)

D4_SHAPE = (2048, 8192)
D4_BATCH = 64


def d1_coeffs(num_terms: int = len(D1_EXPONENTS), seed: int = 0) -> np.ndarray:
    """i.i.d. U(0,1) draws from stream 7 of ``seed``, divided by their sum (so sum = 1)."""
    c = uniform_np(seed, 7, num_terms)
    return c / c.sum()


def d3_shapes(layers: int = 32):
    return [(r, c) for _ in range(layers) for (_, r, c) in LAYER_SHAPES]


def d3_seed(layer: int, index: int) -> int:
    return 1000 + 7 * layer + index


def d2_sigma_np(r: int, seed: int) -> np.ndarray:
    """sigma_i = 10^U(-3, 0), stream 3 of ``seed``."""
    return 10.0 ** (-3.0 + 3.0 * uniform_np(seed, 3, r))


def d4_seed(index: int) -> int:
    """Generator seed of matrix `index` of the e4m3 workload's batch (base seed 3)."""
    return 3000 + index


def d4_sigma(r: int) -> np.ndarray:
    i = np.arange(1, r + 1, dtype=np.float64)
    return i ** -1.5


def load_coeffs(name: str = "gform_v1"):
    """Fixed coefficient vectors stored next to this module (written by the oracle's fit
    script). Returns (exponents, coefficients)."""
    path = os.path.join(os.path.dirname(__file__), "coeffs.json")
    with open(path) as f:
        d = json.load(f)[name]
    return tuple(d["exponents"]), np.array(d["coeffs"], dtype=np.float64)


def load_schedule(name: str):
    """Newton-Schulz step schedules stored next to this module (written by the oracle's
    script). Returns (list of (a, b, c) per step, gelfand_q)."""
    path = os.path.join(os.path.dirname(__file__), "coeffs.json")
    with open(path) as f:
        d = json.load(f)[name]
    return [tuple(float(v) for v in abc) for abc in d["schedule"]], int(d["gelfand_q"])
