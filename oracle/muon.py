"""FP64 oracle of one Muon optimizer step around the orthogonalisation (test infrastructure only).

The paper presents IFNSO as the orthogonalisation step of the Muon optimizer (Sec. 1: Muon
orthogonalises momentum updates, and Eq. (iteration_jordan) is Muon's Newton-Schulz map), but
it does not restate Muon's update. The reading used here, for one weight matrix W (rows x
cols) with gradient G and momentum buffer B:

    B' = mu B + G                                  momentum
    U  = G + mu B'   (Nesterov)   or   U = B'       input of the orthogonalisation
    O  = IFNSO(q(U))                               q: the storage rounding of the input
    W' = (1 - lr wd) W - lr s O,   s = sqrt(max(1, rows / cols))

with decoupled weight decay wd and the shape factor s that keeps the update's RMS per entry
independent of the aspect ratio (O has orthonormal rows for wide W, orthonormal columns for
tall W). The polynomial, basis and normalisation of IFNSO are the plan's.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use this module.
"""
from __future__ import annotations

import math
from typing import Callable, Optional, Sequence

import numpy as np

from .ifnso import ifnso

__all__ = ["muon_scale", "muon_step"]


def muon_scale(rows: int, cols: int) -> float:
    """s = sqrt(max(1, rows / cols))."""
    return math.sqrt(max(1.0, rows / cols))


def muon_step(W, G, B, exponents: Sequence[int], coeffs: Sequence[float], lr: float, momentum: float,
              weight_decay: float = 0.0, nesterov: bool = True, basis: str = "gram", norm: str = "frobenius",
              round_input: Optional[Callable] = None):
    """One step; returns (W', B', O). All arithmetic in float64; `round_input` (for example
    a bfloat16 rounding) is applied to U before the orthogonalisation, as the device stores U
    in the plan's input type."""
    W = np.asarray(W, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    B1 = momentum * B + G
    U = G + momentum * B1 if nesterov else B1
    if round_input is not None:
        U = round_input(U)
    O = ifnso(U, exponents, coeffs, basis, norm)
    W1 = (1.0 - lr * weight_decay) * W - lr * muon_scale(*W.shape) * O
    return W1, B1, O
