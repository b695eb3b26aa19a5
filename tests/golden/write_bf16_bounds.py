"""Writes bf16_bounds.json: the float64 bf16 storage-point model's errors on the full-size parity
inputs, which are too large to recompute in the CPU test suite (about two minutes here).

Every value comes from oracle.bf16_model and the oracle's closed forms on the inputs that the GPU
tests build (workloads generators, same seeds): the relative Frobenius distance of the model's
result to the exact one. tests/test_oracle_bounds.py checks that each GPU tolerance lies between
three and four times the largest value it covers, and recomputes the 4096 x 4096 entry.

Usage: python tests/golden/write_bf16_bounds.py (from the repository root).
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import baselines as BL, bf16_model as BM  # noqa: E402
from workloads import configs, gen  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bf16_bounds.json")
D4_SAMPLED = [0, 21, 42, 63]
# (layer, index) of the gradient-set matrices the full-size test samples: Wq and Wk of layer 0,
# gate (tall) and down (wide) of layer 31
D3_SAMPLED = [(0, 0), (0, 1), (31, 4), (31, 6)]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def d2_schedule_case(rows, cols, seed):
    """Muon's five steps as chained bf16 plans on one matrix of the FP32-versus-BF16 pair."""
    sched, _ = configs.load_schedule("muon_ns5")
    sigma = configs.d2_sigma_np(min(rows, cols), seed)
    M, U, V = gen.spectral_np(rows, cols, sigma, seed)
    f = BL.compose_scalar(sigma / np.sqrt(np.sum(sigma ** 2)), sched)
    Yc = (U * f) @ V.T
    return _rel(BM.ns_chained(gen.round_to_bf16_np(M), sched, 0), Yc)


def d4_case(i):
    """One matrix of the heavy-tailed batch through the bf16 Gram-basis plan (gform_v1)."""
    exps, c = configs.load_coeffs("gform_v1")
    rows, cols = configs.D4_SHAPE
    sigma = configs.d4_sigma(min(rows, cols))
    M, U, V = gen.spectral_np(rows, cols, sigma, configs.d4_seed(i))
    Mb = gen.round_to_bf16_np(M)
    Ym = BM.gram_levels(Mb, exps, c)
    return _rel(Ym, oracle.closed_form(U, sigma, V, exps, c)), _rel(Ym, oracle.ifnso(Mb, exps, c))


def d3_case(layer, index):
    """One matrix of the gradient set (numpy twin of the device generator, rounded to bf16)
    through the bf16 Gram-basis plan (gform_v1), against the polynomial of the same input."""
    exps, c = configs.load_coeffs("gform_v1")
    _, rows, cols = configs.LAYER_SHAPES[index]
    Mb = gen.round_to_bf16_np(gen.lowrank_plus_noise_np(rows, cols, configs.d3_seed(layer, index)))
    return _rel(BM.gram_levels(Mb, exps, c), oracle.ifnso(Mb, exps, c))


def main():
    out = {"d2_schedule_muon_ns5": {}, "d4_gform_v1_closed": {}, "d4_gform_v1_oracle": {},
           "d3_gform_v1_oracle": {}}
    for rows, cols, seed in [(4096, 4096, 1), (14336, 4096, 2)]:
        out["d2_schedule_muon_ns5"][f"{rows}x{cols}"] = d2_schedule_case(rows, cols, seed)
        print(rows, cols, out["d2_schedule_muon_ns5"][f"{rows}x{cols}"], flush=True)
    for i in D4_SAMPLED:
        rc, ro = d4_case(i)
        out["d4_gform_v1_closed"][str(i)] = rc
        out["d4_gform_v1_oracle"][str(i)] = ro
        print(i, rc, ro, flush=True)
    for layer, index in D3_SAMPLED:
        out["d3_gform_v1_oracle"][f"{layer}/{index}"] = d3_case(layer, index)
        print(layer, index, out["d3_gform_v1_oracle"][f"{layer}/{index}"], flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
