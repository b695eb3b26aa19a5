"""The bf16 storage-point models (oracle/bf16_model.py) and every GPU tolerance derived from them.

First the models are pinned: with the rounding replaced by the identity each one is the exact
method (the oracle's polynomial, the Newton-Schulz iteration, the traces of the Gram powers);
with bf16 rounding each stays within the per-value bound that 8 significant bits allow on a
case small enough to check by hand. Then each bf16 tolerance of the GPU tests is recomputed:
the model is run on exactly the inputs the GPU test builds, and the tolerance must lie between
three and four times the largest model error among the cases it covers. A tolerance that was
loosened without the model's support, or left far above it, fails here.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import baselines as BL, bf16_model as BM
from oracle.fp8 import bf16_round
from workloads import configs, gen

import test_gpu_baselines as TB
import test_gpu_fullsize as TF
import test_gpu_parity as TP
import test_gpu_split as TS
import test_gpu_stages as TG

IDENT = (lambda x: np.asarray(x, dtype=np.float64))


def _rel(a, b):
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b)) / nb if nb > 0 else float(np.linalg.norm(a))


def _within(tol, m):
    assert 3.0 * m <= tol <= 4.0 * m, (tol, m, tol / m)


# ---------------------------------------------------------------------------------------------
# the models themselves
# ---------------------------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(40, 90), (90, 40), (1, 30)])
def test_models_without_rounding_are_exact(shape):
    M = gen.gaussian_np(*shape, seed=3)
    for exps, c in [((0, 1, 2, 4, 8), (0.4, 0.3, 0.15, 0.1, 0.05)), ((0, 1), (1.5, -0.5)), ((1,), (1.0,))]:
        for norm in ("frobenius", "gram_frobenius", "none"):
            assert _rel(BM.gram_levels(M, exps, c, norm, store=IDENT), oracle.ifnso(M, exps, c, "gram", norm)) < 1e-12
        for norm in ("frobenius", "gram_frobenius"):
            Yc = oracle.ifnso(M, exps, c, "complement", norm)
            assert _rel(BM.complement_split(M, exps, c, norm, store=IDENT), Yc) < 1e-12
    for name in ("muon_ns5", "cans_ns5_q2", "original_ns8"):
        sched, q = configs.load_schedule(name)
        assert _rel(BM.ns_generic(M, sched, q, store=IDENT), BL.ns_schedule(M, sched, q)) < 1e-12
        assert _rel(BM.ns_chained(M, sched, min(q, 1), store=IDENT), BL.ns_schedule(M, sched, min(q, 1))) < 1e-12
    sig = np.linalg.svd(M, compute_uv=False)
    l2m = oracle.features_from_spectrum(sig) * 8 * 2.0 ** np.arange(8)
    assert np.max(np.abs(BM.gram_traces(M, store=IDENT) - l2m)) < 1e-9


def test_bf16_rounding_and_split_pair():
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, -3.0 - 2.0 ** -7, 2.0 ** -140 * 1.3])
    r = bf16_round(x)
    # 8 significant bits: the spacing just above 1 is 2^-7; ties go to the even neighbour
    assert bf16_round(1.0 + 2.0 ** -8) == 1.0
    assert bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x))
    hi, lo = BM.split_pair(x)
    assert np.all(np.abs(hi + lo - x) <= 2.0 ** -16 * np.abs(x))


# ---------------------------------------------------------------------------------------------
# the GPU tolerances
# ---------------------------------------------------------------------------------------------
def test_classical_ns_bound():
    m = 0.0
    for shape in TP.NS_SHAPES:
        M = gen.round_to_bf16_np(gen.gaussian_np(*shape, seed=0))
        for steps in TP.NS_STEPS:
            m = max(m, _rel(BM.ns_generic(M, [configs.MUON_ABC] * steps, 0),
                            oracle.classical_ns(M, steps, configs.MUON_ABC)))
    _within(TP.TOL_NS["bf16"], m)


@pytest.mark.parametrize("name", TB.SCHEDULES)
def test_schedule_bounds(name):
    sched, q = configs.load_schedule(name)
    m = 0.0
    for shape in TB.BF16_SHAPES:
        M = gen.round_to_bf16_np(gen.gaussian_np(*shape, seed=0))
        m = max(m, _rel(BM.ns_generic(M, sched, q), BL.ns_schedule(M, sched, q)))
    m_h1 = 0.0
    for bname, bq in TB.BATCHED_CASES:
        if bname != name:
            continue
        for i, shape in enumerate(TB.BATCHED_SHAPES):
            M = gen.round_to_bf16_np(gen.gaussian_np(*shape, seed=40 + i))
            r = _rel(BM.ns_chained(M, sched, bq), BL.ns_schedule(M, sched, bq))
            if min(shape) == 1:
                m_h1 = max(m_h1, r)
            else:
                m = max(m, r)
    if name == "muon_ns5":
        for shape in TB.LONG_SHAPES:
            M = gen.round_to_bf16_np(gen.gaussian_np(*shape, seed=21))
            m = max(m, _rel(BM.ns_generic(M, sched, q), BL.ns_schedule(M, sched, q)))
    _within(TB.TOL_BF16[name], m)
    _within(TB.TOL_BF16_H1[name], m_h1)


def test_split_bound():
    """Depth 14 with split operands: the bound rests on the device's measured deviation (see
    tests/test_gpu_split.py); here it must stay at least three times the storage-point model and
    within the bf16 path's 2e-2."""
    exps, c = configs.load_coeffs("paper_L14")
    m = 0.0
    for shape in TS.SHAPES:
        M = gen.round_to_bf16_np(TS._gradient_like(*shape, seed=40 + shape[0]))
        Yo = oracle.ifnso(M, exps, c, "complement", "gram_frobenius")
        m = max(m, _rel(BM.complement_split(M, exps, c, accum=np.float32), Yo))
    assert 3.0 * m <= TS.TOL_SPLIT <= 2e-2, (TS.TOL_SPLIT, m)


def test_split_single_power_bound():
    """Single powers (up to the fourth squaring) with split operands: the model with float32
    accumulation (one rounding per 16 products) follows the device closely here."""
    m = 0.0
    for h in (256, 200):
        v = gen.round_to_bf16_np(TG._input(h, seed=300 + h))
        for j in range(5):
            exps, c = (0, 1 << j), (0.0, 1.0)
            parts = oracle.ifnso_parts(v, exps, c, "complement", "gram_frobenius")
            Y = BM.complement_split(v, exps, c, accum="f32seq")
            m = max(m, _rel(Y[:, h:] * parts["scale"], parts["P"]))
    _within(TG.TOL_SPLIT_POWER, m)


def test_stage_bounds():
    """The bf16 single-power bounds: the one-tile cases (h = 256, 200) and the batched
    multi-tile case of tests/test_gpu_stages.py."""
    cases = [(h, False, "frobenius") for h in (256, 200)] + [(h, t, "none") for h, t in TG.MULTI_TILE]
    worst = {}
    for h, tall, norm in cases:
        if norm == "none":
            v, alpha = TG.multi_tile_input(h, tall)
        else:
            v, alpha = gen.round_to_bf16_np(TG._input(h, seed=300 + h)), None
        for j in range(5):
            exps, c = (0, 1 << j), (0.0, 1.0)
            parts = oracle.ifnso_parts(v, exps, c, "gram", norm)
            Y = BM.gram_levels(v, exps, c, norm, out_bf16=False)
            Yw = Y.T if tall else Y
            r = _rel(Yw[:, h:] / alpha if alpha else Yw[:, h:] * parts["scale"], parts["P"])
            key = "gram" if j == 0 else "power"
            worst[key] = max(worst.get(key, 0.0), r)
    _within(TG.TOL_BF16_GRAM, worst["gram"])
    _within(TG.TOL_BF16_POWER, worst["power"])


def test_fold_bound():
    """The weighted-fold bound of tests/test_gpu_stages.py (every power up to 2^J weighted, the
    multi-tile inputs), and that it separates a fold that misreads a level: dropping any stored
    level's term, or swapping two neighbouring weights, moves P by far more than the bound."""
    worst = 0.0
    for J in TG.FOLD_J:
        exps, c = TG.fold_terms(J)
        for h, tall in TG.MULTI_TILE:
            v, alpha = TG.multi_tile_input(h, tall)
            P = oracle.ifnso_parts(v, exps, c, "gram", "none")["P"]
            Y = BM.gram_levels(v, exps, c, "none", out_bf16=False)
            worst = max(worst, _rel((Y.T if tall else Y)[:, h:] / alpha, P))
    _within(TG.TOL_BF16_FOLD, worst)
    h, tall = TG.MULTI_TILE[0]
    v, _ = TG.multi_tile_input(h, tall)
    for J in TG.FOLD_J:
        exps, c = TG.fold_terms(J)
        P = oracle.ifnso_parts(v, exps, c, "gram", "none")["P"]
        wrong = []
        for k in range(1, J + 1):
            cc = list(c)
            cc[k] = 0.0
            wrong.append(cc)
        for k in range(1, J):
            cc = list(c)
            cc[k], cc[k + 1] = cc[k + 1], cc[k]
            wrong.append(cc)
        for cc in wrong:
            assert _rel(oracle.ifnso_parts(v, exps, cc, "gram", "none")["P"], P) > 10 * TG.TOL_BF16_FOLD


def _golden(golden_dir):
    with open(os.path.join(golden_dir, "bf16_bounds.json")) as f:
        return json.load(f)


def test_fullsize_bounds_from_golden(golden_dir):
    g = _golden(golden_dir)
    _within(TF.TOL_D2_SCHEDULE_BF16, max(g["d2_schedule_muon_ns5"].values()))
    assert set(g["d4_gform_v1_closed"]) == {str(i) for i in TF.D4_SAMPLED}
    _within(TF.TOL_D4_ORACLE, g["d4_gform_v1_oracle"]["0"])
    # the closed-form bound is the path's 2e-2; the model stays under a third of it
    assert 3.0 * max(g["d4_gform_v1_closed"].values()) <= TF.TOL_D4_CLOSED
    assert set(g["d3_gform_v1_oracle"]) == {f"{l}/{i}" for l, i in TF.D3_SAMPLED}
    _within(TF.TOL_D3_ORACLE, max(g["d3_gform_v1_oracle"].values()))


@pytest.mark.slow
def test_golden_d2_entry_recomputed(golden_dir):
    """The 4096 x 4096 entry of the golden file, recomputed (about 20 s)."""
    sched, _ = configs.load_schedule("muon_ns5")
    sigma = configs.d2_sigma_np(4096, 1)
    M, U, V = gen.spectral_np(4096, 4096, sigma, 1)
    f = BL.compose_scalar(sigma / np.sqrt(np.sum(sigma ** 2)), sched)
    r = _rel(BM.ns_chained(gen.round_to_bf16_np(M), sched, 0), (U * f) @ V.T)
    assert abs(r - _golden(golden_dir)["d2_schedule_muon_ns5"]["4096x4096"]) <= 1e-3 * r
