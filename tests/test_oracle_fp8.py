"""Pins of the e4m3 oracle: the OCP e4m3 format's defining values, round trips, ties to
even, PyTorch's float8_e4m3fn conversion as an independent library routine, the scale
rule, the bfloat16 rounding against the bit-level generator routine, and the e4m3 model
reducing to the plain float64 polynomial when its quantisers are the identity."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import fp8 as F
from workloads import configs, gen


def test_decode_defining_values():
    # OCP FP8 e4m3: bias 7, no infinities, S.1111.111 is NaN
    assert F.e4m3_decode(0x7E) == 448.0
    assert F.e4m3_decode(0x08) == 2.0 ** -6       # smallest normal
    assert F.e4m3_decode(0x01) == 2.0 ** -9       # smallest subnormal
    assert F.e4m3_decode(0x07) == 7 * 2.0 ** -9   # largest subnormal
    assert F.e4m3_decode(0x38) == 1.0
    assert F.e4m3_decode(0x40) == 2.0
    assert F.e4m3_decode(0xB8) == -1.0
    assert F.e4m3_decode(0x77) == 240.0
    assert F.e4m3_decode(0x00) == 0.0 and math.copysign(1.0, F.e4m3_decode(0x80)) == -1.0
    assert np.isnan(F.e4m3_decode(0x7F)) and np.isnan(F.e4m3_decode(0xFF))
    vals = F.e4m3_decode(np.arange(0x7F, dtype=np.uint8))
    assert np.all(np.diff(vals) > 0) and len(set(vals.tolist())) == 127


def test_encode_decode_round_trip():
    codes = np.array([c for c in range(256) if (c & 0x7F) != 0x7F], dtype=np.uint8)
    assert np.array_equal(F.e4m3_encode(F.e4m3_decode(codes)), codes)
    assert np.array_equal(F.e4m3_round(F.e4m3_decode(codes)), F.e4m3_decode(codes))


def test_ties_to_even_and_nearest():
    vals = F.e4m3_decode(np.arange(0x7F, dtype=np.uint8))
    for k in range(len(vals) - 1):
        lo, hi = vals[k], vals[k + 1]
        mid = 0.5 * (lo + hi)
        want_mid = lo if k % 2 == 0 else hi      # the even code has the even mantissa
        assert F.e4m3_round(mid) == want_mid, k
        assert F.e4m3_round(-mid) == -want_mid
        eps = (hi - lo) * 1e-6
        assert F.e4m3_round(mid - eps) == lo and F.e4m3_round(mid + eps) == hi


def test_saturation_and_monotonicity():
    assert F.e4m3_round(460.0) == 448.0 and F.e4m3_round(1e9) == 448.0 and F.e4m3_round(-1e9) == -448.0
    x = np.linspace(-500, 500, 200001)
    assert np.all(np.diff(F.e4m3_round(x)) >= 0)


def test_matches_torch_float8_e4m3fn():
    """torch's float8_e4m3fn conversion (round to nearest even) on float32 inputs in range."""
    torch = pytest.importorskip("torch")
    if not hasattr(torch, "float8_e4m3fn"):
        pytest.skip("torch without float8_e4m3fn")
    rng_vals = np.concatenate([
        gen.normal_np(11, 0, 20000) * 40.0,
        np.ldexp(gen.uniform_np(11, 1, 20000) * 2 - 1, (gen.uniform_np(11, 2, 20000) * 20 - 12).astype(int)),
        F.e4m3_decode(np.arange(0x7E, dtype=np.uint8)) * (1 + 2.0 ** -5),   # near and at ties
        0.5 * (F.e4m3_decode(np.arange(0x7E, dtype=np.uint8)) + F.e4m3_decode(np.arange(1, 0x7F, dtype=np.uint8))),
    ]).astype(np.float32)
    rng_vals = rng_vals[np.abs(rng_vals) <= 448.0]
    t = torch.from_numpy(rng_vals).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(F.e4m3_encode(rng_vals.astype(np.float64)), t)


def test_scale_rule():
    amax = np.exp(gen.uniform_np(12, 0, 4000) * 70 - 35)   # inside the unclamped range
    for a in amax:
        s = F.e4m3_scale(a)
        e = math.log2(s)
        assert e == int(e)
        assert 224.0 < a * s <= 448.0
    assert F.e4m3_scale(448.0) == 1.0 and F.e4m3_scale(449.0) == 0.5 and F.e4m3_scale(224.0) == 2.0
    assert F.e4m3_scale(1.0) == 256.0
    assert F.e4m3_scale(0.0) == 1.0 and F.e4m3_scale(float("inf")) == 1.0
    assert F.e4m3_scale(1e-30) == 2.0 ** 63 and F.e4m3_scale(1e30) == 2.0 ** -63


def test_bf16_round_matches_bit_level_rounding():
    x = np.concatenate([gen.normal_np(13, 0, 50000), np.ldexp(gen.uniform_np(13, 1, 50000), 60),
                        np.ldexp(gen.normal_np(13, 2, 50000), -70)])
    assert np.array_equal(F.bf16_round(x), gen.round_to_bf16_np(x))


@pytest.mark.parametrize("shape", [(24, 40), (40, 24), (16, 16), (1, 9)])
@pytest.mark.parametrize("norm", ["frobenius", "gram_frobenius", "none"])
def test_model_reduces_to_float64_polynomial(shape, norm):
    """With identity quantiser and storage the e4m3 model is the plain polynomial."""
    M = gen.normal_np(14, 0, shape[0] * shape[1]).reshape(shape) * 0.3
    exps, coeffs = configs.D2_EXPONENTS, configs.load_coeffs("gform_v1")[1]
    ident = lambda T: np.asarray(T, dtype=np.float64)
    got = F.ifnso_e4m3(M, exps, coeffs, norm=norm, quantize=ident, store=ident)
    want = O.ifnso(M, exps, coeffs, basis="gram", norm=norm)
    assert np.linalg.norm(got - want) <= 1e-11 * max(1.0, np.linalg.norm(want))


def test_model_exact_operands():
    """Entries on the e4m3 grid (times a power of two) are not changed by the quantiser."""
    codes = (gen.uniform_np(15, 0, 32 * 48) * 0x7E).astype(np.uint8)
    A = F.e4m3_decode(codes).reshape(32, 48) * 2.0 ** -7
    Aq, s = F.e4m3_quantize(A)
    assert np.array_equal(Aq, A)
    assert s == F.e4m3_scale(np.max(np.abs(A)))


def test_model_error_is_e4m3_sized():
    """The e4m3 model departs from the float64 polynomial by an amount of the order of e4m3's
    relative precision (2^-4), and by far more than bfloat16 storage alone."""
    M = gen.normal_np(16, 0, 48 * 96).reshape(48, 96)
    exps, coeffs = configs.D2_EXPONENTS, configs.load_coeffs("gform_v1")[1]
    want = O.ifnso(M, exps, coeffs)
    e8 = np.linalg.norm(F.ifnso_e4m3(M, exps, coeffs) - want) / np.linalg.norm(want)
    eb = np.linalg.norm(F.ifnso_e4m3(M, exps, coeffs, quantize=lambda T: T) - want) / np.linalg.norm(want)
    assert eb < 1e-2
    assert 1e-3 < e8 < 0.15 and e8 > 2 * eb


# ---------------------------------------------------------------------------------------------
# per-tile quantisation of the stored levels
# ---------------------------------------------------------------------------------------------
def test_tiles_worked_example():
    """Two 2 x 2 tiles (tile = 2) worked by hand. Left tile: maximum 1 -> scale 2^8; 76.8 and
    25.6 and 12.8 round to the nearest e4m3 values 80, 26, 13 (four significant bits).
    Right tile: maximum 100 -> scale 2^2 (448 / 100 = 4.48); 400 lies halfway between 384 and
    416 and goes to the even significand 1.5 (384); 12, 8, 4 are exact."""
    T = np.array([[1.0, 0.3, 100.0, 3.0], [0.1, 0.05, 2.0, 1.0]])
    want = np.array([[1.0, 80 / 256, 96.0, 3.0], [26 / 256, 13 / 256, 2.0, 1.0]])
    assert np.array_equal(F.e4m3_quantize_tiles(T, tile=2), want)


def test_tiles_are_independent():
    """Each tile is the per-tensor quantisation of that tile alone, edge tiles included, and
    scaling one tile by a power of two scales only its own output, exactly."""
    T = gen.normal_np(17, 0, 10 * 13).reshape(10, 13) * np.repeat(np.repeat(
        np.array([[1.0, 50.0, 1e-3], [7.0, 0.2, 3e4], [1.0, 1.0, 1.0]]), 4, axis=0), 5, axis=1)[:10, :13]
    Q = F.e4m3_quantize_tiles(T, tile=4)
    for r0 in range(0, 10, 4):
        for c0 in range(0, 13, 4):
            assert np.array_equal(Q[r0:r0 + 4, c0:c0 + 4], F.e4m3_quantize(T[r0:r0 + 4, c0:c0 + 4])[0])
    T2 = T.copy()
    T2[4:8, 8:12] *= 2.0 ** 5
    Q2 = F.e4m3_quantize_tiles(T2, tile=4)
    mask = np.zeros(T.shape, bool)
    mask[4:8, 8:12] = True
    assert np.array_equal(Q2[mask], Q[mask] * 2.0 ** 5)
    assert np.array_equal(Q2[~mask], Q[~mask])


def test_one_tile_levels_match_the_per_tensor_rule():
    """Levels of at most 256 rows are a single tile: the default model (per-tile levels) and the
    per-tensor rule give the same result; beyond 256 rows they differ."""
    exps, coeffs = configs.D2_EXPONENTS, configs.load_coeffs("gform_v1")[1]
    per_tensor = lambda T: F.e4m3_quantize(T)[0]  # noqa: E731
    M = gen.normal_np(18, 0, 200 * 300).reshape(200, 300)
    assert np.array_equal(F.ifnso_e4m3(M, exps, coeffs), F.ifnso_e4m3(M, exps, coeffs, quantize_level=per_tensor))
    M = gen.normal_np(19, 0, 300 * 320).reshape(300, 320) * np.linspace(0.2, 3.0, 300)[:, None]
    assert not np.array_equal(F.ifnso_e4m3(M, exps, coeffs), F.ifnso_e4m3(M, exps, coeffs, quantize_level=per_tensor))
