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
    ident = lambda T, m=None: np.asarray(T, dtype=np.float64)  # noqa: E731
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
    eb = np.linalg.norm(F.ifnso_e4m3(M, exps, coeffs, quantize=lambda T, m: T) - want) / np.linalg.norm(want)
    assert eb < 1e-2
    assert 1e-3 < e8 < 0.15 and e8 > 2 * eb


# ---------------------------------------------------------------------------------------------
# the scale of a stored power: the largest magnitude of the product before its rounding
# ---------------------------------------------------------------------------------------------
def test_gram_row_max_is_the_largest_magnitude():
    """For X X^T (any X) and X X (symmetric X) the largest magnitude is the largest squared row
    norm of X (brute force over all entries)."""
    X = gen.normal_np(20, 0, 37 * 53).reshape(37, 53)
    assert np.isclose(F.gram_row_max(X), np.max(np.abs(X @ X.T)), rtol=1e-14, atol=0)
    S = X[:, :37] + X[:, :37].T
    assert np.isclose(F.gram_row_max(S), np.max(np.abs(S @ S)), rtol=1e-14, atol=0)
    assert F.gram_row_max(np.zeros((3, 4))) == 0.0


def test_power_scale_worked_example():
    """X = [1, 1/2, 1/2, 1/2, 2^-5]: X X^T = 1.75 + 2^-10 exactly. Its bfloat16 value is 1.75
    (8 significant bits), whose scale would be 448 / 1.75 = 2^8; the product before rounding
    gives 448 / 1.7509765625 < 2^8, so 2^7. The model takes the latter: the quantiser of the
    first squaring is called with that maximum."""
    X = np.array([[1.0, 0.5, 0.5, 0.5, 2.0 ** -5]])
    assert F.gram_row_max(X) == 1.75 + 2.0 ** -10
    assert F.bf16_round(X @ X.T)[0, 0] == 1.75
    assert F.e4m3_scale(F.gram_row_max(X)) == 2.0 ** 7
    assert F.e4m3_scale(1.75) == 2.0 ** 8
    seen = []

    def q(T, m):
        seen.append(m)
        return F.e4m3_quantize_with(T, m)[0]

    F.ifnso_e4m3(X, (0, 1, 2), (0.5, 0.3, 0.2), norm="none", quantize=q)
    assert seen == [1.0, 1.75 + 2.0 ** -10]  # max|A|, then the Gram's largest row norm


def test_quantize_with_matches_per_tensor_rule():
    T = gen.normal_np(21, 0, 30 * 40).reshape(30, 40)
    a, s = F.e4m3_quantize(T)
    b, t = F.e4m3_quantize_with(T, float(np.max(np.abs(T))))
    assert s == t and np.array_equal(a, b)


def test_power_scale_worked_example_through_the_model():
    """The same rule end to end (the GPU test of it uses this input): A = [Z | I] with Z rows
    [1, 1, 1/2, 1/2, 2^-5, 2^-5] and [13 2^-16, 0, ...]; L1[0][0] = 3.5 + 2^-9 gives the scale
    2^6, under which L1[0][1] = 13 2^-16 is 6.5 e4m3 quanta and rounds to 6, so with the single
    power B^2 the identity block of Y holds L2[0][1] = (3.5 + 1) 3 2^-14 = 13.5 2^-14; the scale
    of the stored maximum 3.5 (2^7) would keep 13 2^-16 and give 4.5 13 2^-16 = 14.625 2^-14."""
    Z = np.zeros((2, 6))
    Z[0] = [1.0, 1.0, 0.5, 0.5, 2.0 ** -5, 2.0 ** -5]
    Z[1, 0] = 13 * 2.0 ** -16
    A = np.concatenate([Z, np.eye(2)], axis=1)
    Y = F.ifnso_e4m3(A, (0, 2), (0.0, 1.0), norm="none")
    assert Y[0, 7] == 13.5 * 2.0 ** -14 and Y[0, 6] == 12.25 and Y[1, 7] == 1.0
    stored_max_rule = F.ifnso_e4m3(A, (0, 2), (0.0, 1.0), norm="none", quantize=lambda T, m: F.e4m3_quantize(T)[0])
    assert stored_max_rule[0, 7] == 14.625 * 2.0 ** -14
