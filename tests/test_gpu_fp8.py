"""The e4m3 compute mode on the GPU, through the C ABI.

* The input quantiser is bit-exact against the oracle's e4m3 encoding (the same bfloat16
  inputs, the same scale rule), with the float64 norm and the maximum it reports.
* Whole plans are compared with the oracle's e4m3 model (the same quantisation points and
  bfloat16 storage, everything else in float64). With float32 output the remaining
  differences are float32 accumulation order, which can flip an e4m3 or bfloat16 rounding
  only for values within ~2^-24 of a rounding boundary: bound 2e-3 (relative Frobenius).
  With bfloat16 output add the output rounding (2^-9 per entry): bound 1e-2.
* The error against the plain float64 polynomial is reported (printed), with only a loose
  sanity bound: e4m3's relative precision is 2^-4.
"""
import numpy as np
import pytest

import oracle
from oracle import fp8 as F
from workloads import configs, gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tdev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_02500_amd as ifn
    ifn.load()
    return torch, torch.device("cuda:0")


def _bf16_dev(torch, dev, M64, ld_pad=0):
    vals = gen.round_to_bf16_np(M64)
    t = torch.zeros((M64.shape[0], M64.shape[1] + ld_pad), dtype=torch.bfloat16, device=dev)
    t[:, :M64.shape[1]] = torch.from_numpy(vals.astype(np.float32)).to(dev).to(torch.bfloat16)
    return t[:, :M64.shape[1]], vals


def _heavy_tailed(rows, cols, seed, scale=0.5):
    """U diag(sigma) V^T with Haar factors and sigma_i = i^-1.5 (the FP8 workload's spectrum)."""
    r = min(rows, cols)
    U = gen.haar_np(rows, r, seed, 1)
    V = gen.haar_np(cols, r, seed, 2)
    return scale * (U * configs.d4_sigma(r)) @ V.T


def _rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def _run(torch, dev, vals_list, Ms, exps, c, norm="frobenius", out="f32", compute="fp8"):
    import paper_2602_02500_amd as ifn
    plan = ifn.Plan(exps, c, [v.shape for v in vals_list], norm=norm, compute=compute,
                    out_dtype=ifn.F32 if out == "f32" else ifn.BF16)
    ydt = torch.float32 if out == "f32" else torch.bfloat16
    Ys = [torch.full(v.shape, float("nan"), dtype=ydt, device=dev) for v in vals_list]
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    if len(Ms) == 1:
        plan.orthogonalize(Ms[0], Ys[0], ws)
    else:
        plan.orthogonalize_batched(Ms, Ys, ws)
    torch.cuda.synchronize()
    return [y.float().cpu().numpy().astype(np.float64) for y in Ys], plan


# ---------------------------------------------------------------------------------------------
# input quantiser
# ---------------------------------------------------------------------------------------------
# the wide rows of the last two cross the 1024-column chunks of the quantiser (one per wave),
# the last chunk ragged; the pre-pass takes several rows per chunk
QSHAPES = [(256, 512, 0, 0), (640, 384, 0, 0), (100, 203, 0, 0), (300, 97, 0, 0), (64, 96, 5, 32),
           (130, 72, 8, 16), (1, 40, 0, 0), (45, 1, 0, 0), (96, 2504, 8, 16), (70, 3000, 0, 0)]


@pytest.mark.parametrize("rows,cols,ld_pad,q_pad", QSHAPES)
def test_quantize_input_bit_exact(tdev, rows, cols, ld_pad, q_pad):
    torch, dev = tdev
    import paper_2602_02500_amd as ifn
    print(f"case rows={rows} cols={cols} ld_pad={ld_pad} q_pad={q_pad}", flush=True)
    M64 = gen.normal_np(rows + 3 * cols, 0, rows * cols).reshape(rows, cols) * 0.02
    Mt, vals = _bf16_dev(torch, dev, M64, ld_pad)
    h, w = min(rows, cols), max(rows, cols)
    ldq = (w + 15) // 16 * 16 + q_pad
    Q = torch.full((h, ldq), 0xAB, dtype=torch.uint8, device=dev)
    out3 = torch.zeros(3, dtype=torch.float64, device=dev)
    ws = torch.empty(ifn.quantize_e4m3_workspace_bytes(rows, cols), dtype=torch.uint8, device=dev)
    ifn.quantize_e4m3(Mt, Q, out3, ws)
    torch.cuda.synchronize()
    A = vals.T if rows > cols else vals
    amax = float(np.max(np.abs(A)))
    s = F.e4m3_scale(amax)
    want = np.zeros((h, ldq), dtype=np.uint8)
    want[:, :w] = F.e4m3_encode(A * s)
    got = Q.cpu().numpy()
    bad = np.argwhere(got != want)
    assert bad.size == 0, (bad[:5], got[tuple(bad[0])], want[tuple(bad[0])])
    o = out3.cpu().numpy()
    assert o[1] == amax and o[2] == s
    n2 = float(np.sum(A * A))
    assert abs(o[0] - n2) <= 1e-6 * n2


def test_quantize_zero_matrix(tdev):
    torch, dev = tdev
    import paper_2602_02500_amd as ifn
    Mt = torch.zeros((48, 80), dtype=torch.bfloat16, device=dev)
    Q = torch.full((48, 80), 7, dtype=torch.uint8, device=dev)
    out3 = torch.full((3,), -1.0, dtype=torch.float64, device=dev)
    ws = torch.empty(ifn.quantize_e4m3_workspace_bytes(48, 80), dtype=torch.uint8, device=dev)
    ifn.quantize_e4m3(Mt, Q, out3, ws)
    torch.cuda.synchronize()
    assert int(Q.max().item()) == 0
    assert out3.cpu().numpy().tolist() == [0.0, 0.0, 1.0]


# ---------------------------------------------------------------------------------------------
# whole plans
# ---------------------------------------------------------------------------------------------
PSHAPES = [(256, 512), (512, 256), (384, 640), (200, 456), (520, 264), (160, 2312)]


@pytest.mark.parametrize("shape", PSHAPES)
@pytest.mark.parametrize("out", ["f32", "bf16"])
def test_plan_matches_e4m3_model(tdev, shape, out):
    torch, dev = tdev
    exps, c = configs.load_coeffs("gform_v1")
    print(f"case shape={shape} out={out}", flush=True)
    Mt, vals = _bf16_dev(torch, dev, _heavy_tailed(*shape, seed=3 + shape[0]))
    (Y,), _ = _run(torch, dev, [vals], [Mt], exps, c, out=out)
    Ym = F.ifnso_e4m3(vals, exps, c)
    Yo = oracle.ifnso(vals, exps, c)
    r_model, r_exact = _rel(Y, Ym), _rel(Y, Yo)
    print(f"  rel vs e4m3 model {r_model:.2e}, vs float64 polynomial {r_exact:.3e}")
    assert r_model <= (2e-3 if out == "f32" else 1e-2)
    assert r_exact < 0.25


@pytest.mark.parametrize("norm", ["gram_frobenius", "none"])
def test_plan_norms(tdev, norm):
    torch, dev = tdev
    exps, c = configs.D1_EXPONENTS, tuple(configs.d1_coeffs())
    M = _heavy_tailed(256, 384, seed=9) * (1.0 if norm != "none" else 0.05)
    Mt, vals = _bf16_dev(torch, dev, M)
    (Y,), _ = _run(torch, dev, [vals], [Mt], exps, c, norm=norm)
    r = _rel(Y, F.ifnso_e4m3(vals, exps, c, norm=norm))
    print(f"norm={norm}: rel vs e4m3 model {r:.2e}")
    assert r <= 2e-3


@pytest.mark.parametrize("exps,c", [((0, 1), (1.5, -0.5)), ((1,), (1.0,)), ((0,), (2.0,)), ((0, 2), (1.2, 0.9))])
def test_short_polynomials(tdev, exps, c):
    """J = 0 (no squaring: the aggregate stage alone forms P = c_1 G), a single squaring, and
    the constant polynomial."""
    torch, dev = tdev
    Mt, vals = _bf16_dev(torch, dev, gen.gaussian_np(192, 320, seed=31))
    (Y,), _ = _run(torch, dev, [vals], [Mt], exps, c)
    r = _rel(Y, F.ifnso_e4m3(vals, exps, c))
    print(f"exps={exps}: rel vs e4m3 model {r:.2e}")
    assert r <= 2e-3


def test_unaligned_input_and_single_rows(tdev):
    """Row pitch that is not a multiple of 8 (generic product, scalar pre-pass) and h = 1
    (the product evaluates p from the float64 norm, so no e4m3 rounding enters)."""
    torch, dev = tdev
    exps, c = configs.load_coeffs("gform_v1")
    Mt, vals = _bf16_dev(torch, dev, _heavy_tailed(136, 300, seed=4), ld_pad=3)
    (Y,), _ = _run(torch, dev, [vals], [Mt], exps, c)
    assert _rel(Y, F.ifnso_e4m3(vals, exps, c)) <= 2e-3
    for shape in [(1, 64), (80, 1)]:
        Mt, vals = _bf16_dev(torch, dev, gen.gaussian_np(*shape, seed=5))
        (Y,), _ = _run(torch, dev, [vals], [Mt], exps, c)
        assert _rel(Y, oracle.ifnso(vals, exps, c)) <= 1e-5


def test_zero_matrix(tdev):
    torch, dev = tdev
    exps, c = configs.load_coeffs("gform_v1")
    Mt = torch.zeros((128, 256), dtype=torch.bfloat16, device=dev)
    (Y,), _ = _run(torch, dev, [np.zeros((128, 256))], [Mt], exps, c)
    assert np.all(Y == 0.0)


def test_batched_equals_single_bitwise(tdev):
    """The grouped launches compute every problem with the same per-tile arithmetic and
    fixed-order reductions as a single-problem call."""
    torch, dev = tdev
    exps, c = configs.load_coeffs("gform_v1")
    shapes = [(256, 512), (512, 256), (200, 456), (384, 640), (64, 1024)]
    Ms, vals = [], []
    for i, s in enumerate(shapes):
        t, v = _bf16_dev(torch, dev, _heavy_tailed(*s, seed=50 + i))
        Ms.append(t)
        vals.append(v)
    Yb, plan = _run(torch, dev, vals, Ms, exps, c)
    assert plan.num_launches == 4 + 6      # J = 4 squarings for exponent 16
    assert plan.launch_info(0)[0] == 4
    for i in range(len(shapes)):
        (Ys,), _ = _run(torch, dev, [vals[i]], [Ms[i]], exps, c)
        assert np.array_equal(Yb[i], Ys), i
        assert _rel(Yb[i], F.ifnso_e4m3(vals[i], exps, c)) <= 2e-3


def test_error_against_bf16_mode(tdev):
    """Report: distance of the e4m3 and bfloat16 modes from the float64 polynomial, and the
    orthogonality error of each, on one FP8-workload-shaped matrix at reduced size."""
    torch, dev = tdev
    import paper_2602_02500_amd as ifn
    exps, c = configs.load_coeffs("gform_v1")
    Mt, vals = _bf16_dev(torch, dev, _heavy_tailed(512, 2048, seed=3))
    Yo = oracle.ifnso(vals, exps, c)
    res = {}
    for comp in ["bf16", "fp8"]:
        (Y,), _ = _run(torch, dev, [vals], [Mt], exps, c, compute=comp)
        res[comp] = (_rel(Y, Yo), oracle.orth_error(Y) / np.sqrt(512))
    print(f"rel vs float64: bf16 {res['bf16'][0]:.3e}, fp8 {res['fp8'][0]:.3e}; "
          f"||YY^T-I||/sqrt(h): bf16 {res['bf16'][1]:.4f}, fp8 {res['fp8'][1]:.4f}, "
          f"float64 {oracle.orth_error(Yo) / np.sqrt(512):.4f}")
    assert res["bf16"][0] <= 2e-2
    assert res["fp8"][0] < 0.25
    assert abs(res["fp8"][1] - res["bf16"][1]) < 0.1
    assert ifn  # the binding is loaded


def test_power_scale_from_exact_maximum(tdev):
    """The scale of a stored power comes from its largest magnitude before the bf16 rounding.
    Worked in exact arithmetic (every product, sum and rounding below is exact on both sides):
    A = [Z | I] (2 x 8), Z rows [1, 1, 1/2, 1/2, 2^-5, 2^-5] and [13 2^-16, 0, ...]. Then
    L1 = A A^T has L1[0][0] = 3.5 + 2^-9 (stored as 3.5) and L1[0][1] = 13 2^-16. The scale
    of L1 is 2^6 (448 / (3.5 + 2^-9) < 2^7); the one of its stored maximum would be 2^7. Under
    2^6, 13 2^-16 scales to 6.5 e4m3 quanta (2^-9) and rounds to 6; under 2^7 it stays exact. So
    the power read off Y's identity block, L2[0][1], is 13.5 2^-14 (it would be 14.625 2^-14)."""
    torch, dev = tdev
    Z = np.zeros((2, 6))
    Z[0] = [1.0, 1.0, 0.5, 0.5, 2.0 ** -5, 2.0 ** -5]
    Z[1, 0] = 13 * 2.0 ** -16
    A = np.concatenate([Z, np.eye(2)], axis=1)
    Mt, vals = _bf16_dev(torch, dev, A)
    assert np.array_equal(vals, A)
    exps, c = (0, 2), (0.0, 1.0)
    (Y,), _ = _run(torch, dev, [vals], [Mt], exps, c, norm="none")
    Ym = F.ifnso_e4m3(vals, exps, c, norm="none")
    assert Ym[0, 7] == 13.5 * 2.0 ** -14 and Ym[0, 6] == 12.25 and Ym[1, 7] == 1.0
    assert np.array_equal(Y[:, 6:], Ym[:, 6:]), (Y[:, 6:], Ym[:, 6:])
