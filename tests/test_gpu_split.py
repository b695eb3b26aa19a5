"""Split-bfloat16 operands (IFNSO_FLAG_SPLIT_BF16) for the paper's complement-basis form on the
GPU, through the C ABI, against the FP64 oracle.

The form is Algorithm 1's: T = I - XX^T with X = A / ||AA^T||_F^(1/2) (Sec. 2.2), powers by
repeated squaring of the shifted power D = T^(2^(l-1)) - I (Sec. 2.4), depth L = 14 with the
"paper_L14" coefficients, whose magnitudes reach 237 with alternating signs. Single bf16
operands lose the small eigencomponents of D that those coefficients amplify; split operands
(hi + lo pairs, three bf16 products per squaring, float32 accumulation, P as a pair) keep
about 16 significant bits.

Tolerance: relative Frobenius distance <= 3e-3 with float32 output. The storage-point model of
the split arithmetic (oracle.bf16_model.complement_split: every squaring operand and P rounded to
a hi + lo bf16 pair, all else exact) gives 1.0e-4 .. 2.1e-4 on SHAPES; the device measures
1.1e-3 .. 1.2e-3. The difference is float32 accumulation: at depth 14 the last levels of D are
close to -I, every squaring re-forms -I + (small) from 2 D + D^2, and the matrix cores' summation
leaves about 2^-19 of the largest entry in each level (a single 2^13 power with coefficient 1
lands 2.6e-5 from the exact one on the device, 3e-9 in the model), which the large alternating
coefficients then scale up. A float64 emulation with one float32 rounding per 16 products does
not reproduce the matrix cores' internal summation, so this bound rests on the measured
deviation: 2.5 times it, and at least three times the storage-point model (checked by
tests/test_oracle_bounds.py). The unsplit bf16 path is reported alongside and must be at least
ten times further from the oracle.
"""
import numpy as np
import pytest

import oracle
from workloads import configs, gen

pytestmark = pytest.mark.gpu

TOL_SPLIT = 3e-3


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


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _run(torch, dev, Ms, shapes, exps, c, split=True, norm="gram_frobenius"):
    import paper_2602_02500_amd as ifn
    plan = ifn.Plan(exps, c, shapes, basis="complement", norm=norm, compute="bf16", out_dtype=ifn.F32,
                    flags=ifn.FLAG_SPLIT_BF16 if split else 0)
    Ys = [torch.full(s, float("nan"), dtype=torch.float32, device=dev) for s in shapes]
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    if len(Ms) == 1:
        plan.orthogonalize(Ms[0], Ys[0], ws)
    else:
        plan.orthogonalize_batched(Ms, Ys, ws)
    torch.cuda.synchronize()
    return [y.cpu().numpy().astype(np.float64) for y in Ys]


def _gradient_like(rows, cols, seed):
    return gen.lowrank_plus_noise_np(rows, cols, seed)


SHAPES = [(256, 512), (512, 256), (200, 456), (520, 264), (384, 384), (1, 64)]


@pytest.mark.parametrize("shape", SHAPES)
def test_paper_depth_matches_oracle(tdev, shape):
    torch, dev = tdev
    exps, c = configs.load_coeffs("paper_L14")
    print(f"case shape={shape}", flush=True)
    Mt, vals = _bf16_dev(torch, dev, _gradient_like(*shape, seed=40 + shape[0]))
    (Y,) = _run(torch, dev, [Mt], [shape], exps, c)
    Yo = oracle.ifnso(vals, exps, c, "complement", "gram_frobenius")
    r = _rel(Y, Yo)
    h = min(shape)
    print(f"  split rel {r:.2e}; orth/sqrt(h): device {oracle.orth_error(Y) / np.sqrt(h):.4f}, "
          f"oracle {oracle.orth_error(Yo) / np.sqrt(h):.4f}")
    assert r <= TOL_SPLIT
    if h > 1:
        (Yu,) = _run(torch, dev, [Mt], [shape], exps, c, split=False)
        ru = _rel(Yu, Yo)
        print(f"  unsplit bf16 rel {ru:.2e}")
        assert ru >= 10 * r


@pytest.mark.parametrize("norm", ["frobenius", "gram_frobenius"])
def test_moderate_terms_and_norms(tdev, norm):
    torch, dev = tdev
    exps, c = (0, 1, 2, 4, 8), (0.4, 0.3, 0.15, 0.1, 0.05)
    for shape in [(160, 416), (416, 160)]:
        Mt, vals = _bf16_dev(torch, dev, gen.gaussian_np(*shape, seed=12))
        (Y,) = _run(torch, dev, [Mt], [shape], exps, c, norm=norm)
        r = _rel(Y, oracle.ifnso(vals, exps, c, "complement", norm))
        print(f"{shape} {norm}: rel {r:.2e}")
        assert r <= 1e-4


def test_no_squarings(tdev):
    """Exponents {0, 1}: no squaring, P = c_1 D_1 from the split Gram operand."""
    torch, dev = tdev
    exps, c = (0, 1), (1.5, -0.5)
    Mt, vals = _bf16_dev(torch, dev, gen.gaussian_np(96, 256, seed=13))
    (Y,) = _run(torch, dev, [Mt], [(96, 256)], exps, c)
    assert _rel(Y, oracle.ifnso(vals, exps, c, "complement", "gram_frobenius")) <= 1e-5


def test_batched_equals_single_bitwise(tdev):
    torch, dev = tdev
    exps, c = configs.load_coeffs("paper_L14")
    shapes = [(256, 512), (512, 256), (200, 456)]
    Ms, vals = [], []
    for i, s in enumerate(shapes):
        t, v = _bf16_dev(torch, dev, _gradient_like(*s, seed=60 + i))
        Ms.append(t)
        vals.append(v)
    Yb = _run(torch, dev, Ms, shapes, exps, c)
    for i, s in enumerate(shapes):
        (Ys,) = _run(torch, dev, [Ms[i]], [s], exps, c)
        assert np.array_equal(Yb[i], Ys), i


def test_unaligned_problem_is_rejected(tdev):
    """Only the 256-tile kernels know the split layout: a row pitch that is not a multiple of 8
    elements is refused at call time instead of being computed by the generic kernels."""
    torch, dev = tdev
    import paper_2602_02500_amd as ifn
    exps, c = configs.load_coeffs("paper_L14")
    Mt, _ = _bf16_dev(torch, dev, gen.gaussian_np(64, 128, seed=14), ld_pad=3)
    plan = ifn.Plan(exps, c, [(64, 128)], basis="complement", norm="gram_frobenius", compute="bf16",
                    out_dtype=ifn.F32, flags=ifn.FLAG_SPLIT_BF16)
    Y = torch.zeros((64, 128), dtype=torch.float32, device=dev)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    with pytest.raises(ifn.IfnsoError):
        plan.orthogonalize(Mt, Y, ws)
