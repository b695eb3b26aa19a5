"""Stage-level parity on the GPU: the Gram matrix and each squaring level, one at a time,
against the FP64 oracle's intermediates.

The output exposes them without reading the workspace. For M = [Z | I] (h x 2h), X = M / s
and Y = P X, so the right block of Y is P / s. With exponents {0, 2^j} and coefficients
(0, 1) the sum P is the single power B^(2^j): the Gram matrix B = X X^T for j = 0, then the
level that the j-th squaring produces (B = I - X X^T in the complement basis). Each case
therefore checks one more stage than the one before it.

Bounds (relative Frobenius distance to the oracle's power on the same input bytes): float32
1e-4; split bf16 (complement basis) 1.8e-5, three to four times what the split model with float32
accumulation gives for the fourth squaring (oracle.bf16_model.complement_split, "f32seq":
4.9e-6; the device measures 4.4e-6 .. 4.9e-6). Single bf16 operands:
three to four times what the float64 model of the bf16 storage points (oracle.bf16_model.
gram_levels: the input, each stored level and the output rounded to bf16) gives on these
inputs: 1.7e-3 for the Gram (bound 3 * 2^-9 = 5.9e-3) and 2.2e-3 .. 4.3e-3 for the powers after
one to four squarings (bound 1.5e-2). tests/test_oracle_bounds.py recomputes them.

The one-tile cases (h <= 256) check each kernel's arithmetic; the batched multi-tile case puts
several problems of 3 to 6 tiles per side, wide and tall, into one plan with per-XCD queues:
off-diagonal tiles, their mirrors, per-problem level scales and partials, and the last squaring
with the aggregation folded in are all on the path of the power read off each output.
"""
import numpy as np
import pytest

import oracle
from workloads import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tdev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_02500_amd as ifn
    ifn.load()
    return torch, torch.device("cuda:0")


def _input(h, seed):
    Z = gen.gaussian_np(h, h, seed) * 0.5
    return np.concatenate([Z, np.eye(h)], axis=1)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


TOL_BF16_GRAM = 3.0 * 2.0 ** -9   # j = 0
TOL_BF16_POWER = 1.5e-2           # j >= 1
TOL_SPLIT_POWER = 1.8e-5          # split operands, complement basis, j <= 4
# batched multi-tile case: (h, tall); input alpha [Z | I] (h x 2h) with Z = 0.5 N(0, 1) from seed
# 300 + h, transposed for the tall problem, and no normalisation (norm "none"): alpha puts the
# largest eigenvalue of B = M M^T at 0.98, so that every power up to B^16 stays of order one.
# (With the Frobenius scale the largest eigenvalue is about 4 / h and B^16 falls below 1e-37,
# the bottom of the float32 range, at these sizes.)
MULTI_TILE = [(768, False), (1000, False), (1536, False), (896, True)]


def multi_tile_input(h, tall):
    """(bf16 values of the multi-tile case's input, the bf16 value of alpha); see MULTI_TILE. The
    right block of Y = P M is then alpha P."""
    M = _input(h, seed=300 + h)
    lam = np.linalg.eigvalsh(M @ M.T)[-1]
    v = gen.round_to_bf16_np(M * np.sqrt(0.98 / lam))
    return (np.ascontiguousarray(v.T) if tall else v), float(v[0, h])


def bf16_power_bound(j):
    return TOL_BF16_GRAM if j == 0 else TOL_BF16_POWER


CASES = [
    # (compute, basis, norm, flags, tolerance)
    ("f32", "gram", "frobenius", 0, 1e-4),
    ("bf16", "gram", "frobenius", 0, None),
    ("f32", "complement", "gram_frobenius", 0, 1e-4),
    ("bf16", "complement", "gram_frobenius", "split", TOL_SPLIT_POWER),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}-{c[1]}-{'split' if c[3] else 'plain'}")
@pytest.mark.parametrize("h", [256, 200])
@pytest.mark.parametrize("j", [0, 1, 2, 3, 4])
def test_single_power(tdev, case, h, j):
    torch, dev = tdev
    import paper_2602_02500_amd as ifn
    compute, basis, norm, flags, tol = case
    exps, coeffs = (0, 1 << j), (0.0, 1.0)
    M = _input(h, seed=300 + h)
    if compute == "f32":
        vals = M.astype(np.float32).astype(np.float64)
        Mt = torch.from_numpy(vals.astype(np.float32)).to(dev)
    else:
        vals = gen.round_to_bf16_np(M)
        Mt = torch.from_numpy(vals.astype(np.float32)).to(dev).to(torch.bfloat16)
    fl = ifn.FLAG_SPLIT_BF16 if flags == "split" else 0
    plan = ifn.Plan(exps, coeffs, [(h, 2 * h)], basis=basis, norm=norm, compute=compute,
                    out_dtype=ifn.F32, flags=fl)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    Y = torch.full((h, 2 * h), float("nan"), dtype=torch.float32, device=dev)
    plan.orthogonalize(Mt, Y, ws)
    torch.cuda.synchronize()
    parts = oracle.ifnso_parts(vals, exps, coeffs, basis, norm)
    P_gpu = Y.cpu().numpy().astype(np.float64)[:, h:] * parts["scale"]
    if tol is None:
        tol = bf16_power_bound(j)
    r = _rel(P_gpu, parts["P"])
    print(f"{case[:2]} h={h} power 2^{j}: rel {r:.2e}")
    assert r <= tol


@pytest.mark.parametrize("j", [0, 1, 2, 3, 4])
def test_single_power_batched_multitile(tdev, j):
    """One bf16 Gram-basis plan over MULTI_TILE (three wide problems and a tall one, 3 to 6 tiles
    per side) with per-XCD task queues: each problem's power 2^j against the oracle's (the right
    block of Y is alpha times the power). A second
    plan with another schedule (queue group, panel block and workgroups per XCD changed, then
    plain striding without queues) gives the same bits: the partial sums are reduced in a fixed
    order whatever tile runs where."""
    torch, dev = tdev
    import paper_2602_02500_amd as ifn
    exps, coeffs = (0, 1 << j), (0.0, 1.0)
    Ms, vals, shapes = [], [], []
    alphas = []
    for h, tall in MULTI_TILE:
        v, alpha = multi_tile_input(h, tall)
        alphas.append(alpha)
        vals.append(v)
        shapes.append(v.shape)
        Ms.append(torch.from_numpy(v.astype(np.float32)).to(dev).to(torch.bfloat16))
    print(f"case multi-tile j={j} shapes {shapes}", flush=True)

    def run(cfgs):
        plan = ifn.Plan(exps, coeffs, shapes, norm="none", compute="bf16", out_dtype=ifn.F32)
        for stage, cfg in cfgs.items():
            plan.set_config(stage, cfg)
        ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
        Ys = [torch.full(s, float("nan"), dtype=torch.float32, device=dev) for s in shapes]
        plan.orthogonalize_batched(Ms, Ys, ws)
        torch.cuda.synchronize()
        return [y.cpu().numpy().astype(np.float64) for y in Ys]

    Ys = run({})
    for (h, tall), v, alpha, Y in zip(MULTI_TILE, vals, alphas, Ys):
        parts = oracle.ifnso_parts(v, exps, coeffs, "gram", "none")
        Yw = Y.T if tall else Y
        r = _rel(Yw[:, h:] / alpha, parts["P"])
        print(f"  h={h} tall={tall} power 2^{j}: rel {r:.2e}")
        assert r <= bf16_power_bound(j)
    alt = {ifn.STAGE_GRAM: dict(xcd_sched=1, group=8, block_rows=2, block_cols=2, wg_per_xcd=24),
           ifn.STAGE_SQUARE: dict(xcd_sched=1, group=16, block_rows=2, block_cols=4, wg_per_xcd=20),
           ifn.STAGE_PRODUCT: dict(xcd_sched=1, group=4, block_rows=1, block_cols=4, wg_per_xcd=28)}
    for Y0, Y1 in zip(Ys, run(alt)):
        assert np.array_equal(Y0, Y1)
    plain = {st: dict(xcd_sched=0, group=1, block_rows=1, block_cols=1, wg_per_xcd=32) for st in alt}
    for Y0, Y1 in zip(Ys, run(plain)):
        assert np.array_equal(Y0, Y1)


# weighted fold: every power 2^0 .. 2^J of the multi-tile inputs with a weight of its own, so
# that the last squaring's fold reads each stored level (J >= 5 takes a second pass of its
# four-level loop). Bound: three to four times what the bf16 storage-point model gives on the
# same inputs (3.8e-3 .. 4.2e-3 for J = 4, 5, 6; tests/test_oracle_bounds.py recomputes it).
# Dropping one level's term or swapping two neighbouring weights moves P by 0.32 or more.
TOL_BF16_FOLD = 1.5e-2
FOLD_J = [4, 5, 6]


def fold_terms(J):
    """Exponents 0, 1, 2, 4, .., 2^J and weights 0 (no identity term, so the right block of Y is
    alpha P), then (-1)^k (1 + k / 4) for 2^k."""
    exps = (0,) + tuple(1 << k for k in range(J + 1))
    return exps, (0.0,) + tuple((-1) ** k * (1.0 + 0.25 * k) for k in range(J + 1))


@pytest.mark.parametrize("J", FOLD_J)
def test_weighted_fold_batched_multitile(tdev, J):
    """The bf16 Gram-basis plan over MULTI_TILE with every power weighted: the sum P that the
    last squaring forms from its own product and the J stored levels, against the oracle's."""
    torch, dev = tdev
    import paper_2602_02500_amd as ifn
    exps, coeffs = fold_terms(J)
    ins = [multi_tile_input(h, tall) for h, tall in MULTI_TILE]
    shapes = [v.shape for v, _ in ins]
    print(f"case weighted fold J={J} shapes {shapes}", flush=True)
    Ms = [torch.from_numpy(v.astype(np.float32)).to(dev).to(torch.bfloat16) for v, _ in ins]
    plan = ifn.Plan(exps, coeffs, shapes, norm="none", compute="bf16", out_dtype=ifn.F32)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    Ys = [torch.full(s, float("nan"), dtype=torch.float32, device=dev) for s in shapes]
    plan.orthogonalize_batched(Ms, Ys, ws)
    torch.cuda.synchronize()
    for (h, tall), (v, alpha), Y in zip(MULTI_TILE, ins, Ys):
        Y = Y.cpu().numpy().astype(np.float64)
        P = oracle.ifnso_parts(v, exps, coeffs, "gram", "none")["P"]
        r = _rel((Y.T if tall else Y)[:, h:] / alpha, P)
        print(f"  h={h} tall={tall} J={J}: rel {r:.2e}")
        assert r <= TOL_BF16_FOLD


@pytest.mark.parametrize("h", [256, 192])
@pytest.mark.parametrize("j", [0, 1, 2, 3, 4])
def test_single_power_e4m3(tdev, h, j):
    """The e4m3 mode stage by stage against the oracle's e4m3 model (the same quantisation
    points, everything else float64). The two sides accumulate in a different order, so a few
    entries of a level that sit at an e4m3 or bf16 rounding boundary round differently and move
    by one step (up to 2^-3 relative for e4m3); a squaring doubles the relative deviation of its
    operand. Bound: (2^(j+1) - 1) 1e-3 for level j (1e-3 for the Gram, 3.1e-2 after four
    squarings); end to end, where the c_0 A term dominates, the same paths stay within 2e-3."""
    torch, dev = tdev
    import paper_2602_02500_amd as ifn
    from oracle import fp8 as F
    exps, coeffs = (0, 1 << j), (0.0, 1.0)
    vals = gen.round_to_bf16_np(_input(h, seed=400 + h))
    Mt = torch.from_numpy(vals.astype(np.float32)).to(dev).to(torch.bfloat16)
    plan = ifn.Plan(exps, coeffs, [(h, 2 * h)], compute="fp8", out_dtype=ifn.F32)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    Y = torch.full((h, 2 * h), float("nan"), dtype=torch.float32, device=dev)
    plan.orthogonalize(Mt, Y, ws)
    torch.cuda.synchronize()
    Ym = F.ifnso_e4m3(vals, exps, coeffs)
    r = _rel(Y.cpu().numpy().astype(np.float64)[:, h:], Ym[:, h:])
    print(f"e4m3 h={h} power 2^{j}: rel vs model {r:.2e}")
    assert r <= (2 ** (j + 1) - 1) * 1e-3
