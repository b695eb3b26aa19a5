"""Full-size parity: the two single matrices of the FP32-versus-BF16 workload (4096x4096 and
14336x4096, U diag(sigma) V^T with Haar factors and sigma log-uniform on [1e-3, 1], seeds 1 and 2)
through one batched plan, as the benchmark launches it, against the exact result. For a matrix
with known singular value decomposition the method's output is U diag(f(sigma~)) V^T with
f(x) = x p(x^2) (the oracle's closed form), so no float64 run of the whole method is needed at
this size.

Bounds: float32 path 1e-4. bfloat16 path 2e-2; it includes the bfloat16 rounding of the input
(about 1e-3 relative in the output, since the polynomial is close to linear at these sigma~)."""
import numpy as np
import pytest

import oracle
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


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_d2_pair_against_closed_form(tdev):
    torch, dev = tdev
    import paper_2602_02500_amd as ifn
    exps, c = configs.load_coeffs("gform_v1")
    cases = [(4096, 4096, 1), (14336, 4096, 2)]
    mats, closed = [], []
    for rows, cols, seed in cases:
        print(f"case d2 {rows}x{cols} seed {seed}", flush=True)
        sigma = configs.d2_sigma_np(min(rows, cols), seed)
        M, U, V = gen.spectral_torch(rows, cols, sigma, seed, device=dev)
        closed.append(oracle.closed_form(U.cpu().numpy(), sigma, V.cpu().numpy(), exps, c))
        mats.append(M)
        del U, V
    shapes = [tuple(m.shape) for m in mats]
    for compute, dt, tol in [("f32", torch.float32, 1e-4), ("bf16", torch.bfloat16, 2e-2)]:
        plan = ifn.Plan(exps, c, shapes, compute=compute)
        Ms = [m.to(dt).contiguous() for m in mats]
        Ys = [torch.empty_like(m) for m in Ms]
        ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
        plan.orthogonalize_batched(Ms, Ys, ws)
        plan.orthogonalize_batched(Ms, Ys, ws)  # the replayed graph
        torch.cuda.synchronize()
        for (rows, cols, _), Y, Yc in zip(cases, Ys, closed):
            r = _rel(Y.double().cpu().numpy(), Yc)
            print(f"  {compute} {rows}x{cols}: rel vs closed form {r:.3e}")
            assert r <= tol, (compute, rows, cols, r)
        del ws, Ys, Ms, plan


def test_d2_pair_schedule_against_closed_form(tdev):
    """Muon's five Newton-Schulz steps through chained batched plans (the `ns` benchmark's
    launch configuration) on the same pair: the iteration acts on singular values only, so the
    exact result is U diag(phi(sigma / ||sigma||)) V^T with phi the composed scalar map.
    Bounds: float32 1e-4; bfloat16 0.1, three times what a float64 model of the bf16 storage
    points (input, Gram operand, P, iterates) gives on a 1024x3584 matrix with the same
    spectrum law (3.4e-2)."""
    torch, dev = tdev
    import paper_2602_02500_amd as ifn
    from oracle import baselines as BL
    sched, q = configs.load_schedule("muon_ns5")
    cases = [(4096, 4096, 1), (14336, 4096, 2)]
    mats, closed = [], []
    for rows, cols, seed in cases:
        print(f"case d2 schedule {rows}x{cols} seed {seed}", flush=True)
        sigma = configs.d2_sigma_np(min(rows, cols), seed)
        M, U, V = gen.spectral_torch(rows, cols, sigma, seed, device=dev)
        f = BL.compose_scalar(sigma / np.sqrt(np.sum(sigma ** 2)), sched)
        closed.append((U.cpu().numpy() * f) @ V.cpu().numpy().T)
        mats.append(M)
        del U, V
    shapes = [tuple(m.shape) for m in mats]
    for compute, dt, tol in [("f32", torch.float32, 1e-4), ("bf16", torch.bfloat16, 0.1)]:
        sp = ifn.SchedulePlan(sched, shapes, gelfand_q=q, compute=compute)
        Ms = [m.to(dt).contiguous() for m in mats]
        Ys = [torch.empty_like(m) for m in Ms]
        tmp = [torch.empty_like(m) for m in Ms]
        ws = torch.empty(sp.workspace_bytes, dtype=torch.uint8, device=dev)
        sp.orthogonalize_batched(Ms, Ys, ws, tmp)
        torch.cuda.synchronize()
        for (rows, cols, _), Y, Yc in zip(cases, Ys, closed):
            r = _rel(Y.double().cpu().numpy(), Yc)
            print(f"  {compute} {rows}x{cols}: rel vs closed form {r:.3e}")
            assert r <= tol, (compute, rows, cols, r)
        del ws, Ys, Ms, tmp, sp
