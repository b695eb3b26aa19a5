"""ifnso_orthogonalize_static, the entry point that allocates nothing: its fixed scratch area
gives the same bits as ifnso_orthogonalize with a workspace, call after call, including a
smaller problem after a larger one (the area keeps the previous call's contents) and the
split-Gram path whose chunk counters live in the workspace; plans that need more than the
area are refused before anything is enqueued."""
import ctypes

import numpy as np
import pytest

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


def _case(torch, dev, shape, compute, basis, norm, coeffs_name, seed):
    import paper_2602_02500_amd as ifn
    exps, c = configs.load_coeffs(coeffs_name)
    M = gen.gaussian_np(*shape, seed=seed)
    if compute == "f32":
        Mt = torch.from_numpy(M.astype(np.float32)).to(dev)
    else:
        Mt = torch.from_numpy(gen.round_to_bf16_np(M).astype(np.float32)).to(dev).to(torch.bfloat16)
    plan = ifn.Plan(exps, c, [shape], basis=basis, norm=norm, compute=compute)
    assert plan.workspace_bytes <= ifn.STATIC_SCRATCH_BYTES
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    Yr = torch.full_like(Mt, float("nan"))
    plan.orthogonalize(Mt, Yr, ws)
    return plan, Mt, Yr


CASES = [
    # (shape, compute, basis, norm, coefficients, seed): the second of each pair is smaller
    ((520, 1100), "bf16", "gram", "frobenius", "gform_v1", 1),
    ((200, 456), "bf16", "gram", "frobenius", "gform_v1", 2),
    ((128, 4096), "f32", "complement", "gram_frobenius", "paper_L14", 3),   # split Gram (counters)
    ((100, 3000), "f32", "complement", "gram_frobenius", "paper_L14", 4),
]


def test_static_entry_matches_workspace_entry(tdev):
    torch, dev = tdev
    import paper_2602_02500_amd as ifn
    L = ifn.load()
    stream = torch.cuda.current_stream().cuda_stream
    for shape, compute, basis, norm, name, seed in CASES:
        print(f"case static {shape} {compute} {basis}", flush=True)
        plan, Mt, Yr = _case(torch, dev, shape, compute, basis, norm, name, seed)
        for rep in range(2):
            Ys = torch.full_like(Mt, float("nan"))
            if rep == 0:  # straight through the C ABI
                st = L.ifnso_orthogonalize_static(plan._h, Mt.data_ptr(), Mt.stride(0), Ys.data_ptr(), Ys.stride(0),
                                                  stream)
                assert st == 0, L.ifnso_last_error()
            else:
                plan.orthogonalize_static(Mt, Ys)
            torch.cuda.synchronize()
            assert torch.equal(Ys.float(), Yr.float()), (shape, rep)


def test_static_entry_refuses_large_plans(tdev):
    torch, dev = tdev
    import paper_2602_02500_amd as ifn
    L = ifn.load()
    exps, c = configs.load_coeffs("gform_v1")
    plan = ifn.Plan(exps, c, [(4096, 4096)], compute="bf16")
    assert plan.workspace_bytes > ifn.STATIC_SCRATCH_BYTES
    st = L.ifnso_orthogonalize_static(plan._h, 0, 4096, 0, 4096, torch.cuda.current_stream().cuda_stream)
    assert st == 3, L.ifnso_last_error()  # IFNSO_ERR_WORKSPACE_TOO_SMALL, before any argument is used
