"""One Muon optimizer step on the GPU (ifnso_muon_step) against the FP64 oracle's step.

The device keeps W and the momentum B in float32 and stores the orthogonalisation input U in
the plan's input type (bf16 here); the oracle runs the same step in float64 and rounds U to
bf16 at the same point. Bounds:
* B' (float32 momentum): relative Frobenius error <= 1e-6 (one float32 multiply-add per entry).
* The weight change W' - W: <= 2e-2, the bf16 orthogonalisation's bound; the decay part is
  float32-exact to ~1e-7.
"""
import numpy as np
import pytest

from oracle import fp8 as F
from oracle import muon as MU
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
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def _setup(torch, dev, shapes, seed, pad=0):
    Ws, Gs, Bs, host = [], [], [], []
    for i, (r, c) in enumerate(shapes):
        W = gen.gaussian_np(r, c, seed + i, 0, 0.02).astype(np.float32)
        G = gen.round_to_bf16_np(gen.lowrank_plus_noise_np(r, c, seed + 100 + i))
        B = gen.gaussian_np(r, c, seed + 200 + i, 0, 0.01).astype(np.float32)
        tw = torch.zeros((r, c + pad), dtype=torch.float32, device=dev)[:, :c]
        tw.copy_(torch.from_numpy(W))
        tg = torch.zeros((r, c + pad), dtype=torch.bfloat16, device=dev)[:, :c]
        tg.copy_(torch.from_numpy(G.astype(np.float32)).to(torch.bfloat16))
        tb = torch.zeros((r, c + pad), dtype=torch.float32, device=dev)[:, :c]
        tb.copy_(torch.from_numpy(B))
        Ws.append(tw)
        Gs.append(tg)
        Bs.append(tb)
        host.append((W.astype(np.float64), G, B.astype(np.float64)))
    return Ws, Gs, Bs, host


def _step(torch, dev, shapes, Ws, Gs, Bs, lr, mu, wd, nesterov):
    import paper_2602_02500_amd as ifn
    exps, c = configs.load_coeffs("gform_v1")
    plan = ifn.Plan(exps, c, shapes, compute="bf16")
    ws = torch.empty(plan.muon_workspace_bytes, dtype=torch.uint8, device=dev)
    plan.muon_step(Ws, Gs, Bs, ws, lr, mu, wd, nesterov)
    torch.cuda.synchronize()
    return exps, c


@pytest.mark.parametrize("nesterov", [True, False])
def test_step_matches_oracle(tdev, nesterov):
    torch, dev = tdev
    shapes = [(256, 512), (512, 256), (200, 456), (100, 203), (64, 96)]
    Ws, Gs, Bs, host = _setup(torch, dev, shapes, seed=70)
    lr, mu, wd = 0.02, 0.95, 0.01
    exps, c = _step(torch, dev, shapes, Ws, Gs, Bs, lr, mu, wd, nesterov)
    for i, (W0, G, B0) in enumerate(host):
        W1o, B1o, _ = MU.muon_step(W0, G, B0, exps, c, lr, mu, wd, nesterov, round_input=F.bf16_round)
        W1 = Ws[i].cpu().numpy().astype(np.float64)
        B1 = Bs[i].cpu().numpy().astype(np.float64)
        rb, rw = _rel(B1, B1o), _rel(W1 - W0, W1o - W0)
        print(f"{shapes[i]} nesterov={nesterov}: momentum rel {rb:.1e}, weight change rel {rw:.2e}")
        assert rb <= 1e-6
        assert rw <= 2e-2


def test_zero_gradient_only_decays(tdev):
    torch, dev = tdev
    shapes = [(128, 320)]
    Ws, Gs, Bs, host = _setup(torch, dev, shapes, seed=80)
    Gs[0].zero_()
    Bs[0].zero_()
    _step(torch, dev, shapes, Ws, Gs, Bs, lr=0.1, mu=0.9, wd=0.25, nesterov=True)
    W0 = host[0][0]
    W1 = Ws[0].cpu().numpy().astype(np.float64)
    assert _rel(W1, (1 - 0.1 * 0.25) * W0) <= 1e-6
    assert not Bs[0].any().item()


def test_padded_rows_take_the_scalar_path(tdev):
    """Leading dimensions that are not a multiple of 4 (no 16-byte rows) give the same step."""
    torch, dev = tdev
    shapes = [(96, 160), (160, 96)]
    a = _setup(torch, dev, shapes, seed=90)
    b = _setup(torch, dev, shapes, seed=90, pad=3)
    for Ws, Gs, Bs, _ in (a, b):
        _step(torch, dev, shapes, Ws, Gs, Bs, lr=0.05, mu=0.9, wd=0.0, nesterov=True)
    for i in range(len(shapes)):
        assert np.allclose(a[0][i].cpu().numpy(), b[0][i].cpu().numpy(), rtol=0, atol=1e-6)
        assert np.allclose(a[2][i].cpu().numpy(), b[2][i].cpu().numpy(), rtol=1e-6, atol=0)


def test_argument_checks(tdev):
    torch, dev = tdev
    import paper_2602_02500_amd as ifn
    exps, c = configs.load_coeffs("gform_v1")
    shapes = [(64, 128)]
    plan = ifn.Plan(exps, c, shapes, compute="bf16")
    Ws, Gs, Bs, _ = _setup(torch, dev, shapes, seed=95)
    small = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)  # the plan's alone is too small
    with pytest.raises(ValueError):  # the binding refuses it before the call
        plan.muon_step(Ws, Gs, Bs, small, 0.1, 0.9)
    # and so does the library itself, called directly
    import ctypes
    L = ifn.load()
    n = len(shapes)
    arr = lambda ts: (ctypes.c_void_p * n)(*[t.data_ptr() for t in ts])  # noqa: E731
    lds = lambda ts: (ctypes.c_int64 * n)(*[t.stride(0) for t in ts])  # noqa: E731
    hp = ifn.MuonParams(0.1, 0.9, 0.0, 1)
    st = L.ifnso_muon_step(plan._h, ctypes.byref(hp), arr(Ws), lds(Ws), arr(Gs), lds(Gs), arr(Bs), lds(Bs),
                           small.data_ptr(), small.numel(), torch.cuda.current_stream().cuda_stream)
    assert st == 3, L.ifnso_last_error()  # IFNSO_ERR_WORKSPACE_TOO_SMALL
    ws = torch.empty(plan.muon_workspace_bytes, dtype=torch.uint8, device=dev)
    with pytest.raises(ifn.IfnsoError):
        plan.muon_step(Ws, Gs, Bs, ws, float("nan"), 0.9)
    with pytest.raises(ifn.IfnsoError):
        plan.muon_step(Ws, Gs, Ws, ws, 0.1, 0.9)  # momentum buffer aliases the weights


def test_learned_plan_in_the_loop(tdev):
    """A Muon step with a learned plan: the coefficient network picks each matrix's polynomial
    inside the step (from the traces of the Gram powers of its own U). The oracle's step with the
    coefficients the device used (plan.stats()) gives the same update: momentum to float32
    rounding, the weight change within the bf16 bound; the network was used for every matrix."""
    torch, dev = tdev
    import oracle
    import paper_2602_02500_amd as ifn
    exps, fixed = configs.load_coeffs("gform_v1")
    theta = oracle.mlp_init(11).astype(np.float32)
    shapes = [(256, 512), (512, 256), (384, 640)]
    Ws, Gs, Bs, host = _setup(torch, dev, shapes, seed=120)
    lr, mu, wd = 0.02, 0.95, 0.01
    plan = ifn.Plan(exps, fixed, shapes, compute="bf16", mlp_params=theta)
    ws = torch.empty(plan.muon_workspace_bytes, dtype=torch.uint8, device=dev)
    plan.muon_step(Ws, Gs, Bs, ws, lr, mu, wd, True)
    torch.cuda.synchronize()
    st = plan.stats()
    for i, (W0, G, B0) in enumerate(host):
        assert st[i][25] == 1.0
        c_dev = np.array(st[i][9:15])
        assert not np.allclose(c_dev, fixed)
        W1o, B1o, _ = MU.muon_step(W0, G, B0, exps, c_dev, lr, mu, wd, True, round_input=F.bf16_round)
        W1 = Ws[i].cpu().numpy().astype(np.float64)
        B1 = Bs[i].cpu().numpy().astype(np.float64)
        rb, rw = _rel(B1, B1o), _rel(W1 - W0, W1o - W0)
        print(f"{shapes[i]} learned: momentum rel {rb:.1e}, weight change rel {rw:.2e}, c = {np.round(c_dev, 3)}")
        assert rb <= 1e-6
        assert rw <= 2e-2


MUON_SAMPLED = [(0, 0), (0, 1), (31, 4)]  # Wq, Wk of layer 0; gate of layer 31


def test_step_on_gradient_set_full_size(tdev):
    """One Nesterov Muon step over the 224 matrices of the gradient set (the Muon benchmark's
    shapes, gradients and hyperparameters; the momentum starts from a seeded nonzero state), in
    one call; sampled matrices against the oracle's step with the bounds above."""
    torch, dev = tdev
    import paper_2602_02500_amd as ifn
    exps, c = configs.load_coeffs("gform_v1")
    lr, mu, wd = 0.02, 0.95, 0.01
    Ws, Gs, Bs, shapes = [], [], [], []
    for layer in range(32):
        for idx, (_, r, cc) in enumerate(configs.LAYER_SHAPES):
            i = len(Ws)
            Ws.append(gen.gaussian_torch(r, cc, 5000 + i, 0, 0.02, device=dev).float())
            m = gen.lowrank_plus_noise_torch(r, cc, configs.d3_seed(layer, idx), device=dev)
            Gs.append(gen.round_to_bf16_torch(m))
            del m
            Bs.append(gen.gaussian_torch(r, cc, 6000 + i, 0, 0.01, device=dev).float())
            shapes.append((r, cc))
    per_layer = len(configs.LAYER_SHAPES)
    host = {k: (Ws[k].double().cpu().numpy(), Gs[k].double().cpu().numpy(), Bs[k].double().cpu().numpy())
            for k in (layer * per_layer + idx for layer, idx in MUON_SAMPLED)}
    print(f"case Muon step, gradient set: {len(Ws)} matrices", flush=True)
    plan = ifn.Plan(exps, c, shapes, compute="bf16")
    ws = torch.empty(plan.muon_workspace_bytes, dtype=torch.uint8, device=dev)
    plan.muon_step(Ws, Gs, Bs, ws, lr, mu, wd, True)
    torch.cuda.synchronize()
    for k, (W0, G, B0) in host.items():
        W1o, B1o, _ = MU.muon_step(W0, G, B0, exps, c, lr, mu, wd, True, round_input=F.bf16_round)
        W1 = Ws[k].cpu().numpy().astype(np.float64)
        B1 = Bs[k].cpu().numpy().astype(np.float64)
        rb, rw = _rel(B1, B1o), _rel(W1 - W0, W1o - W0)
        print(f"  matrix {k} {shapes[k]}: momentum rel {rb:.1e}, weight change rel {rw:.2e}")
        assert rb <= 1e-6
        assert rw <= 2e-2
