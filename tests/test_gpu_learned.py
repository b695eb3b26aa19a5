"""Learned coefficients on the GPU: kernels against the FP64 oracle, training determinism,
the learned plan end to end, and the gain of a trained network over the fixed coefficients."""
import numpy as np
import pytest

import oracle
from oracle import bf16_model
from workloads import configs, gen, spectra

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tdev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_02500_amd as ifn
    ifn.load()
    return torch, torch.device("cuda:0")


def _spectra_dev(torch, dev, samples, smax=1024):
    sig, nsig = spectra.pad_spectra(samples, smax)
    return torch.from_numpy(sig).to(dev), torch.from_numpy(nsig).to(dev)


def test_features_match_oracle(tdev):
    torch, dev = tdev
    import paper_2602_02500_amd as ifn
    samples = spectra.spectral_mixture(12, seed=21)
    sig, nsig = _spectra_dev(torch, dev, samples)
    feats = torch.empty((len(samples), 8), dtype=torch.float32, device=dev)
    ifn.mlp_features(sig, nsig, feats)
    got = feats.cpu().numpy()
    for i, (_, _, s) in enumerate(samples):
        want = oracle.features_from_spectrum(s.astype(np.float32).astype(np.float64))
        assert np.max(np.abs(got[i] - want)) < 1e-5 * max(1.0, np.max(np.abs(want))), i


def test_forward_matches_oracle(tdev):
    torch, dev = tdev
    import paper_2602_02500_amd as ifn
    theta = oracle.mlp_init(1).astype(np.float32)
    feats = np.stack([oracle.features_from_spectrum(s) for _, _, s in spectra.spectral_mixture(6, seed=3)])
    f_d = torch.from_numpy(feats.astype(np.float32)).to(dev)
    p_d = torch.from_numpy(theta).to(dev)
    out = torch.empty((6, 6), dtype=torch.float64, device=dev)
    ifn.mlp_forward(f_d, p_d, out)
    got = out.cpu().numpy()
    for i in range(6):
        want, _ = oracle.mlp_forward(theta.astype(np.float64), feats[i].astype(np.float32).astype(np.float64))
        assert np.max(np.abs(got[i] - want)) < 1e-5 * max(1.0, np.max(np.abs(want)))


def test_train_step_gradient_matches_oracle(tdev):
    """FP32 device backprop vs FP64 oracle backprop on the same batch (lr = 0 leaves theta)."""
    torch, dev = tdev
    import paper_2602_02500_amd as ifn
    theta = oracle.mlp_init(2).astype(np.float32)
    samples = spectra.spectral_mixture(16, seed=33, hmax=512)
    sig, nsig = _spectra_dev(torch, dev, samples, smax=512)
    feats = torch.empty((16, 8), dtype=torch.float32, device=dev)
    ifn.mlp_features(sig, nsig, feats)
    p_d = torch.from_numpy(theta).to(dev)
    m = torch.zeros_like(p_d)
    v = torch.zeros_like(p_d)
    g = torch.empty_like(p_d)
    lo = torch.empty(1, dtype=torch.float32, device=dev)
    ws = torch.empty(ifn.mlp_train_workspace_bytes(16), dtype=torch.uint8, device=dev)
    ifn.mlp_train_step(feats, sig, nsig, p_d, m, v, 1, 0.0, ws, grad_out=g, loss_out=lo)
    torch.cuda.synchronize()
    fh = feats.cpu().numpy().astype(np.float64)
    batch = [(fh[i], s.astype(np.float32).astype(np.float64)) for i, (_, _, s) in enumerate(samples)]
    loss, grad = oracle.mlp_loss_and_grad(theta.astype(np.float64), batch)
    gd = g.cpu().numpy().astype(np.float64)
    assert abs(lo.item() - loss) <= 1e-4 * max(1.0, loss)
    assert np.linalg.norm(gd - grad) <= 1e-4 * np.linalg.norm(grad)
    assert np.array_equal(p_d.cpu().numpy(), theta)  # lr = 0


def test_training_is_deterministic(tdev):
    torch, dev = tdev
    from paper_2602_02500_amd import learn
    samples = spectra.spectral_mixture(512, seed=44, hmax=256)
    sig, nsig = _spectra_dev(torch, dev, samples, smax=256)
    outs = []
    for _ in range(2):
        p = torch.from_numpy(oracle.mlp_init(5).astype(np.float32)).to(dev)
        learn.train(sig, nsig, p, epochs=2, batch=64, lr=3e-3)
        outs.append(p.cpu().numpy())
    assert np.array_equal(outs[0].view(np.uint32), outs[1].view(np.uint32))


def test_learned_plan_matches_oracle(tdev):
    """A learned plan: its per-matrix coefficients equal the oracle network on the oracle's
    traces, and its output equals the oracle polynomial with those coefficients."""
    torch, dev = tdev
    import paper_2602_02500_amd as ifn
    theta = oracle.mlp_init(8).astype(np.float32)
    exps, fixed = configs.load_coeffs("gform_v1")
    shapes = [(256, 512), (512, 768), (384, 256)]
    Ms, vals = [], []
    for i, s in enumerate(shapes):
        v = gen.round_to_bf16_np(gen.gaussian_np(*s, seed=70 + i))
        vals.append(v)
        Ms.append(torch.from_numpy(v.astype(np.float32)).to(dev).to(torch.bfloat16))
    plan = ifn.Plan(exps, fixed, shapes, compute="bf16", mlp_params=theta)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    Ys = [torch.empty_like(m) for m in Ms]
    plan.orthogonalize_batched(Ms, Ys, ws)
    st = plan.stats()
    for i, v in enumerate(vals):
        sig = np.linalg.svd(v, compute_uv=False)
        phi = oracle.features_from_spectrum(sig)
        # log2 m_j on the device against the exact spectrum's, per j: within three times what the
        # bf16 storage-point model of the trace computation deviates (up to 0.04 for m_7 on these
        # inputs) plus 1e-4 for float32 accumulation
        l2m = phi * (8 * 2.0 ** np.arange(8))
        dev_l2m = np.array(st[i][1:9])
        bound = 3.0 * np.abs(bf16_model.gram_traces(v) - l2m) + 1e-4
        print(f"  problem {i}: |log2 m_j| deviations {np.abs(dev_l2m - l2m)}, bounds {bound}")
        assert np.all(np.abs(dev_l2m - l2m) <= bound), i
        c_or, _ = oracle.mlp_forward(theta.astype(np.float64), phi)
        c_gpu = np.array(st[i][9:15])
        assert st[i][25] == 1.0
        assert np.max(np.abs(c_gpu - c_or)) < 1e-3 * max(1.0, np.max(np.abs(c_or)))
        Yo = oracle.ifnso(v, exps, c_gpu)
        Yd = Ys[i].float().cpu().numpy().astype(np.float64)
        assert np.linalg.norm(Yd - Yo) / np.linalg.norm(Yo) < 2e-2


def test_trained_network_beats_fixed_coefficients(tdev):
    """Train on the GPU on the seeded spectral mixture, then compare the mean polar distance
    (the training loss) on held-out spectra with the fixed-coefficient fallback."""
    torch, dev = tdev
    from paper_2602_02500_amd import learn
    train_s = spectra.spectral_mixture(8192, seed=5)
    sig, nsig = _spectra_dev(torch, dev, train_s)
    p = torch.from_numpy(oracle.mlp_init(0).astype(np.float32)).to(dev)
    learn.train(sig, nsig, p, epochs=3, batch=256, lr=2e-3)
    theta = p.cpu().numpy().astype(np.float64)
    _, fixed = configs.load_coeffs("gform_v1")
    held = spectra.spectral_mixture(300, seed=6)
    lf, ll = [], []
    for _, _, s in held:
        c, _ = oracle.mlp_forward(theta, oracle.features_from_spectrum(s))
        ll.append(oracle.spectral_loss(c, s)[0])
        lf.append(oracle.spectral_loss(fixed, s)[0])
    print(f"held-out mean polar distance^2/h: learned {np.mean(ll):.4f}, fixed {np.mean(lf):.4f}")
    assert np.mean(ll) < 0.8 * np.mean(lf)


# learned plan at full size: the gradient set with a network trained on the device as the learned
# benchmark trains it. The bound is computed per matrix: four times the bf16 storage-point model's
# error (oracle.bf16_model.gram_levels) on the same input with the device's coefficients, which
# reach magnitudes of 400 with alternating signs (the device follows the model to three digits),
# and never above the bf16 path's 2e-2.
LEARNED_SAMPLED = [(0, 0), (0, 1), (31, 4), (31, 6)]  # Wq, Wk of layer 0; gate, down of layer 31


def test_learned_plan_gradient_set_full_size(tdev):
    """Train the network on the benchmark's seeded spectra (3 epochs), run the learned plan over
    the 224 matrices of the gradient set in one batched call, and compare sampled matrices with
    the float64 polynomial under the coefficients the device chose for each."""
    torch, dev = tdev
    import paper_2602_02500_amd as ifn
    from paper_2602_02500_amd import learn
    exps, fixed = configs.load_coeffs("gform_v1")
    sig, nsig = _spectra_dev(torch, dev, spectra.spectral_mixture(100000, seed=5))
    params = torch.from_numpy(gen.fan_in_uniform_np(0, learn.PARAM_LAYOUT).astype(np.float32)).to(dev)
    learn.train(sig, nsig, params, epochs=3, batch=256, lr=2e-3)
    theta = params.cpu().numpy()
    Ms = []
    for layer in range(32):
        for idx, (_, r, c) in enumerate(configs.LAYER_SHAPES):
            m = gen.lowrank_plus_noise_torch(r, c, configs.d3_seed(layer, idx), device=dev)
            Ms.append(gen.round_to_bf16_torch(m))
            del m
    shapes = [tuple(m.shape) for m in Ms]
    print(f"case learned plan, gradient set: {len(Ms)} matrices", flush=True)
    plan = ifn.Plan(exps, fixed, shapes, compute="bf16", mlp_params=theta)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    Ys = [torch.empty_like(m) for m in Ms]
    plan.orthogonalize_batched(Ms, Ys, ws)
    torch.cuda.synchronize()
    st = plan.stats()
    for layer, idx in LEARNED_SAMPLED:
        k = layer * len(configs.LAYER_SHAPES) + idx
        assert st[k][25] == 1.0  # the network's coefficients, not the fallback
        c = np.array(st[k][9:15])
        vals = Ms[k].double().cpu().numpy()
        Yo = oracle.ifnso(vals, exps, c)
        model = np.linalg.norm(bf16_model.gram_levels(vals, exps, c) - Yo) / np.linalg.norm(Yo)
        r = np.linalg.norm(Ys[k].double().cpu().numpy() - Yo) / np.linalg.norm(Yo)
        print(f"  layer {layer} {configs.LAYER_SHAPES[idx][0]}: coefficients {np.round(c, 1)}, "
              f"rel vs the polynomial {r:.3e} (model {model:.3e})")
        assert r <= min(4.0 * model, 2e-2), (layer, idx, r, model)
