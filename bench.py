"""Throughput of the batched IFNSO path on one MI355X.

Workload (the metric's configuration): the weight-gradient set of a synthetic 32-layer
transformer, hidden size 4096 with GQA and SwiGLU -- per layer Wq, Wo 4096x4096, Wk, Wv
1024x4096, gate, up 14336x4096, down 4096x14336 (224 matrices); bfloat16 entries
N(0, 0.02^2) plus a rank-16 component of Frobenius norm 0.5, generated on the device from
the seeded counter generator. Exponents {0,1,2,4,8,16}, fixed coefficients "gform_v1".
One step = one batched call over all 224 matrices (Gram, 4 squarings, product).

Prints one JSON line. `value` is matrices/s over the timed region, with the inputs
already resident in HBM. The roofline entry is for the kernel with the largest time per
step, timed with HIP events recorded around each stage inside the timed region.

`--workload e4m3` measures the e4m3 variant instead: 64 matrices 2048x8192 built as
U diag(sigma) V^T with Haar factors and sigma_i = i^-1.5 (seed 3), e4m3 Gram and squarings
with per-tensor scales, bfloat16 aggregation and product; it reports the error of the
e4m3 and bfloat16 modes against the FP64 oracle on a sample of the batch. `--workload
learned` trains the coefficient network and runs the set with it; `--workload tform` runs
the paper's complement-basis form (depth 14) on the set in bfloat16; `--workload muon` runs
whole Muon optimizer steps on the set; `--workload table1` reproduces the paper's Table 1
comparison (five methods, three sizes) on the device; `--workload ns` runs the
Newton-Schulz baselines on the gradient set through the batched path, beside IFNSO.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_BF16_TFLOPS = 2500.0  # MI355X dense bf16 MFMA
PEAK_FP8_TFLOPS = 5000.0   # MI355X dense fp8 MFMA
PEAK_F32_TFLOPS = 157.3    # MI355X dense fp32 MFMA


def _hip():
    lib = ctypes.CDLL("libamdhip64.so")
    lib.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    lib.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
    lib.hipEventSynchronize.argtypes = [ctypes.c_void_p]
    lib.hipEventDestroy.argtypes = [ctypes.c_void_p]
    return lib


def make_d3(torch, dev, layers=32):
    from workloads import configs, gen
    Ms = []
    for l in range(layers):
        for idx, (_, r, c) in enumerate(configs.LAYER_SHAPES):
            m = gen.lowrank_plus_noise_torch(r, c, configs.d3_seed(l, idx), device=dev)
            Ms.append(gen.round_to_bf16_torch(m))
            del m
    torch.cuda.synchronize()
    return Ms


def schedule(args, torch, plan, Ms, Ys, ws, compute, exps, log):
    """Applies cached tuned schedules for this plan, or tunes them (--tune). Returns a record."""
    from paper_2602_02500_amd import tune
    props = torch.cuda.get_device_properties(0)
    device = f"{getattr(props, 'gcnArchName', 'gpu').split(':')[0]}-{props.multi_processor_count}cu"
    key = tune.plan_key(device, [tuple(m.shape) for m in Ms], compute, exps)
    if args.tune:
        res = tune.tune(plan, Ms, Ys, ws, log=log)
        os.makedirs(os.path.dirname(args.tune_out), exist_ok=True)
        tune.save_cache(args.tune_out, key, res, note=f"{len(Ms)} matrices, compute {compute}")
        return {"source": "tuned now", "key": key, "stages": {k: v["config"] for k, v in res.items()},
                "ms": {k: [v["default_ms"], v["ms"]] for k, v in res.items()}}
    entry = tune.load_cache(args.schedules).get(key)
    if entry:
        tune.apply(plan, entry)
        return {"source": os.path.relpath(args.schedules, ROOT), "key": key, "stages": entry["stages"]}
    return {"source": "defaults", "key": key}


def make_e4m3_set(torch, dev, batch):
    from workloads import configs, gen
    r, c = configs.D4_SHAPE
    sigma = configs.d4_sigma(min(r, c))
    Ms = []
    for i in range(batch):
        m, u, v = gen.spectral_torch(r, c, sigma, configs.d4_seed(i), device=dev)
        Ms.append(gen.round_to_bf16_torch(m))
        del m, u, v
    torch.cuda.synchronize()
    return Ms


def stage_flops(shapes, J):
    """Algorithmic flops per launch: Gram h^2 w (symmetric), squaring h^3 (symmetric),
    product 2 h^2 w, summed over the problems of the launch."""
    g = sum(min(r, c) ** 2 * max(r, c) for r, c in shapes)
    s = sum(min(r, c) ** 3 for r, c in shapes)
    p = sum(2 * min(r, c) ** 2 * max(r, c) for r, c in shapes)
    return {"gram": float(g), "square": float(s), "product": float(p), "step": float(g + J * s + p)}


# kernel of a bench launch name -> its name in the rocprofv3 traffic summary
PROFILE_KERNEL = {"square": "kf_square<true, false, false>", "square_last": "kf_square<true, false, true>",
                  "gram_wide": "kf_gram<false, false>",
                  "gram_tall": "kf_gram<true, false>", "product_wide": "kf_product<false, false>",
                  "product_tall": "kf_product<true, false>",
                  "aggregate": "kf_aggregate"}
# the e4m3 workload: only its bf16 products come from the source file the summary's hash covers
E4M3_PROFILE_KERNEL = {"product_wide": "kf_product<false, false>", "product_tall": "kf_product<true, false>"}
# the paper's form with split bf16 operands: the squaring over K = 3 hp
TFORM_PROFILE_KERNEL = {"square": "kf_square<false, true, false>"}


def _attach_traffic(line, kernel, summary, names=None):
    """Adds the measured HBM bytes per launch of `kernel` to the line's roofline, when known."""
    tr = measured_traffic(kernel, os.path.join(ROOT, "profiles", summary), names)
    if tr is not None:
        line["roofline"].update({"traffic": round(tr["bytes"]), "traffic_read": round(tr["read"]),
                                 "traffic_write": round(tr["write"]), "traffic_source": tr["source"]})


def measured_traffic(kernel, summary, names=None):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary
    (calibrated against a plain copy of known size), or None when the summary is missing, lacks
    the kernel, or was taken on a different revision of the kernel source."""
    import hashlib
    try:
        with open(summary) as f:
            prof = json.load(f)
        with open(os.path.join(ROOT, prof["source"]), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != prof["source_sha256"]:
                return None
        k = prof["kernels"][(names or PROFILE_KERNEL)[kernel]]
    except (OSError, KeyError, ValueError):
        return None
    return {"bytes": k["read_bytes"] + k["write_bytes"], "read": k["read_bytes"], "write": k["write_bytes"],
            "source": os.path.relpath(summary, ROOT)}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(Ms_host, exps, coeffs, Ys_dev):
    """The FP64 oracle on a bounded sample (layer 0: its 7 matrices), on the host cores; then
    layer 0's two 1024x4096 matrices again on one thread."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    import oracle
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    t0 = time.perf_counter()
    outs = [oracle.ifnso(M, exps, coeffs) for M in Ms_host]
    dt = time.perf_counter() - t0
    rel = []
    for Yo, Yd in zip(outs, Ys_dev):
        rel.append(float(np.linalg.norm(Yd - Yo) / np.linalg.norm(Yo)))
    orth = [oracle.orth_error(Yo) / math.sqrt(min(Yo.shape)) for Yo in outs]
    small = [M for M in Ms_host if min(M.shape) == 1024][:2]
    with threadpool_limits(1):
        t1 = time.perf_counter()
        for M in small:
            oracle.ifnso(M, exps, coeffs)
        dt1 = time.perf_counter() - t1
    return {"value": len(Ms_host) / dt, "unit": "matrices/s", "cores": int(threads), "kind": "oracle",
            "sample": f"layer 0 of the set ({len(Ms_host)} matrices: 2x 4096x4096, 2x 1024x4096, "
                      f"2x 14336x4096, 1x 4096x14336), float64 numpy, {dt:.1f} s",
            "cpu_model": _cpu_model(), "host_cpus": os.cpu_count(),
            "one_core": {"value": len(small) / dt1, "unit": "matrices/s", "threads": 1,
                         "sample": f"layer 0's {len(small)} matrices of 1024x4096 on one thread, {dt1:.2f} s"}}, \
        rel, orth


def _oracle_threads():
    from threadpoolctl import threadpool_info
    return int(max([i.get("num_threads", 1) for i in threadpool_info()] or [1]))


def cpu_baseline_learned(theta, coeffs, held):
    """The FP64 oracle on the coefficient-network part of the learned workload: features,
    network and polar distance^2 / h of the learned and the fixed polynomial for each held-out
    spectrum."""
    import numpy as np

    import oracle
    t0 = time.perf_counter()
    ll, lf = [], []
    for _, _, sgm in held:
        c, _ = oracle.mlp_forward(np.asarray(theta, dtype=np.float64), oracle.features_from_spectrum(sgm))
        ll.append(oracle.spectral_loss(c, sgm)[0])
        lf.append(oracle.spectral_loss(coeffs, sgm)[0])
    dt = time.perf_counter() - t0
    cpu = {"value": len(held) / dt, "unit": "spectra/s", "cores": _oracle_threads(), "kind": "oracle",
           "cpu_model": _cpu_model(),
           "sample": f"{len(held)} held-out spectra: features, network, polar distance of the learned and "
                     f"fixed polynomials, float64 numpy, {dt:.1f} s"}
    return cpu, {"learned": float(np.mean(ll)), "fixed": float(np.mean(lf)), "spectra": len(held)}


def cpu_baseline_tform(Mh, Yd, exps, coeffs):
    """The FP64 oracle of the complement-basis form on a bounded sample (host matrices `Mh`),
    with the relative distance of the device results `Yd` and the oracle's orthogonality error."""
    import numpy as np

    import oracle
    t0 = time.perf_counter()
    outs = [oracle.ifnso(M, exps, coeffs, "complement", "gram_frobenius") for M in Mh]
    dt = time.perf_counter() - t0
    rel = [float(np.linalg.norm(Y - Yo) / np.linalg.norm(Yo)) for Y, Yo in zip(Yd, outs)]
    orth = [float(oracle.orth_error(Yo) / np.sqrt(min(Yo.shape))) for Yo in outs]
    cpu = {"value": len(Mh) / dt, "unit": "matrices/s", "cores": _oracle_threads(), "kind": "oracle",
           "cpu_model": _cpu_model(),
           "sample": f"layer 0's {len(Mh)} matrices of 1024x4096, complement basis, depth 14, float64 numpy, "
                     f"{dt:.1f} s"}
    return cpu, rel, orth


def slot_names(plan):
    """Kernel name of each launch slot of a Gram-basis bf16 plan, from the stage the library
    reports for it (the two Grams and products are the wide and the tall list)."""
    names, g, p = [], 0, 0
    for i in range(plan.num_launches):
        st = plan.launch_info(i)[0]
        if st == 0:
            names.append(("gram_wide", "gram_tall")[g])
            g += 1
        elif st == 1:
            names.append("square")
        elif st == 2:
            names.append(("product_wide", "product_tall")[p])
            p += 1
        else:
            names.append("aggregate" if st == 3 else "prep")
    return names


def roofline_of(kern):
    """The roofline object of the kernel with the largest time per step (bf16 MFMA peak)."""
    dom = max((k for k in kern if kern[k][2] > 0), key=lambda k: kern[k][0])
    dur_ms = kern[dom][0] / kern[dom][1]
    achieved = kern[dom][2] / kern[dom][1] / (dur_ms * 1e-3) / 1e12
    return dom, {"bound": "mfma", "kernel": dom, "achieved": round(achieved, 2), "peak": PEAK_BF16_TFLOPS,
                 "unit": "TFLOP/s", "frac": round(achieved / PEAK_BF16_TFLOPS, 4), "traffic": None,
                 "avg_launch_ms": round(dur_ms, 3)}


def time_plan(torch, hip, plan, Ms, Ys, ws, names, steps, warmup, log, slots=True):
    """Warm-up calls, then the timed region: `steps` calls as a user makes them (the plan's
    captured graph replayed), bracketed by torch.cuda.synchronize() and timed by the wall clock
    and by HIP events around the whole region on the calls' stream. Then, unless `slots` is
    false, a separate pass of `steps` calls with a HIP event before every launch slot and one
    after the last (launched directly, not from the graph) for the per-kernel times. Returns
    per-kernel (ms per step, launches per step, algorithmic flops per step), the timed wall
    time, the event time of the timed region and the per-slot pass's ms per step."""
    import numpy as np
    nl = plan.num_launches
    info = [plan.launch_info(i) for i in range(nl)]
    for _ in range(warmup):
        plan.orthogonalize_batched(Ms, Ys, ws)
    torch.cuda.synchronize()
    log("warmup done")

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        plan.orthogonalize_batched(Ms, Ys, ws)
    e1.record()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    event_ms = e0.elapsed_time(e1)
    log(f"timed {steps} steps: {elapsed:.3f} s")
    if not slots:
        return {"kern": {}, "elapsed": elapsed, "event_ms": event_ms, "slot_pass_ms": None, "slot_ms": None}

    # per-slot pass: a HIP event before every launch slot and one after the last
    evs = []
    for _ in range(steps):
        row = []
        for _ in range(nl + 1):
            e = ctypes.c_void_p()
            assert hip.hipEventCreate(ctypes.byref(e)) == 0
            row.append(e.value)
        evs.append(row)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(steps):
        plan.launch_events(evs[k])
        plan.orthogonalize_batched(Ms, Ys, ws)
    torch.cuda.synchronize()
    slot_pass_ms = (time.perf_counter() - t1) / steps * 1e3
    slot_ms = np.zeros((steps, nl))
    f = ctypes.c_float()
    for k in range(steps):
        for i in range(nl):
            assert hip.hipEventElapsedTime(ctypes.byref(f), evs[k][i], evs[k][i + 1]) == 0
            slot_ms[k, i] = f.value
    for row in evs:
        for e in row:
            hip.hipEventDestroy(e)
    per = slot_ms.mean(axis=0)
    kern = {}
    for i, nm in enumerate(names):
        t, n_l, flop = kern.get(nm, (0.0, 0, 0.0))
        if info[i][1] > 0 or (info[i][0] in (3, 4) and per[i] > 0.001):  # memory-bound slots
            kern[nm] = (t + per[i], n_l + 1, flop + info[i][1])
    return {"kern": kern, "elapsed": elapsed, "event_ms": event_ms, "slot_pass_ms": slot_pass_ms, "slot_ms": per}


def run_e4m3(args, torch, dev, hip, log):
    import numpy as np

    import paper_2602_02500_amd as ifn
    from workloads import configs
    exps, coeffs = configs.load_coeffs("gform_v1")
    t0 = time.perf_counter()
    Ms = make_e4m3_set(torch, dev, args.batch)
    shapes = [tuple(m.shape) for m in Ms]
    n = len(Ms)
    log(f"generated {n} matrices in {time.perf_counter() - t0:.1f} s")
    Ys = [torch.empty_like(m) for m in Ms]
    plan = ifn.Plan(exps, coeffs, shapes, compute="fp8")
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    log(f"workspace {plan.workspace_bytes / 2**30:.1f} GiB")
    sched = schedule(args, torch, plan, Ms, Ys, ws, "fp8", exps, log)
    nl = plan.num_launches
    J = nl - 6
    fl = stage_flops(shapes, J)
    names = ["prepass_quant", "gram8_wide", "gram8_tall"] + ["square8"] * (J - 1) + ["square8_last"] + \
            ["aggregate", "product_wide", "product_tall"]
    t = time_plan(torch, hip, plan, Ms, Ys, ws, names, args.steps, args.warmup, log)
    kern, elapsed = t["kern"], t["elapsed"]
    slot = t["slot_ms"]
    ms_per_step = elapsed / args.steps * 1e3
    value = n * args.steps / elapsed
    peak = {"gram8_wide": PEAK_FP8_TFLOPS, "gram8_tall": PEAK_FP8_TFLOPS, "square8": PEAK_FP8_TFLOPS,
            "square8_last": PEAK_FP8_TFLOPS, "product_wide": PEAK_BF16_TFLOPS, "product_tall": PEAK_BF16_TFLOPS}
    dom = max((k for k in kern if kern[k][2] > 0), key=lambda k: kern[k][0])
    dur_ms = kern[dom][0] / kern[dom][1]
    achieved = kern[dom][2] / kern[dom][1] / (dur_ms * 1e-3) / 1e12
    # mixed roofline of the step: e4m3 Gram and squarings, bfloat16 product
    t_min_ms = ((fl["gram"] + J * fl["square"]) / (PEAK_FP8_TFLOPS * 1e12) + fl["product"] / (PEAK_BF16_TFLOPS * 1e12)) * 1e3
    hw = sum(r * c for r, c in shapes)
    prep_bytes = 5.0 * hw  # pre-pass reads M, quantisation reads M and writes e4m3 A
    extra = {"event_ms_per_step": round(t["event_ms"] / args.steps, 3),
             "slot_pass_ms_per_step": round(t["slot_pass_ms"], 3), "schedules": sched,
             "kernels": {k: {"ms_per_step": round(v[0], 3), "launches": v[1],
                             "tflops": round(v[2] / (v[0] * 1e-3) / 1e12, 1) if v[0] > 0 and v[2] > 0 else None}
                         for k, v in kern.items()},
             "prepass_quant_gbps": round(prep_bytes / (slot[0] * 1e-3) / 1e9, 1) if slot[0] > 0 else None,
             "algorithmic_tflop_per_step": round(fl["step"] / 1e12, 3),
             "mixed_roofline_ms": round(t_min_ms, 3), "mixed_roofline_frac": round(t_min_ms / ms_per_step, 4)}
    # the same batch in bfloat16, for the speed ratio and the error comparison
    Yb = [torch.empty_like(m) for m in Ms]
    del ws
    planb = ifn.Plan(exps, coeffs, shapes, compute="bf16")
    wsb = torch.empty(planb.workspace_bytes, dtype=torch.uint8, device=dev)
    planb.orthogonalize_batched(Ms, Yb, wsb)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    for _ in range(3):
        planb.orthogonalize_batched(Ms, Yb, wsb)
    torch.cuda.synchronize()
    tb = (time.perf_counter() - tb) / 3
    extra["bf16_path"] = {"matrices_per_s": round(n / tb, 2), "speedup_e4m3_over_bf16": round(value / (n / tb), 3)}
    del wsb, planb
    out = torch.empty(n, dtype=torch.float64, device=dev)
    ows = torch.empty(ifn.orth_error_workspace_bytes(n), dtype=torch.uint8, device=dev)
    hs = np.sqrt([min(s) for s in shapes])
    ifn.orth_error(Ys, out, ows)
    extra["orth_err_over_sqrt_h_mean"] = {"e4m3": float((out.cpu().numpy() / hs).mean())}
    ifn.orth_error(Yb, out, ows)
    extra["orth_err_over_sqrt_h_mean"]["bf16"] = float((out.cpu().numpy() / hs).mean())
    cpu = None
    if not args.no_cpu:
        import oracle
        from oracle import fp8 as F
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        idx = [0, 1]
        log("running the CPU oracle on 2 matrices ...")
        rel8, relb, relm = [], [], []
        dt = 0.0
        for i in idx:
            Mh = Ms[i].float().cpu().numpy().astype(np.float64)
            c0 = time.perf_counter()
            Yo = oracle.ifnso(Mh, exps, coeffs)
            dt += time.perf_counter() - c0
            y8 = Ys[i].float().cpu().numpy().astype(np.float64)
            yb = Yb[i].float().cpu().numpy().astype(np.float64)
            rel8.append(float(np.linalg.norm(y8 - Yo) / np.linalg.norm(Yo)))
            relb.append(float(np.linalg.norm(yb - Yo) / np.linalg.norm(Yo)))
            Ym = F.ifnso_e4m3(Mh, exps, coeffs)
            relm.append(float(np.linalg.norm(y8 - Ym) / np.linalg.norm(Ym)))
        extra["rel_err_vs_fp64_oracle"] = {"e4m3": rel8, "bf16": relb, "e4m3_vs_e4m3_model": relm}
        cpu = {"value": len(idx) / dt, "unit": "matrices/s", "cores": int(threads), "kind": "oracle",
               "cpu_model": _cpu_model(),
               "sample": f"{len(idx)} matrices of the batch (2048x8192), float64 numpy, {dt:.1f} s"}
    line = {
        "metric": "matrices/s on the e4m3 workload; ||Y - Y_fp64|| vs FP64 oracle",
        "value": round(value, 3), "unit": "matrices/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp8_e4m3+bf16", "data": "synthetic",
        "config": {"workload": f"{n} x 2048x8192, U diag(i^-1.5) V^T Haar (seed 3), bf16 storage",
                   "matrices": n, "exponents": list(exps), "coeffs": "gform_v1", "compute": "fp8_e4m3",
                   "parallelism": "single GPU, one grouped launch per stage"},
        "roofline": {"bound": "mfma", "kernel": dom, "achieved": round(achieved, 2), "peak": peak[dom],
                     "unit": "TFLOP/s", "frac": round(achieved / peak[dom], 4), "traffic": None,
                     "avg_launch_ms": round(dur_ms, 3)},
        "cpu_baseline": cpu,
    }
    if n == 64:
        _attach_traffic(line, dom, "traffic_e4m3_batch64_2048x8192.json", E4M3_PROFILE_KERNEL)
    line.update(extra)
    print(json.dumps(line), flush=True)


def run_learned(args, torch, dev, hip, log):
    """Trains the coefficient network on seeded spectra (h in [64, 1024], the three-family
    mixture), then orthogonalises the gradient set with the learned plan and with the fixed
    coefficients (the fallback), and reports ||Y Y^T - I||_F / sqrt(h) per shape class."""
    import numpy as np

    import paper_2602_02500_amd as ifn
    from paper_2602_02500_amd import learn
    from workloads import configs, gen, spectra
    exps, coeffs = configs.load_coeffs("gform_v1")
    t0 = time.perf_counter()
    samples = spectra.spectral_mixture(args.train_samples, seed=5)
    sig, nsig = spectra.pad_spectra(samples)
    sig_d, nsig_d = torch.from_numpy(sig).to(dev), torch.from_numpy(nsig).to(dev)
    log(f"generated {len(samples)} training spectra in {time.perf_counter() - t0:.1f} s")
    params = torch.from_numpy(gen.fan_in_uniform_np(0, learn.PARAM_LAYOUT).astype(np.float32)).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = []
    learn.train(sig_d, nsig_d, params, epochs=args.epochs, batch=256, lr=2e-3, losses=losses)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    steps = len(losses)
    first = float(torch.stack(losses[:50]).mean())
    last = float(torch.stack(losses[-50:]).mean())
    theta = params.cpu().numpy()
    log(f"trained {steps} steps in {train_s:.2f} s: loss {first:.4f} -> {last:.4f}")
    held_out, cpu = None, None
    if not args.no_cpu:
        log("running the CPU oracle on the held-out spectra ...")
        cpu, held_out = cpu_baseline_learned(theta, coeffs, spectra.spectral_mixture(1000, seed=6))
    Ms = make_d3(torch, dev, args.layers)
    shapes = [tuple(m.shape) for m in Ms]
    n = len(Ms)
    res = {}
    for mode in ["learned", "fixed"]:
        plan = ifn.Plan(exps, coeffs, shapes, compute="bf16", mlp_params=theta if mode == "learned" else None)
        ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
        Ys = [torch.empty_like(m) for m in Ms]
        for _ in range(args.warmup):
            plan.orthogonalize_batched(Ms, Ys, ws)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            plan.orthogonalize_batched(Ms, Ys, ws)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / args.steps
        out = torch.empty(n, dtype=torch.float64, device=dev)
        ows = torch.empty(ifn.orth_error_workspace_bytes(n), dtype=torch.uint8, device=dev)
        ifn.orth_error(Ys, out, ows)
        oe = out.cpu().numpy() / np.sqrt([min(s) for s in shapes])
        per = {}
        for nm, r, c in configs.LAYER_SHAPES:
            idx = [i for i, s in enumerate(shapes) if s == (r, c)]
            per[f"{r}x{c}"] = round(float(oe[idx].mean()), 5)
        entry = {"matrices_per_s": round(n / dt, 2), "ms_per_step": round(dt * 1e3, 3),
                 "orth_err_over_sqrt_h_mean": round(float(oe.mean()), 5), "per_shape": per}
        if mode == "learned":
            st = plan.stats()
            entry["network_used_fraction"] = float(np.mean([row[25] for row in st]))
            # per-launch times with HIP events on the call's stream, for the roofline
            tp = time_plan(torch, hip, plan, Ms, Ys, ws, slot_names(plan), 3, 1, log)
            dom, roof = roofline_of(tp["kern"])
        res[mode] = entry
        del ws, Ys, plan
    value = res["learned"]["matrices_per_s"]
    line = {
        "metric": "learned coefficients on the 32-layer gradient set: ||YY^T - I||_F / sqrt(h) vs fixed fallback",
        "value": value, "unit": "matrices/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["learned"]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"train on {len(samples)} seeded spectra (h 64..1024, w/h 1..4, log-uniform / "
                               f"power-law / near-1 mixture), run on the d3 gradient set ({n} matrices)",
                   "exponents": list(exps), "fallback_coeffs": "gform_v1"},
        "training": {"samples": len(samples), "epochs": args.epochs, "batch": 256, "steps": steps,
                     "seconds": round(train_s, 3), "loss_first50": first, "loss_last50": last},
        "held_out_polar_dist2_over_h": held_out,
        "gradset": res,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if args.layers == 32:  # the same matrices and squaring kernel as the gradient-set summary
        _attach_traffic(line, dom, "traffic_gradset_224_bf16.json")
    print(json.dumps(line), flush=True)


def run_tform(args, torch, dev, hip, log):
    """The paper's own form on the gradient set: complement basis T = I - XX^T with
    X = A / ||AA^T||_F^(1/2), depth L = 14 (exponents 0, 1, 2, ..., 2^13: 13 squarings of the
    shifted power D = T - I), coefficients "paper_L14", bfloat16 compute with split (hi + lo)
    operands; `--unsplit` uses single bfloat16 operands instead. Reports throughput, the
    orthogonality error on all matrices beside the Gram-basis form's and beside the same form
    through the float32 path (speed and error; `--no-f32` skips it), and the parity of layer
    0's two 1024x4096 matrices against the float64 oracle."""
    import numpy as np

    import paper_2602_02500_amd as ifn
    from workloads import configs
    exps, coeffs = configs.load_coeffs("paper_L14")
    Ms = make_d3(torch, dev, args.layers)
    shapes = [tuple(m.shape) for m in Ms]
    n = len(Ms)
    Ys = [torch.empty_like(m) for m in Ms]
    split = not args.unsplit
    plan = ifn.Plan(exps, coeffs, shapes, basis="complement", norm="gram_frobenius", compute="bf16",
                    flags=ifn.FLAG_SPLIT_BF16 if split else 0)
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    log(f"workspace {plan.workspace_bytes / 2**30:.1f} GiB")
    nl = plan.num_launches
    J = nl - 6
    names = ["prep"] + ["gram_wide", "gram_tall"] + ["square"] * J + ["aggregate", "product_wide", "product_tall"]
    t = time_plan(torch, hip, plan, Ms, Ys, ws, names, args.steps, args.warmup, log)
    kern, elapsed = t["kern"], t["elapsed"]
    dom = max((k for k in kern if kern[k][2] > 0), key=lambda k: kern[k][0])
    dur_ms = kern[dom][0] / kern[dom][1]
    achieved = kern[dom][2] / kern[dom][1] / (dur_ms * 1e-3) / 1e12
    ms_per_step = elapsed / args.steps * 1e3

    def orth(Yl):
        out = torch.empty(n, dtype=torch.float64, device=dev)
        ows = torch.empty(ifn.orth_error_workspace_bytes(n), dtype=torch.uint8, device=dev)
        ifn.orth_error(Yl, out, ows)
        oe = out.cpu().numpy() / np.sqrt([min(s) for s in shapes])
        per = {}
        for nm, r, c in configs.LAYER_SHAPES:
            idx = [i for i, s in enumerate(shapes) if s == (r, c)]
            per[f"{r}x{c}"] = round(float(oe[idx].mean()), 5)
        return {"mean": float(oe.mean()), "max": float(oe.max()), "per_shape": per}

    err_t = orth(Ys)
    # CPU leg: layer 0's Wk, Wv through the float64 oracle (13 squarings of 1024^2 in numpy)
    cpu, rel, orth_o = None, None, None
    if not args.no_cpu:
        sel = [i for i in range(min(n, 7)) if shapes[i] == (1024, 4096)]
        log("running the CPU oracle on layer 0's 1024x4096 matrices ...")
        cpu, rel, orth_o = cpu_baseline_tform([Ms[i].float().cpu().numpy().astype(np.float64) for i in sel],
                                              [Ys[i].float().cpu().numpy().astype(np.float64) for i in sel],
                                              exps, coeffs)
    del ws, plan
    eg, cg = configs.load_coeffs("gform_v1")
    plan_g = ifn.Plan(eg, cg, shapes, compute="bf16")
    ws = torch.empty(plan_g.workspace_bytes, dtype=torch.uint8, device=dev)
    Yg = [torch.empty_like(m) for m in Ms]
    plan_g.orthogonalize_batched(Ms, Yg, ws)
    torch.cuda.synchronize()
    err_g = orth(Yg)
    del Yg, ws, plan_g
    # the same form through the plain float32 path (generic kernels, float32 operands): speed and
    # orthogonality beside the bf16 path's, where the form does orthogonalise
    f32 = None
    if not args.no_f32:
        M32 = [m.float() for m in Ms]
        Y32 = [torch.empty_like(m) for m in M32]
        plan32 = ifn.Plan(exps, coeffs, shapes, basis="complement", norm="gram_frobenius", compute="f32")
        ws32 = torch.empty(plan32.workspace_bytes, dtype=torch.uint8, device=dev)
        f32_steps = 2
        t32 = time_plan(torch, hip, plan32, M32, Y32, ws32, None, f32_steps, 1, log, slots=False)["elapsed"]
        t32 /= f32_steps
        err32 = orth(Y32)
        f32 = {"matrices_per_s": round(n / t32, 3), "speedup_bf16_over_f32": round(ms_per_step ** -1 * 1e3 * t32, 3),
               "timed_steps": f32_steps, "warmup": 1, "orth_err_over_sqrt_h": err32,
               "orth_err_mean_bf16_over_f32": round(err_t["mean"] / err32["mean"], 4)}
        del M32, Y32, ws32, plan32
    line = {
        "metric": "paper form (complement basis, L = 14) on the 32-layer gradient set: matrices/s and "
                  "||YY^T - I||_F / sqrt(h)",
        "value": round(n * args.steps / elapsed, 3), "unit": "matrices/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"d3 gradient set, {args.layers} layers x 7 matrices; complement basis, "
                               "Gram-Frobenius scaling, exponents 0..2^13", "matrices": n,
                   "coeffs": "paper_L14", "compute": "bf16", "operands": "split bf16 pairs" if split else "bf16"},
        "roofline": {"bound": "mfma", "kernel": dom, "achieved": round(achieved, 2), "peak": PEAK_BF16_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_BF16_TFLOPS, 4), "traffic": None,
                     "avg_launch_ms": round(dur_ms, 3)},
        "cpu_baseline": cpu,
        "kernels": {k: {"ms_per_step": round(v[0], 3), "launches": v[1],
                        "tflops": round(v[2] / (v[0] * 1e-3) / 1e12, 1) if v[0] > 0 and v[2] > 0 else None}
                    for k, v in kern.items()},
        "orth_err_over_sqrt_h": err_t,
        "gram_basis_gform_v1_orth_err_over_sqrt_h": err_g,
        "parity_layer0_1024x4096_rel_vs_oracle": rel,
        "oracle_orth_err_over_sqrt_h_layer0_1024x4096": orth_o,
        "f32_path": f32,
    }
    if args.layers == 32 and split:
        _attach_traffic(line, dom, "traffic_tform_gradset_224_bf16.json", TFORM_PROFILE_KERNEL)
    print(json.dumps(line), flush=True)


def run_muon(args, torch, dev, hip, log):
    """One Muon optimizer step per timed step on the gradient set: float32 weights and momentum,
    the bf16 gradients as G, Nesterov momentum 0.95, lr 0.02, weight decay 0.01, the fixed
    Gram-basis coefficients as the orthogonalisation (with --learned: the coefficient network,
    trained first, picks each matrix's coefficients inside every step). Reports matrices/s of
    whole steps and the time of the orthogonalisation alone on the same inputs."""
    import numpy as np

    import paper_2602_02500_amd as ifn
    from workloads import configs, gen
    exps, coeffs = configs.load_coeffs("gform_v1")
    theta, training = None, None
    if args.learned:  # the coefficient network in the loop: trained first, as the learned workload does
        from paper_2602_02500_amd import learn
        from workloads import spectra
        samples = spectra.spectral_mixture(args.train_samples, seed=5)
        sig, nsig = spectra.pad_spectra(samples)
        params = torch.from_numpy(gen.fan_in_uniform_np(0, learn.PARAM_LAYOUT).astype(np.float32)).to(dev)
        t0 = time.perf_counter()
        learn.train(torch.from_numpy(sig).to(dev), torch.from_numpy(nsig).to(dev), params, epochs=args.epochs,
                    batch=256, lr=2e-3)
        torch.cuda.synchronize()
        training = {"samples": len(samples), "epochs": args.epochs, "seconds": round(time.perf_counter() - t0, 3)}
        theta = params.cpu().numpy()
        log(f"trained the coefficient network in {training['seconds']} s")
    Gs = make_d3(torch, dev, args.layers)
    shapes = [tuple(g.shape) for g in Gs]
    n = len(Gs)
    Ws = [gen.gaussian_torch(r, c, 5000 + i, 0, 0.02, device=dev).float() for i, (r, c) in enumerate(shapes)]
    Bs = [torch.zeros(s, dtype=torch.float32, device=dev) for s in shapes]
    plan = ifn.Plan(exps, coeffs, shapes, compute="bf16", mlp_params=theta)
    ws = torch.empty(plan.muon_workspace_bytes, dtype=torch.uint8, device=dev)
    log(f"muon workspace {plan.muon_workspace_bytes / 2**30:.1f} GiB")
    hp = dict(lr=0.02, momentum=0.95, weight_decay=0.01, nesterov=True)
    for _ in range(args.warmup):
        plan.muon_step(Ws, Gs, Bs, ws, **hp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.muon_step(Ws, Gs, Bs, ws, **hp)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    Ys = [torch.empty_like(g) for g in Gs]
    for _ in range(args.warmup):
        plan.orthogonalize_batched(Gs, Ys, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.orthogonalize_batched(Gs, Ys, ws)
    torch.cuda.synchronize()
    dto = (time.perf_counter() - t0) / args.steps
    elems = sum(r * c for r, c in shapes)
    # elementwise bytes: momentum pass reads B, G and writes B, U; update pass reads W, Y, writes W
    ew_bytes = elems * (4 + 2 + 4 + 2 + 4 + 2 + 4)
    finite = all(bool(torch.isfinite(w).all()) for w in Ws)
    network = None
    if args.learned:
        st = plan.stats()
        network = {"used_fraction": float(np.mean([row[25] for row in st])), "training": training,
                   "coeffs_mean": [round(float(v), 4) for v in np.mean([row[9:15] for row in st], axis=0)]}
    line = {
        "metric": "Muon optimizer steps on the 32-layer gradient set (momentum, IFNSO, weight update)",
        "value": round(n / dt, 3), "unit": "matrices/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"d3 gradient set, {args.layers} layers x 7 matrices as gradients; float32 weights "
                               "N(0, 0.02^2) and momentum", "matrices": n,
                   "coeffs": "learned (fixed fallback gform_v1)" if args.learned else "gform_v1",
                   "optimizer": hp},
        "coefficient_network": network,
        "roofline": None, "cpu_baseline": None,
        "orthogonalize_ms": round(dto * 1e3, 3),
        "elementwise_ms": round((dt - dto) * 1e3, 3),
        "elementwise_bytes": ew_bytes,
        "elementwise_gbps": round(ew_bytes / max(dt - dto, 1e-9) / 1e9, 1),
        "weights_finite": finite,
    }
    print(json.dumps(line), flush=True)


def run_ns(args, torch, dev, hip, log):
    """Newton-Schulz iterations on the gradient set through the batched 256-tile path, beside
    IFNSO: Muon's quintic (5 steps), the Cesista-form quintics (5 steps), the cubic (8 steps)
    and the CANS quintics (5 steps, Gelfand q = 1), each step one Gram-basis plan with
    exponents {0, 1, 2} (bf16 iterates between steps); then the fixed-coefficient IFNSO plan.
    Reports matrices/s and ||YY^T - I||_F / sqrt(h) per method."""
    import numpy as np

    import paper_2602_02500_amd as ifn
    from workloads import configs
    Ms = make_d3(torch, dev, args.layers)
    shapes = [tuple(m.shape) for m in Ms]
    n = len(Ms)
    Ys = [torch.empty_like(m) for m in Ms]
    out = torch.empty(n, dtype=torch.float64, device=dev)
    ows = torch.empty(ifn.orth_error_workspace_bytes(n), dtype=torch.uint8, device=dev)
    hs = np.sqrt([min(s) for s in shapes])
    res = {}

    def measure(call):
        for _ in range(args.warmup):
            call()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            call()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        ifn.orth_error(Ys, out, ows)
        oe = out.cpu().numpy() / hs
        per = {}
        for _, r, c in configs.LAYER_SHAPES:
            idx = [i for i, s in enumerate(shapes) if s == (r, c)]
            per[f"{r}x{c}"] = round(float(oe[idx].mean()), 5)
        return {"matrices_per_s": round(n / dt, 2), "ms_per_step": round(dt * 1e3, 3),
                "orth_err_over_sqrt_h_mean": round(float(oe.mean()), 5), "per_shape": per}

    for name, q in (("muon_ns5", 0), ("cesista_ns5", 0), ("original_ns8", 0), ("cans_ns5_q2", 1)):
        sched, _ = configs.load_schedule(name)
        sp = ifn.SchedulePlan(sched, shapes, gelfand_q=q, compute="bf16")
        ws = torch.empty(sp.workspace_bytes, dtype=torch.uint8, device=dev)
        res[name] = measure(lambda: sp.orthogonalize_batched(Ms, Ys, ws))
        res[name]["steps"] = len(sched)
        res[name]["gelfand_q"] = q
        log(f"{name}: {res[name]['matrices_per_s']} matrices/s")
        del ws, sp
    exps, coeffs = configs.load_coeffs("gform_v1")
    plan = ifn.Plan(exps, coeffs, shapes, compute="bf16")
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    res["ifnso_gform_v1"] = measure(lambda: plan.orthogonalize_batched(Ms, Ys, ws))
    del ws, plan
    value = res["muon_ns5"]["matrices_per_s"]
    line = {
        "metric": "Newton-Schulz baselines on the 32-layer gradient set, batched 256-tile path: matrices/s and "
                  "||YY^T - I||_F / sqrt(h), beside IFNSO",
        "value": value, "unit": "matrices/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["muon_ns5"]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"d3 gradient set, {args.layers} layers x 7 matrices; value: Muon's quintic, "
                               "5 steps", "matrices": n},
        "roofline": None, "cpu_baseline": None,
        "methods": res,
        "ifnso_speedup_over_muon_ns5": round(res["ifnso_gform_v1"]["matrices_per_s"] / value, 3),
    }
    print(json.dumps(line), flush=True)


TABLE1_SHAPES = ((128, 128), (128, 512), (128, 1024))


def _call_ms(torch, call, reps, warmup=3):
    """Median time per call (ms) from CUDA events around each call, after `warmup` calls."""
    import numpy as np
    for _ in range(warmup):
        call()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        call()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts)), float(np.percentile(ts, 10)), float(np.percentile(ts, 90))


def run_d1(args, torch, dev, hip, log):
    """The small parity configuration: one 256x512 float32 N(0,1) matrix (seed 0); Muon's five
    Newton-Schulz steps and the Gram-basis polynomial with exponents {0,1,2,4,8} and the seeded
    coefficients, each in float32 and bf16, one call at a time (latency-bound: a handful of
    one-tile launches). Reports the median time per call and the distance to the float64
    oracle; `value` is IFNSO's bf16 calls per second."""
    import numpy as np

    import oracle
    import paper_2602_02500_amd as ifn
    from workloads import configs, gen
    rows, cols = 256, 512
    M64 = gen.gaussian_np(rows, cols, seed=0)
    exps, c = configs.D1_EXPONENTS, configs.d1_coeffs()
    res = {}
    for compute in ("f32", "bf16"):
        vals = M64.astype(np.float32).astype(np.float64) if compute == "f32" else gen.round_to_bf16_np(M64)
        dt = torch.float32 if compute == "f32" else torch.bfloat16
        Mt = torch.from_numpy(vals.astype(np.float32)).to(dev).to(dt)
        Y = torch.empty_like(Mt)
        plan = ifn.Plan(exps, c, [(rows, cols)], compute=compute)
        ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
        med, p10, p90 = _call_ms(torch, lambda: plan.orthogonalize(Mt, Y, ws), args.steps * 10)
        rel = float(np.linalg.norm(Y.double().cpu().numpy() - oracle.ifnso(vals, exps, c)) /
                    np.linalg.norm(oracle.ifnso(vals, exps, c)))
        res[f"ifnso_{compute}"] = {"ms_per_call": round(med, 4), "p10": round(p10, 4), "p90": round(p90, 4),
                                   "rel_vs_oracle": rel}
        wns = torch.empty(ifn.classical_ns_workspace_bytes(rows, cols, compute), dtype=torch.uint8, device=dev)
        Yn = torch.empty_like(Mt)
        med, p10, p90 = _call_ms(torch, lambda: ifn.classical_ns(Mt, Yn, 5, configs.MUON_ABC, compute, wns),
                                 args.steps * 10)
        Yo = oracle.classical_ns(vals, 5, configs.MUON_ABC)
        rel = float(np.linalg.norm(Yn.double().cpu().numpy() - Yo) / np.linalg.norm(Yo))
        res[f"ns5_{compute}"] = {"ms_per_call": round(med, 4), "p10": round(p10, 4), "p90": round(p90, 4),
                                 "rel_vs_oracle": rel}
    cpu = None
    if not args.no_cpu:
        t0 = time.perf_counter()
        reps = 20
        for _ in range(reps):
            oracle.ifnso(M64, exps, c)
        dt = time.perf_counter() - t0
        cpu = {"value": reps / dt, "unit": "matrices/s", "cores": _oracle_threads(), "kind": "oracle",
               "cpu_model": _cpu_model(), "sample": f"{reps} calls of the IFNSO oracle on the 256x512 matrix, "
                                                   f"float64 numpy, {dt:.2f} s"}
    line = {
        "metric": "256x512 single-matrix latency: IFNSO vs Muon's 5-step Newton-Schulz, float32 and bf16",
        "value": round(1e3 / res["ifnso_bf16"]["ms_per_call"], 2), "unit": "matrices/s", "n_gpus": 1,
        "steps": args.steps * 10, "warmup": 3, "ms_per_step": res["ifnso_bf16"]["ms_per_call"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "256x512 N(0,1) seed 0; IFNSO exponents {0,1,2,4,8} with the seeded coefficients; "
                               "NS: 5 steps (3.4445, -4.7750, 2.0315)", "matrices": 1},
        "roofline": None, "cpu_baseline": cpu, "calls": res,
    }
    print(json.dumps(line), flush=True)


def run_d2(args, torch, dev, hip, log):
    """The FP32-versus-BF16 pair: 4096x4096 (seed 1) and 14336x4096 (seed 2), U diag(sigma) V^T
    with Haar factors and sigma log-uniform on [1e-3, 1], exponents {0..16} with the fixed
    coefficients, through one batched plan per path. Reports matrices/s of each path, the
    speed-up, and each path's distance to the exact result U diag(f(sigma~)) V^T."""
    import numpy as np

    import oracle
    import paper_2602_02500_amd as ifn
    from workloads import configs, gen
    exps, c = configs.load_coeffs("gform_v1")
    cases = [(4096, 4096, 1), (14336, 4096, 2)]
    mats, closed = [], []
    for rows, cols, seed in cases:
        sigma = configs.d2_sigma_np(min(rows, cols), seed)
        M, U, V = gen.spectral_torch(rows, cols, sigma, seed, device=dev)
        closed.append(oracle.closed_form(U.cpu().numpy(), sigma, V.cpu().numpy(), exps, c))
        mats.append(M)
        del U, V
    shapes = [tuple(m.shape) for m in mats]
    res = {}
    for compute, dt in (("f32", torch.float32), ("bf16", torch.bfloat16)):
        Ms = [m.to(dt).contiguous() for m in mats]
        Ys = [torch.empty_like(m) for m in Ms]
        plan = ifn.Plan(exps, c, shapes, compute=compute)
        ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
        t = time_plan(torch, hip, plan, Ms, Ys, ws, None, args.steps, args.warmup, log, slots=False)
        ms = t["elapsed"] / args.steps * 1e3
        rel = [float(np.linalg.norm(Y.double().cpu().numpy() - Yc) / np.linalg.norm(Yc)) for Y, Yc in zip(Ys, closed)]
        res[compute] = {"matrices_per_s": round(2 / (ms * 1e-3), 2), "ms_per_step": round(ms, 3),
                        "rel_vs_closed_form": rel}
        del Ms, Ys, ws, plan
    line = {
        "metric": "FP32 vs BF16 path on the 4096x4096 and 14336x4096 pair: matrices/s and error vs the exact result",
        "value": res["bf16"]["matrices_per_s"], "unit": "matrices/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["bf16"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "4096x4096 (seed 1) and 14336x4096 (seed 2), Haar factors, sigma log-uniform "
                               "[1e-3, 1]; exponents {0,1,2,4,8,16}, gform_v1", "matrices": 2},
        "roofline": None, "cpu_baseline": None, "paths": res,
        "speedup_bf16_over_f32": round(res["bf16"]["matrices_per_s"] / res["f32"]["matrices_per_s"], 2),
    }
    print(json.dumps(line), flush=True)


def cpu_baseline_table1(methods, inputs):
    """The FP64 oracle of every Table 1 method on the three inputs; its ||YY^T - I||_F."""
    import numpy as np

    import oracle
    from oracle import baselines as BL
    t0 = time.perf_counter()
    errs = {}
    for name, m in methods.items():
        for shape, Mh in inputs.items():
            if m["kind"] == "schedule":
                Yo = BL.ns_schedule(Mh, m["schedule"], m["q"])
            else:
                Yo = oracle.ifnso(Mh, m["exps"], m["coeffs"], m["basis"], m["norm"])
            errs[(name, shape)] = float(oracle.orth_error(Yo))
    dt = time.perf_counter() - t0
    calls = len(methods) * len(inputs)
    cpu = {"value": calls / dt, "unit": "matrices/s", "cores": _oracle_threads(), "kind": "oracle",
           "cpu_model": _cpu_model(),
           "sample": f"all {calls} method x size cases of the table, float64 numpy, {dt:.2f} s"}
    return cpu, errs


def run_table1(args, torch, dev, hip, log):
    """Table 1 of the paper on one MI355X: the orthogonality error ||YY^T - I||_F and the time
    per call of Newton-Schulz with the cubic (8 steps), Muon's quintic (5 steps), Cesista-form
    quintics (5 steps), CANS minimax quintics with Gelfand q = 2 (5 steps), and IFNSO in the
    paper's form (complement basis, depth 14) and in the Gram basis (exponents up to 16), on
    N(0,1) matrices 128x128, 128x512 and 128x1024 (seed 0), float32. FLOPs follow the paper's
    dense count. The paper's own values, measured on other inputs, are printed beside them."""
    import numpy as np

    import paper_2602_02500_amd as ifn
    from workloads import configs, gen
    methods = {}
    for name in ("original_ns8", "muon_ns5", "cesista_ns5", "cans_ns5_q2"):
        sched, q = configs.load_schedule(name)
        methods[name] = {"kind": "schedule", "schedule": sched, "q": q}
    e, c = configs.load_coeffs("paper_L14")
    methods["ifnso_paper_L14"] = {"kind": "plan", "exps": e, "coeffs": c, "basis": "complement",
                                  "norm": "gram_frobenius"}
    e, c = configs.load_coeffs("gform_v1")
    methods["ifnso_gform_v1"] = {"kind": "plan", "exps": e, "coeffs": c, "basis": "gram", "norm": "frobenius"}
    paper_name = {"original_ns8": "original_ns", "muon_ns5": "muon_ns", "cesista_ns5": "cesista_ns",
                  "cans_ns5_q2": "cans", "ifnso_paper_L14": "ifnso"}
    with open(os.path.join(ROOT, "tests", "golden", "table1.json")) as f:
        printed = {(r["method"], r["h"], r["w"]): r for r in json.load(f)["rows"]}
    inputs = {s: gen.gaussian_np(*s, seed=0).astype(np.float32).astype(np.float64) for s in TABLE1_SHAPES}
    reps = max(args.steps, 20)
    rows, times = [], {}
    for shape, Mh in inputs.items():
        h, w = shape
        Mt = torch.from_numpy(Mh.astype(np.float32)).to(dev)
        Y = torch.empty_like(Mt)
        out = torch.empty(1, dtype=torch.float64, device=dev)
        ows = torch.empty(ifn.orth_error_workspace_bytes(1), dtype=torch.uint8, device=dev)
        for name, m in methods.items():
            if m["kind"] == "schedule":
                ws = torch.empty(ifn.classical_ns_workspace_bytes(h, w, "f32"), dtype=torch.uint8, device=dev)
                call = lambda: ifn.ns_schedule(Mt, Y, m["schedule"], m["q"], "f32", ws)  # noqa: E731
                steps = len(m["schedule"])
                longp = 2 if name == "original_ns8" else 3
                flops = steps * longp * 2.0 * h * h * w
            else:
                plan = ifn.Plan(m["exps"], m["coeffs"], [shape], basis=m["basis"], norm=m["norm"], compute="f32")
                ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
                call = lambda: plan.orthogonalize(Mt, Y, ws)  # noqa: E731
                sq = len(m["exps"]) - 2
                flops = 4.0 * h * h * w + 2.0 * sq * h ** 3
            for _ in range(args.warmup):
                call()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                call()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            ifn.orth_error([Y], out, ows)
            err = float(out.item())
            pr = printed.get((paper_name.get(name, ""), h, w))
            rows.append({"method": name, "h": h, "w": w, "error": round(err, 4), "ms": round(dt * 1e3, 4),
                         "flops_dense": flops, "paper_error": pr["error"] if pr else None,
                         "paper_flops": pr["flops"] if pr else None})
            times[(name, shape)] = dt
            del ws
    cpu = None
    if not args.no_cpu:
        log("running the CPU oracle on every case ...")
        cpu, errs = cpu_baseline_table1(methods, inputs)
        for r in rows:
            r["oracle_error"] = round(errs[(r["method"], (r["h"], r["w"]))], 4)
    value = 1.0 / times[("ifnso_paper_L14", (128, 1024))]
    line = {
        "metric": "Table 1 on MI355X: ||YY^T - I||_F and time per call of five orthogonalisation methods",
        "value": round(value, 3), "unit": "matrices/s", "n_gpus": 1, "steps": reps, "warmup": args.warmup,
        "ms_per_step": round(1e3 / value, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "N(0,1) 128x128, 128x512, 128x1024 (seed 0), float32; value: IFNSO paper form on "
                               "128x1024, one call at a time", "methods": list(methods)},
        "roofline": None, "cpu_baseline": cpu,
        "table": rows,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--layers", type=int, default=32)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-check", action="store_true", help="skip the float64 orthogonality check")
    ap.add_argument("--no-f32", action="store_true", help="skip the plain float32 comparison")
    ap.add_argument("--workload", choices=["gradset", "e4m3", "learned", "tform", "muon", "table1", "ns", "d1", "d2"],
                    default="gradset",
                    help="gradset: the 32-layer gradient set in bf16 (the headline); e4m3: 64 x 2048x8192 "
                         "heavy-tailed matrices with e4m3 Gram and squarings; learned: train the coefficient "
                         "network on the GPU, then run the gradient set with learned and fixed coefficients; "
                         "tform: the paper's complement-basis form (L = 14) on the gradient set; muon: whole "
                         "Muon optimizer steps on the gradient set (--learned: the coefficient network in the "
                         "loop); table1: the paper's Table 1 methods on the device; ns: Newton-Schulz baselines "
                         "on the gradient set; d1: 256x512 single-matrix latency; d2: FP32 vs BF16 on the "
                         "4096x4096 / 14336x4096 pair")
    ap.add_argument("--train-samples", type=int, default=100000, help="learned workload: training spectra")
    ap.add_argument("--epochs", type=int, default=3, help="learned workload: training epochs")
    ap.add_argument("--batch", type=int, default=64, help="e4m3 workload: matrices in the batch")
    ap.add_argument("--unsplit", action="store_true", help="tform workload: single bf16 operands")
    ap.add_argument("--learned", action="store_true", help="muon workload: the coefficient network in the loop")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="first run a plain elementwise copy (out = x + 0, float32) that reads and writes BYTES, "
                         "as a known-size reference for hardware byte counters")
    ap.add_argument("--tune", action="store_true",
                    help="time candidate tile schedules per stage first and keep the fastest (written to --tune-out)")
    ap.add_argument("--tune-out", default=os.path.join(ROOT, "tuned_schedules.json"))
    ap.add_argument("--schedules", default=os.path.join(ROOT, "paper_2602_02500_amd", "schedules.json"),
                    help="tuned schedules to apply when the plan's key is present")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the 224 matrices are independent and would be sharded by matrix across GPUs)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2602_02500_amd as ifn
    from workloads import configs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    hip = _hip()
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    if args.copy_calibration > 0:
        x = torch.ones(args.copy_calibration // 4, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        torch.add(x, 0, out=y)
        torch.cuda.synchronize()
        del x, y
    if args.workload == "e4m3":
        return run_e4m3(args, torch, dev, hip, log)
    if args.workload == "learned":
        return run_learned(args, torch, dev, hip, log)
    if args.workload == "tform":
        return run_tform(args, torch, dev, hip, log)
    if args.workload == "muon":
        return run_muon(args, torch, dev, hip, log)
    if args.workload == "table1":
        return run_table1(args, torch, dev, hip, log)
    if args.workload == "ns":
        return run_ns(args, torch, dev, hip, log)
    if args.workload == "d1":
        return run_d1(args, torch, dev, hip, log)
    if args.workload == "d2":
        return run_d2(args, torch, dev, hip, log)

    exps, coeffs = configs.load_coeffs("gform_v1")
    t0 = time.perf_counter()
    Ms = make_d3(torch, dev, args.layers)
    shapes = [tuple(m.shape) for m in Ms]
    n = len(Ms)
    log(f"generated {n} matrices in {time.perf_counter() - t0:.1f} s")
    Ys = [torch.empty_like(m) for m in Ms]
    plan = ifn.Plan(exps, coeffs, shapes, compute="bf16")
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    log(f"workspace {plan.workspace_bytes / 2**30:.1f} GiB")
    sched = schedule(args, torch, plan, Ms, Ys, ws, "bf16", exps, log)
    nl = plan.num_launches
    J = nl - 6
    fl = stage_flops(shapes, J)
    # kernel of each launch slot (squaring levels share one kernel; the last one forms P, the
    # aggregation folded into its epilogue, and leaves the aggregate slot empty)
    names = ["prep"] + ["gram_wide", "gram_tall"] + ["square"] * (J - 1) + ["square_last"] + \
        ["aggregate", "product_wide", "product_tall"]

    t = time_plan(torch, hip, plan, Ms, Ys, ws, names, args.steps, args.warmup, log)
    kern, elapsed = t["kern"], t["elapsed"]
    dom = max((k for k in kern if kern[k][2] > 0), key=lambda k: kern[k][0])
    dur_ms = kern[dom][0] / kern[dom][1]
    flop_per_launch = kern[dom][2] / kern[dom][1]
    achieved = flop_per_launch / (dur_ms * 1e-3) / 1e12
    ms_per_step = elapsed / args.steps * 1e3
    value = n * args.steps / elapsed
    step_tflops = fl["step"] / (ms_per_step * 1e-3) / 1e12

    extra = {"event_ms_per_step": round(t["event_ms"] / args.steps, 3),
             "slot_pass_ms_per_step": round(t["slot_pass_ms"], 3), "schedules": sched,
             "kernels": {k: {"ms_per_step": round(v[0], 3), "launches": v[1],
                             "tflops": round(v[2] / (v[0] * 1e-3) / 1e12, 1) if v[0] > 0 and v[2] > 0 else None}
                         for k, v in kern.items()},
             "algorithmic_tflop_per_step": round(fl["step"] / 1e12, 2),
             "mfma_util": round(step_tflops / PEAK_BF16_TFLOPS, 4)}

    # orthogonality (float64 on the device), not timed
    if not args.no_check:
        out = torch.empty(n, dtype=torch.float64, device=dev)
        ows = torch.empty(ifn.orth_error_workspace_bytes(n), dtype=torch.uint8, device=dev)
        ifn.orth_error(Ys, out, ows)
        oe = out.cpu().numpy() / np.sqrt([min(s) for s in shapes])
        extra["orth_err_over_sqrt_h"] = {"mean": float(oe.mean()), "max": float(oe.max())}

    # plain float32 path on the same matrices (two steps), for the speed-up and error targets
    if not args.no_f32:
        M32 = [m.float() for m in Ms]
        Y32 = [torch.empty_like(m) for m in M32]
        del ws
        plan32 = ifn.Plan(exps, coeffs, shapes, compute="f32")
        ws32 = torch.empty(plan32.workspace_bytes, dtype=torch.uint8, device=dev)
        f32_steps = 5
        t32 = time_plan(torch, hip, plan32, M32, Y32, ws32, None, f32_steps, 2, log, slots=False)["elapsed"]
        t32 /= f32_steps
        extra["f32_path"] = {"matrices_per_s": n / t32, "speedup_bf16_over_f32": value / (n / t32),
                             "timed_steps": f32_steps, "warmup": 2}
        if not args.no_check:
            out = torch.empty(n, dtype=torch.float64, device=dev)
            ows = torch.empty(ifn.orth_error_workspace_bytes(n), dtype=torch.uint8, device=dev)
            ifn.orth_error(Y32, out, ows)
            oe32 = out.cpu().numpy() / np.sqrt([min(s) for s in shapes])
            extra["f32_path"]["orth_err_over_sqrt_h_mean"] = float(oe32.mean())
            rel = []
            for a, b in zip(Ys, Y32):
                rel.append(float(torch.linalg.norm(a.float() - b) / torch.linalg.norm(b)))
            extra["f32_path"]["bf16_vs_f32_rel_max"] = max(rel)
        del M32, Y32, ws32, plan32

    cpu = None
    if not args.no_cpu:
        idx = list(range(7))
        Mh = [Ms[i].float().cpu().numpy().astype(np.float64) for i in idx]
        Yd = [Ys[i].float().cpu().numpy().astype(np.float64) for i in idx]
        log("running the CPU oracle on layer 0 ...")
        cpu, rel, orth = cpu_baseline(Mh, exps, coeffs, Yd)
        extra["parity_layer0_rel_max"] = max(rel)
        extra["oracle_orth_err_over_sqrt_h_layer0_mean"] = float(np.mean(orth))

    line = {
        "metric": "matrices/s + MFMA util on 32-layer grad set; ||XX^T-I|| vs FP64 oracle",
        "value": round(value, 3), "unit": "matrices/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"d3 gradient set, {args.layers} layers x 7 matrices, hidden 4096 GQA SwiGLU, "
                               "bf16 N(0,0.02^2) + rank-16 (norm 0.5)",
                   "matrices": n, "exponents": list(exps), "coeffs": "gform_v1", "compute": "bf16",
                   "parallelism": "single GPU, one grouped launch per stage"},
        "roofline": {"bound": "mfma", "kernel": dom, "achieved": round(achieved, 2), "peak": PEAK_BF16_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_BF16_TFLOPS, 4), "traffic": None,
                     "avg_launch_ms": round(dur_ms, 3)},
        "cpu_baseline": cpu,
    }
    if args.layers == 32:
        _attach_traffic(line, dom, "traffic_gradset_224_bf16.json")
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
