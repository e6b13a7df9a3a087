#!/usr/bin/env python3
"""Throughput of the VGGT-L-shaped aggregator forward on one MI355X.

Workload (default): 24 frame/global attention pairs, C=1024, 16 heads x 64,
MLP 4096, S=1000 frames x P=1374 tokens (1,374,000 global tokens), bfloat16
operands with float32 accumulation, float32 softmax statistics and residual
stream, outputs of layers 4/11/17/23 kept.  One step is one whole aggregator
forward over that batch; inputs (tokens N(0,1), weights N(0,0.02)) are
synthetic, drawn on the device with a seeded generator and resident in HBM
before timing starts.

A wall-clock budget (--wall-budget, from process start) bounds the run: at
S=1000 one step takes minutes, so the timed steps beyond the first and the
warm-up steps are cut to what fits (one-frame calls load the kernels first;
the counts actually run are reported beside the requested ones; room is kept
for the FP8 legs).  After the bfloat16 headline, and while the budget allows:
one forward with FP8 P V global attention (bfloat16 scores, E4M3
probabilities and values), one with all-E4M3 global attention, the float32
global-attention rate on one head at the same S, and the accuracy of each
precision's global attention against the float32 kernel in three logit
regimes.

Prints one JSON line: frames/s, global attention TFLOP/s (from the library's
per-launch HIP events), peak HBM, the roofline of the dominant kernel and the
FP64 oracle's throughput on the host CPU (extrapolated from a bounded
sample).
"""
import time

T_START = time.perf_counter()  # wall-budget origin: before the heavy imports

import argparse  # noqa: E402
import hashlib  # noqa: E402
import json  # noqa: E402
import math  # noqa: E402
import os  # noqa: E402
import sys  # noqa: E402
import threading  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

import synth  # noqa: E402
from paper_2509_25191_amd import vggtx as vg  # noqa: E402

# MI355X dense MFMA peaks; "fp8pv" (bfloat16 Q K^T, E4M3 P V: half the flops
# at each rate) is the harmonic mean of the two
PEAK_TFLOPS = {"fp8": 5000.0, "bf16": 2500.0, "f32": 157.3, "fp8pv": 2.0 / (1.0 / 2500.0 + 1.0 / 5000.0)}
PREC = {"fp8": vg.FP8_E4M3, "bf16": vg.BF16, "f32": vg.F32}
P_TOKENS = 1374
OUT_LAYERS = (4, 11, 17, 23)


def measured_traffic(prec, S):
    """HBM bytes per launch of the global-attention kernel at S=1000, from the
    committed rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE, each scaled
    by the same counter's reading for a plain copy of known size).  None when
    no summary exists for this workload or when it was taken on a different
    attention source than the one built now."""
    if S != 1000:
        return None
    path = os.path.join(ROOT, "profiles", f"attn_{prec}_kernel_vggt_l_s1000_traffic.txt")
    src = os.path.join(ROOT, "paper_2509_25191_amd", "csrc", "attention.hip")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.lstrip().startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    with open(src, "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    if kv.get("attention_hip_sha256") != digest or "hbm_bytes_per_launch" not in kv:
        return None
    return float(kv["hbm_bytes_per_launch"])


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_weights(model, gen, dtype, dev):
    layers = []
    C, F = model.dim, model.mlp_hidden
    shapes = {"ln1_g": (C,), "ln1_b": (C,), "w_qkv": (3 * C, C), "b_qkv": (3 * C,), "w_o": (C, C), "b_o": (C,),
              "ln2_g": (C,), "ln2_b": (C,), "w_fc1": (F, C), "b_fc1": (F,), "w_fc2": (C, F), "b_fc2": (C,)}
    for _ in range(model.depth):
        l = {}
        for part in ("frame", "global"):
            blk = {}
            for name in synth.BLOCK_FIELDS:
                t = torch.empty(shapes[name], device=dev, dtype=torch.float32).normal_(0.0, 0.02, generator=gen)
                if name.endswith("_g"):
                    t += 1.0
                blk[name] = t.to(dtype)
            l[part] = blk
        layers.append(l)
    return layers


def attn_only_rate(h, S, prec, dev, gen, heads=16):
    """Standalone global attention over one scene of S frames: TFLOP/s from the library's events."""
    N, H, D = S * P_TOKENS, heads, 64
    dt = torch.float32 if prec == vg.F32 else torch.bfloat16
    q = torch.empty((N, H, D), device=dev, dtype=torch.float32).normal_(0, 0.64, generator=gen).to(dt)
    k = torch.empty((N, H, D), device=dev, dtype=torch.float32).normal_(0, 0.64, generator=gen).to(dt)
    v = torch.empty((N, H, D), device=dev, dtype=torch.float32).normal_(0, 1.0, generator=gen).to(dt)
    o = torch.empty_like(q)
    ws = torch.empty(max(256, vg.attn_workspace_size(h, [0, N], H, D, prec)), dtype=torch.uint8, device=dev)
    vg.attn_global(h, q, k, v, o, [0, N], prec, ws=ws)  # untimed first call
    torch.cuda.synchronize()
    vg.timing_enable(h, True)
    vg.attn_global(h, q, k, v, o, [0, N], prec, ws=ws)
    torch.cuda.synchronize()
    t = vg.timing_read(h)["attn_global"]
    vg.timing_enable(h, False)
    del q, k, v, o, ws
    torch.cuda.empty_cache()
    return t["flops"] / (t["ms"] * 1e-3) / 1e12, t["ms"]


def cpu_baseline(S, P, C=1024, H=16, F=4096, depth=24):
    """FP64 oracle throughput on the host, extrapolated to the whole forward
    from timed pieces (about 10 s of CPU work): the frame block on 4 frames;
    the token-local part of a block (LN, QKV, out-projection, MLP) on a
    16384-row slab; global attention of 512 query rows of one head against
    all S*P keys."""
    import threadpoolctl

    import oracle
    rng = np.random.default_rng(0)
    N = S * P
    w = synth.gen_block(rng, C, F)
    w64 = {k: v.astype(np.float64) for k, v in w.items()}
    nf = 4
    x1 = rng.standard_normal((nf * P, C))

    def best(fn, reps=2):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter(); fn(); ts.append(time.perf_counter() - t0)
        return min(ts)

    t_frame = best(lambda: oracle.block(x1, w64, [(f * P, (f + 1) * P) for f in range(nf)], H, 1e-6)) / nf
    rows = 16384
    xs = rng.standard_normal((rows, C))

    def token_local():
        hh = oracle.layer_norm(xs, w64["ln1_g"], w64["ln1_b"], 1e-6)
        oracle.linear(hh, w64["w_qkv"], w64["b_qkv"])
        x1_ = xs + oracle.linear(hh, w64["w_o"], w64["b_o"])
        h2 = oracle.layer_norm(x1_, w64["ln2_g"], w64["ln2_b"], 1e-6)
        oracle.linear(oracle.gelu(oracle.linear(h2, w64["w_fc1"], w64["b_fc1"])), w64["w_fc2"], w64["b_fc2"])

    t_tok = best(token_local)
    qrows = 512
    q = rng.standard_normal((1, qrows, 64))
    k = rng.standard_normal((1, N, 64))
    v = rng.standard_normal((1, N, 64))
    t_att = best(lambda: oracle.attention(q, k, v), reps=1)
    per_layer = S * t_frame + (N / rows) * t_tok + (N * H / qrows) * t_att
    total = depth * per_layer
    info = threadpoolctl.threadpool_info()
    cores = max([i.get("num_threads", 1) for i in info] + [1])
    sample = (f"oracle pieces timed: frame block on {nf} frames of {P} tokens ({nf * t_frame:.2f}s), token-local block "
              f"ops on {rows} rows ({t_tok:.2f}s), global attention of {qrows} query rows x 1 head over {N} keys "
              f"({t_att:.2f}s); extrapolated x{S} frames, x{N / rows:.0f} slabs, x{N * H / qrows:.0f} row groups, "
              f"x{depth} layers = {total:.3g}s per forward")
    return {"value": S / total, "unit": "frames/s", "cores": int(cores), "kind": "oracle", "sample": sample}


def make_embed_weights(model, gen, dtype, dev, n_patch, depth):
    """Front-end parameters (shapes of the C ABI's vggtx_embed_w), N(0, 0.02), norm_g = 1 + N(0, 0.02)."""
    C = model.dim

    def draw(shape, one=False):
        t = torch.empty(shape, device=dev, dtype=torch.float32).normal_(0.0, 0.02, generator=gen)
        return (t + 1.0 if one else t).to(dtype)

    w = {"w_patch": draw((C, 588)), "b_patch": draw((C,)), "pos": draw((1 + n_patch, C)), "cls": draw((C,)),
         "reg": draw((4, C))}
    w["blocks"] = [l["frame"] for l in make_weights(synth.ModelConfig(depth=depth), gen, dtype, dev)]
    w.update({"norm_g": draw((C,), one=True), "norm_b": draw((C,)), "cam": draw((2, C)), "agg_reg": draw((2, 4, C))})
    return w


def embed_cpu_baseline(w_np, img_np, H):
    """FP64 oracle front end on one frame (the front end is per frame), scaled to frames/s."""
    import threadpoolctl

    import oracle
    t0 = time.perf_counter()
    oracle.embed(img_np, w_np, H, 1e-6, frames=[0])
    t = time.perf_counter() - t0
    info = threadpoolctl.threadpool_info()
    cores = max([i.get("num_threads", 1) for i in info] + [1])
    return {"value": 1.0 / t, "unit": "frames/s", "cores": int(cores), "kind": "oracle",
            "sample": f"oracle front end on 1 frame of 518x518 with 24 blocks ({t:.2f}s); frames are independent"}


def bench_embed(args, dev):
    """Patch-embedding front end (per-frame ViT-L/14 at 518 x 518, 24 blocks, BF16)."""
    S, Hi, Wi, depth = args.frames, 518, 518, 24
    model = synth.ModelConfig()
    n_patch = (Hi // 14) * (Wi // 14)
    P = 5 + n_patch
    gen = torch.Generator(device=dev)
    gen.manual_seed(args.seed)
    log(f"front end: generating S={S} images {Hi}x{Wi}, depth {depth}")
    images = torch.empty((S, 3, Hi, Wi), device=dev, dtype=torch.float32).normal_(0, 1, generator=gen)
    w = make_embed_weights(model, gen, torch.bfloat16, dev, n_patch, depth)
    h = vg.Handle(0, dim=model.dim, heads=model.heads, head_dim=model.head_dim, mlp_hidden=model.mlp_hidden,
                  ln_eps=model.ln_eps, frame_chunk=model.frame_chunk)
    ws = torch.empty(vg.embed_workspace_size(h.h, S, Hi, Wi, vg.BF16), dtype=torch.uint8, device=dev)
    out = torch.empty((S, P, model.dim), device=dev, dtype=torch.float32)
    vg.embed(h.h, images[:1], w, vg.BF16, out=out[:1], ws=ws)  # loads the kernels (not a step)
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats(dev)
    for i in range(args.warmup):
        vg.embed(h.h, images, w, vg.BF16, out=out, ws=ws)
        torch.cuda.synchronize()
        log(f"warmup step {i} done")
    vg.timing_enable(h.h, True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(args.steps):
        vg.embed(h.h, images, w, vg.BF16, out=out, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3
    tm = vg.timing_read(h.h)
    vg.timing_enable(h.h, False)
    log(f"front end: {args.steps} step(s) in {sec:.3f}s")
    gm, fa = tm["gemm"], tm["attn_frame"]
    g_tf = gm["flops"] / (gm["ms"] * 1e-3) / 1e12 if gm["ms"] > 0 else None
    f_tf = fa["flops"] / (fa["ms"] * 1e-3) / 1e12 if fa["ms"] > 0 else None
    res = {
        "metric": "front-end frames/s (per-frame patch embedding + 24 ViT-L/14 blocks at 518x518)",
        "value": S * args.steps / sec, "unit": "frames/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"bf16": "bf16", "fp8pv": "bf16 scores, e4m3 P V", "fp8": "e4m3"}[head], "data": "synthetic (images N(0,1), weights N(0,0.02), seeded, device-generated)",
        "config": {"workload": f"vitl14_frontend_S{S}_{Hi}x{Wi}", "frames": S, "image": [Hi, Wi],
                   "tokens_per_frame": P, "dim": model.dim, "heads": model.heads, "mlp_hidden": model.mlp_hidden,
                   "depth": depth, "frame_chunk": model.frame_chunk},
        "gemm_tflops": g_tf, "frame_attn_tflops": f_tf,
        "kernel_time_ms": {k: v["ms"] for k, v in tm.items() if isinstance(v, dict)},
        "peak_hbm_gb": torch.cuda.max_memory_allocated(dev) / 1e9,
        "roofline": {"kernel": "gemm_bf16_kernel (projections, MLP, patch embedding)", "bound": "mfma",
                     "achieved": g_tf, "peak": PEAK_TFLOPS["bf16"], "unit": "TFLOP/s",
                     "frac": g_tf / PEAK_TFLOPS["bf16"] if g_tf else None, "traffic": None,
                     "flops_per_launch": gm["flops"] / max(1, gm["launches"]),
                     "avg_launch_ms": gm["ms"] / max(1, gm["launches"]), "launches": gm["launches"]},
    }
    h.close()
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle front end on one frame")
        w_np = {k: (v.float().cpu().numpy() if k != "blocks" else [{kk: vv.float().cpu().numpy() for kk, vv in b.items()}
                                                                 for b in v]) for k, v in w.items()}
        res["cpu_baseline"] = embed_cpu_baseline(w_np, images[:1].cpu().numpy(), model.heads)
    print(json.dumps(res), flush=True)


def ga_inputs(n_cams, per_pair, seed, dev):
    """Cameras on a full ring looking at the origin (the predicted cameras are
    the true ones perturbed: 1 degree rotation, 0.05 centre, 2% focal), pairs
    under 30 degrees chosen by the library's host rule, and per pair
    `per_pair` correspondences: points N(0, 0.7^2) projected into both true
    cameras, 0.5 px noise, 20% outliers; drawn on the device."""
    rng = np.random.default_rng(seed)
    true, init = synth.gen_ga_cameras(rng, n_cams, arc_deg=360.0)
    init["true_R"], init["true_t"] = true["R"], true["t"]
    pairs = vg.ga_select_pairs(init["R"], 30.0)
    P = len(pairs)
    offsets = [per_pair * m for m in range(P + 1)]
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    Rt = torch.from_numpy(true["R"]).to(dev); tt = torch.from_numpy(true["t"]).to(dev)
    ft = torch.from_numpy(true["f"]).to(dev); ct = torch.from_numpy(true["c"]).to(dev)
    pa = torch.tensor(pairs, dtype=torch.int64, device=dev)
    corr = torch.empty((P * per_pair, 4), dtype=torch.float32, device=dev)
    step = max(1, (1 << 24) // per_pair)
    for m0 in range(0, P, step):
        m1 = min(P, m0 + step)
        n = (m1 - m0) * per_pair
        X = torch.empty((m1 - m0, per_pair, 3), dtype=torch.float64, device=dev).normal_(0, 0.7, generator=gen)
        cols = []
        for side in (0, 1):
            cam = pa[m0:m1, side]
            Rc, tc = Rt[cam], tt[cam]
            Xc = [sum(Rc[:, r, k][:, None] * X[..., k] for k in range(3)) + tc[:, r][:, None] for r in range(3)]
            cols.append(ft[cam][:, None] * Xc[0] / Xc[2] + ct[cam][:, None, 0])
            cols.append(ft[cam][:, None] * Xc[1] / Xc[2] + ct[cam][:, None, 1])
        a = torch.stack(cols, -1).reshape(n, 4)
        a += torch.empty_like(a).normal_(0, 0.5, generator=gen)
        bad = torch.rand(n, device=dev, dtype=torch.float64, generator=gen) < 0.2
        a[bad, 2:] = torch.rand((int(bad.sum()), 2), device=dev, dtype=torch.float64, generator=gen) * 518.0
        corr[m0 * per_pair:m1 * per_pair] = a.float()
    return init, pairs, offsets, corr


def bench_ga(args, dev):
    """Camera global alignment: N cameras, pairs under 30 degrees, 4096
    correspondences per pair, the paper's 300 iterations."""
    n_cams, per_pair = args.cameras, 4096
    log(f"GA: generating {n_cams} cameras, {per_pair} correspondences per pair")
    init, pairs, offsets, corr = ga_inputs(n_cams, per_pair, args.seed, dev)
    P, K = len(pairs), offsets[-1]
    log(f"GA: {P} pairs, {K} correspondences ({K * 16 / 1e9:.2f} GB)")
    cams = [torch.from_numpy(np.ascontiguousarray(init[k])).to(dev) for k in ("R", "t", "f", "c")]
    h = vg.Handle(0, dim=256, heads=4, mlp_hidden=1024)
    ws = torch.empty(vg.ga_workspace_size(h.h, n_cams, P, K), dtype=torch.uint8, device=dev)
    cfg = vg.ga_config_default()
    for i in range(args.warmup):
        vg.ga_align(h.h, *cams, pairs, offsets, corr, cfg, ws=ws)
        torch.cuda.synchronize()
        log(f"warmup run {i} done")
    vg.timing_enable(h.h, True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(args.steps):
        R, t, f, w, lo = vg.ga_align(h.h, *cams, pairs, offsets, corr, cfg, ws=ws)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3
    tm = vg.timing_read(h.h)
    vg.timing_enable(h.h, False)
    lo = lo.cpu().numpy()
    log(f"GA: {args.steps} run(s) in {sec:.3f}s; loss {lo[0]:.4f} -> {lo[-1]:.4f}")
    tr = [torch.from_numpy(np.ascontiguousarray(init["true_" + k])).to(dev) for k in ("R", "t")]
    auc0, _ = vg.auc30(h.h, cams[0], cams[1], *tr)
    a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a0.record()
    auc1, _ = vg.auc30(h.h, R, t, *tr)
    a1.record()
    torch.cuda.synchronize()
    auc_ms = a0.elapsed_time(a1)
    log(f"GA: pose AUC@30 (both orders) {auc0.item():.4f} -> {auc1.item():.4f}")
    oth = tm["other"]
    avg_ms = oth["ms"] / max(1, oth["launches"])
    bytes_per_launch = K * 17.0  # float32 x 4 correspondence + uint8 weight bin, per pass
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    res = {
        "metric": "global alignment: correspondence-iterations/s (300 Adam iterations, pairs under 30 deg, 4096 per pair)",
        "value": K * cfg.iterations * args.steps / sec, "unit": "correspondence-iterations/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": sec * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (ring of cameras, projected points with 0.5 px noise and 20% outliers, seeded)",
        "config": {"workload": f"ga_ring_N{n_cams}_4096perpair", "cameras": n_cams, "pairs": P,
                   "correspondences": K, "iterations": cfg.iterations},
        "loss_first_last": [float(lo[0]), float(lo[-1])],
        "pose_auc30_initial_aligned": [auc0.item(), auc1.item()],
        "auc30_ms": auc_ms,
        "roofline": {"kernel": "ga_pair_kernel (residual + gradient pass)", "bound": "hbm", "achieved": achieved,
                     "peak": 8000.0, "unit": "GB/s", "frac": achieved / 8000.0, "traffic": None,
                     "bytes_per_launch": bytes_per_launch, "avg_launch_ms": avg_ms, "launches": oth["launches"]},
    }
    h.close()
    if not args.no_cpu_baseline:
        from oracle import ga as oga
        sub = min(P, 64)
        c_np = corr[:sub * per_pair].cpu().numpy()
        off = np.arange(sub + 1) * per_pair
        pr = np.array(pairs[:sub])
        bins = oga.hist_bins(oga.all_residuals({k: init[k] for k in ("R", "t", "f", "c")}, pr, off, c_np))
        _, table = oga.weight_table(bins)
        p0 = {"q": oga.rot_to_quat(init["R"]), "t": init["t"].copy(), "phi": np.zeros(n_cams)}
        t0 = time.perf_counter()
        oga.gradient(p0, init["f"], init["c"], pr, off, c_np, table, bins)
        oga.loss(p0, init["f"], init["c"], pr, off, c_np, table, bins)
        tcpu = time.perf_counter() - t0
        import threadpoolctl
        cores = max([i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()] + [1])
        res["cpu_baseline"] = {"value": sub * per_pair / tcpu, "unit": "correspondence-iterations/s",
                               "cores": int(cores), "kind": "oracle",
                               "sample": f"one oracle iteration (loss + gradient) over {sub} pairs x {per_pair} ({tcpu:.2f}s)"}
    print(json.dumps(res), flush=True)


def bench_heads(args, dev):
    """Head-input packing of the aggregator output at S frames (4 kept layers,
    P = 1374, 2C = 2048, bfloat16): bytes moved per second."""
    S, n_out, C2, gh = args.frames, 4, 2048, 37
    P = 5 + gh * gh
    gen = torch.Generator(device=dev)
    gen.manual_seed(args.seed)
    feats = torch.empty((n_out, S, P, C2), device=dev, dtype=torch.float32)
    for l in range(n_out):
        feats[l].normal_(0, 1, generator=gen)
    feats = feats.to(torch.bfloat16)
    out = torch.empty((n_out, S, C2, gh, gh), device=dev, dtype=torch.bfloat16)
    h = vg.Handle(0, dim=1024, heads=16, mlp_hidden=4096)
    vg.pack_head_inputs(h.h, feats, gh, gh, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        vg.pack_head_inputs(h.h, feats, gh, gh, out=out)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3 / args.steps
    moved = 2.0 * n_out * S * (P - 5) * C2 * 2  # read the patch rows once, write them once
    h.close()
    print(json.dumps({
        "metric": "head-input packing GB/s (4 kept layers, S frames, 37x37 patches, 2C=2048, bf16)",
        "value": moved / sec / 1e9, "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic (N(0,1) features)", "config": {"workload": f"head_packing_S{S}", "frames": S},
        "roofline": {"kernel": "pack_heads_kernel", "bound": "hbm", "achieved": moved / sec / 1e9, "peak": 8000.0,
                     "unit": "GB/s", "frac": moved / sec / 1e9 / 8000.0, "traffic": None}}), flush=True)


def plan_steps(req_steps, req_warmup, est_step_s, budget_s):
    """Timed steps and warm-up steps that fit a wall-clock budget.

    At least one timed step always runs.  Further timed steps, then warm-up
    steps, are added while est_step_s times their count stays within
    budget_s; requested counts are never exceeded."""
    fit = int(budget_s // est_step_s) if est_step_s > 0 else req_steps + req_warmup
    steps = max(1, min(req_steps, fit))
    warmup = max(0, min(req_warmup, fit - steps))
    return steps, warmup


def forward_flops(S, P, model, depth=None):
    """Algorithmic flops of one aggregator forward over one scene of S frames."""
    N, C, F = S * P, model.dim, model.mlp_hidden
    depth = model.depth if depth is None else depth
    per_block = 2.0 * N * C * (3 * C + C + 2 * F)
    return depth * (2 * per_block + 4.0 * S * P * P * C + 4.0 * N * N * C)


def wait_logged(ev, h, tag, n_ga, t0, every_s=15.0):
    """Wait for event `ev`, printing how many global-attention launches have
    finished every `every_s` seconds (a step runs for minutes at S=1000)."""
    last = time.perf_counter()
    while not ev.query():
        time.sleep(1.0)
        if time.perf_counter() - last >= every_s:
            last = time.perf_counter()
            _, _, ga_done = vg.timing_poll(h)
            log(f"{tag}: global attention launches finished {ga_done}/{n_ga} ({last - t0:.0f}s)")
    ev.synchronize()


def enqueue_logged(fn, ev, h, tag, n_ga, t0):
    """Run `fn` (which enqueues forwards and records `ev` last) on a worker
    thread and wait for `ev`, printing finished global-attention launches as
    they complete.  At S=1000 enqueueing one forward blocks in the launch
    queue for most of its run time, so the waiting happens on this thread."""
    err = []

    def work():
        try:
            fn()
        except BaseException as e:  # re-raised below
            err.append(e)

    th = threading.Thread(target=work, daemon=True)
    th.start()
    last = time.perf_counter()
    while th.is_alive():
        th.join(1.0)
        if time.perf_counter() - last >= 15.0:
            last = time.perf_counter()
            _, _, ga_done = vg.timing_poll(h)
            log(f"{tag}: global attention launches finished {ga_done}/{n_ga} ({last - t0:.0f}s)")
    if err:
        raise err[0]
    wait_logged(ev, h, tag, n_ga, t0)


def run_forward(h, tokens, layers, prec, out, ws, steps, warmup, tag, draw, fwd=None, n_ga=None):
    """`warmup` untimed and `steps` timed aggregator forwards; returns (seconds
    of the timed steps from device events, library kernel timing, peak HBM GB).
    The handle runs the residual stream in the tokens buffer (tokens_inplace),
    so `draw` (the seeded N(0, 1) draw of the input, a few milliseconds against
    minutes per forward) refills it before every forward.  `fwd` replaces the
    single-scene forward (the varlen stage); `n_ga` is the number of global
    attention launches per forward (progress lines only)."""
    dev = tokens.device
    if fwd is None:
        def fwd():
            vg.aggregate(h, tokens, layers, OUT_LAYERS, prec, out=out, ws=ws)
    n_ga = max(OUT_LAYERS) + 1 if n_ga is None else n_ga
    for i in range(warmup):
        e = torch.cuda.Event()
        vg.timing_enable(h, True)

        def one():
            draw()
            fwd()
            e.record()

        enqueue_logged(one, e, h, f"{tag} warmup {i}", n_ga, time.perf_counter())
        vg.timing_enable(h, False)
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats(dev)
    vg.timing_enable(h, True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()

    def timed():
        for i in range(steps):
            draw()
            fwd()
        e1.record()

    enqueue_logged(timed, e1, h, f"{tag} timed", n_ga * steps, t0)
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) * 1e-3
    tm = vg.timing_read(h)
    vg.timing_enable(h, False)
    if tm["dropped"]:
        raise RuntimeError(f"{tm['dropped']} kernel timing records were dropped")
    peak = torch.cuda.max_memory_allocated(dev) / 1e9
    log(f"{tag}: {steps} timed step(s) in {sec:.3f}s (host wall {time.perf_counter() - t0:.1f}s), peak {peak:.1f} GB")
    return sec, tm, peak


def attn_rate(tm):
    ga = tm["attn_global"]
    return ga["flops"] / (ga["ms"] * 1e-3) / 1e12 if ga["ms"] > 0 else None


def accuracy_vs_f32(h, precs, dev, seed=1):
    """max|g - r| / max|r| of global attention at each precision against the
    float32 kernel (itself within 1e-4 of the float64 definition) on the
    same bf16-valued Q, K, V: 4 heads, 8 frames x 86 tokens, in the three
    logit regimes (R0 random-init, R1 logit std ~3, R2 peaked)."""
    res = {}
    for regime in ("R0", "R1", "R2"):
        q, k, v = synth.gen_qkv(np.random.default_rng(seed), 4, 8 * 86, 64, regime, frames=8, bf16=True)
        t32 = [torch.from_numpy(np.ascontiguousarray(a.transpose(1, 0, 2), dtype=np.float32)).to(dev)
               for a in (q, k, v)]
        ref = torch.empty_like(t32[0])
        vg.attn_global(h, *t32, ref, [0, 8 * 86], vg.F32)
        r = ref.double()
        for name, prec in precs.items():
            tb = [a.to(torch.bfloat16) for a in t32]
            o = torch.empty_like(tb[0])
            vg.attn_global(h, *tb, o, [0, 8 * 86], prec)
            e = float((o.double() - r).abs().max() / r.abs().max())
            res.setdefault(name, {})[regime] = e
    torch.cuda.synchronize()
    return res


def bench_aggregator(args, dev):
    """Headline: the bfloat16 aggregator forward at S frames; then, as far as
    the wall budget allows, the FP8 forwards and the float32 attention rate."""
    S, P = args.frames, P_TOKENS
    model = synth.ModelConfig()
    gen = torch.Generator(device=dev)
    gen.manual_seed(args.seed)
    log(f"generating inputs: S={S} P={P} C={model.dim} depth={model.depth}")
    tokens = torch.empty((S, P, model.dim), device=dev, dtype=torch.float32)
    gen_tok = torch.Generator(device=dev)

    def draw():
        tokens.normal_(0, 1, generator=gen_tok.manual_seed(args.seed + 7))

    draw()
    layers = make_weights(model, gen, torch.bfloat16, dev)
    h = vg.Handle(0, dim=model.dim, heads=model.heads, head_dim=model.head_dim, mlp_hidden=model.mlp_hidden,
                  ln_eps=model.ln_eps, frame_chunk=model.frame_chunk, tokens_inplace=True,
                  attn_schedule=vg.SCHEDULE_GRID if args.schedule == "grid" else vg.SCHEDULE_QUEUE)
    # bfloat16 headline, then the FP8 mode that keeps the scores in bfloat16
    # (E4M3 P and V), then the all-E4M3 one
    lowp = {"bf16": vg.BF16, "fp8pv": vg.FP8_PV, "fp8": vg.FP8_E4M3}
    ws = torch.empty(max(vg.workspace_size(h.h, S, P, p) for p in lowp.values()), dtype=torch.uint8, device=dev)
    out = torch.empty((len(OUT_LAYERS), S, P, 2 * model.dim), device=dev, dtype=torch.bfloat16)
    for p in lowp.values():  # load the kernels with one-frame calls (not steps)
        vg.aggregate(h.h, tokens[:1], layers, [0], p, out=out[:1, :1], ws=ws)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - T_START
    fl = forward_flops(S, P, model)
    est = fl / (args.assumed_tflops * 1e12)
    # keep room for one forward of each FP8 mode (measured at about 0.75 and 0.85 of a bfloat16 one)
    extra = 0.0 if args.no_extra else est * (0.75 + (0.85 if "fp8pv" in lowp else 0.0))
    steps, warmup = plan_steps(args.steps, args.warmup, est, args.wall_budget - elapsed - args.reserve - extra)
    log(f"setup done at {elapsed:.0f}s; estimated {est:.1f}s per step; running {warmup} warm-up + {steps} timed "
        f"step(s) (requested {args.warmup} + {args.steps})")
    head = args.headline
    sec, tm, peak = run_forward(h.h, tokens, layers, lowp[head], out, ws, steps, warmup, head, draw)
    step_s = sec / steps
    ga_tf = attn_rate(tm)
    ga = tm["attn_global"]
    per_prec = {head: {"frames_per_s": S * steps / sec, "ms_per_step": step_s * 1e3, "global_attn_tflops": ga_tf,
                       "global_attn_frac_of_peak": ga_tf / PEAK_TFLOPS[head] if ga_tf else None,
                       "peak_hbm_gb": peak, "kernel_time_ms": {k: v["ms"] for k, v in tm.items()
                                                               if isinstance(v, dict)}}}
    # FP8 forwards while they fit (their steps take about as long as the global attention's share allows);
    # a mode whose forward does not fit gets the rate of one standalone 16-head global attention launch
    standalone = []
    for name in [n for n in lowp if n != head]:
        if args.no_extra:
            break
        guess = step_s * {"bf16": 1.0, "fp8pv": 0.85, "fp8": 0.75}[name] / {"bf16": 1.0, "fp8pv": 0.85, "fp8": 0.75}[head]
        left = args.wall_budget - (time.perf_counter() - T_START) - args.reserve
        if guess > left:
            per_prec[name] = {"forward_skipped": f"wall budget: about {guess:.0f}s needed, {left:.0f}s left"}
            log(f"{name}: forward skipped ({per_prec[name]['forward_skipped']}); standalone attention rate instead")
            standalone.append(name)
            continue
        s2, tm2, pk2 = run_forward(h.h, tokens, layers, lowp[name], out, ws, 1, 0, name, draw)
        r2 = attn_rate(tm2)
        per_prec[name] = {"frames_per_s": S / s2, "ms_per_step": s2 * 1e3, "global_attn_tflops": r2,
                          "global_attn_frac_of_peak": r2 / PEAK_TFLOPS[name] if r2 else None, "peak_hbm_gb": pk2,
                          "kernel_time_ms": {k: v["ms"] for k, v in tm2.items() if isinstance(v, dict)}}
    del out, ws
    torch.cuda.empty_cache()
    if not args.no_extra:
        gen2 = torch.Generator(device=dev)
        gen2.manual_seed(args.seed + 1)
        for name in standalone:
            r, ms = attn_only_rate(h.h, S, lowp[name], dev, gen2, heads=model.heads)
            per_prec[name].update({"global_attn_tflops": r, "global_attn_frac_of_peak": r / PEAK_TFLOPS[name],
                                   "sample": f"standalone global attention, {model.heads} heads of 64 over S*P = "
                                             f"{S * P} tokens ({ms:.0f} ms, one launch of the layer's shape)"})
            log(f"{name} global attention, standalone, S={S}: {r:.1f} TFLOP/s")
        r, ms = attn_only_rate(h.h, S, vg.F32, dev, gen2, heads=1)
        per_prec["f32"] = {"global_attn_tflops": r, "global_attn_frac_of_peak": r / PEAK_TFLOPS["f32"],
                           "sample": f"standalone global attention, one head of 64 over S*P = {S * P} tokens "
                                     f"({ms:.0f} ms; the full layer has 16 identical heads)"}
        log(f"f32 global attention, one head, S={S}: {r:.1f} TFLOP/s")
        acc = accuracy_vs_f32(h.h, {k: v for k, v in lowp.items()}, dev)
        for name, errs in acc.items():
            gate = 2e-2 if name == "bf16" else 6e-2
            entry = per_prec.setdefault(name, {})
            entry["attn_max_abs_rel_vs_f32"] = errs
            entry["accuracy_gate"] = gate
            entry["meets_gate_in"] = [rg for rg, e in errs.items() if e < gate]
        log(f"accuracy against the float32 kernel: {acc}")
    h.close()

    avg_ms = ga["ms"] / max(1, ga["launches"])
    res = {
        "metric": "frames/sec + global-attn TFLOP/s at S=1000 (BF16 vs FP8 vs FP32), peak HBM GB",
        "value": S * steps / sec,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "steps_requested": args.steps,
        "warmup_requested": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16": "bf16", "fp8pv": "bf16 scores, e4m3 P V", "fp8": "e4m3"}[head],
        "data": "synthetic (tokens N(0,1) drawn on the device with a fixed seed before every forward, which runs "
                "its residual stream in that buffer; weights N(0,0.02), seeded)",
        "config": {"workload": f"vggt_l_aggregator_S{S}_P{P}_{head}", "frames": S, "tokens_per_frame": P,
                   "global_tokens": S * P, "dim": model.dim, "heads": model.heads, "head_dim": model.head_dim,
                   "mlp_hidden": model.mlp_hidden, "depth": model.depth, "out_layers": list(OUT_LAYERS),
                   "frame_chunk": model.frame_chunk, "attn_schedule": args.schedule},
        "wall_budget_s": args.wall_budget,
        "global_attn_tflops": ga_tf,
        "peak_hbm_gb": peak,
        "precisions": per_prec,
        "roofline": {
            "kernel": f"attn_{head}_kernel (global attention)",
            "bound": "mfma",
            "achieved": ga_tf,
            "peak": PEAK_TFLOPS[head],
            "unit": "TFLOP/s",
            "frac": (ga_tf / PEAK_TFLOPS[head]) if ga_tf else None,
            "traffic": measured_traffic(head, S),
            "flops_per_launch": ga["flops"] / max(1, ga["launches"]),
            "avg_launch_ms": avg_ms,
            "launches": ga["launches"],
        },
    }
    if args.copy_calibration:
        src = torch.empty(1 << 30, dtype=torch.bfloat16, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy done: 2 GiB read, 2 GiB written")
        del src, dst
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a bounded sample")
        res["cpu_baseline"] = cpu_baseline(S, P)
    log(f"done at {time.perf_counter() - T_START:.0f}s")
    print(json.dumps(res), flush=True)


def varlen_flops(frames, P, model):
    """Algorithmic flops of one aggregator forward over scenes of the given
    frame counts (global attention within each scene only)."""
    N, C, F = sum(frames) * P, model.dim, model.mlp_hidden
    per_block = 2.0 * N * C * (3 * C + C + 2 * F)
    glob = sum(4.0 * (f * P) ** 2 * C for f in frames)
    return model.depth * (2 * per_block + 4.0 * N * P * C + glob)


def bench_varlen(args, dev):
    """The batched multi-scene workload: 12 scenes of 16..300 frames (seeded
    uniform draw, 1684 frames, 2.31M tokens) as one varlen aggregator forward
    in bfloat16; each global layer is one attention launch over all scenes,
    longest scene first."""
    frames = synth.varlen_scene_frames()
    S, P = sum(frames), P_TOKENS
    offs = [0]
    for f in frames:
        offs.append(offs[-1] + f)
    model = synth.ModelConfig()
    gen = torch.Generator(device=dev)
    gen.manual_seed(args.seed)
    log(f"varlen: {len(frames)} scenes, frames {list(frames)}, S={S}, P={P}")
    tokens = torch.empty((S, P, model.dim), device=dev, dtype=torch.float32)
    gen_tok = torch.Generator(device=dev)

    def draw():
        tokens.normal_(0, 1, generator=gen_tok.manual_seed(args.seed + 7))

    draw()
    layers = make_weights(model, gen, torch.bfloat16, dev)
    h = vg.Handle(0, dim=model.dim, heads=model.heads, head_dim=model.head_dim, mlp_hidden=model.mlp_hidden,
                  ln_eps=model.ln_eps, frame_chunk=model.frame_chunk, tokens_inplace=True,
                  attn_schedule=vg.SCHEDULE_GRID if args.schedule == "grid" else vg.SCHEDULE_QUEUE)
    prec = vg.BF16
    ws = torch.empty(vg.workspace_size(h.h, S, P, prec), dtype=torch.uint8, device=dev)
    out = torch.empty((len(OUT_LAYERS), S, P, 2 * model.dim), device=dev, dtype=torch.bfloat16)
    vg.aggregate(h.h, tokens[:1], layers, [0], prec, out=out[:1, :1], ws=ws)  # load the kernels
    torch.cuda.synchronize()

    def fwd():
        vg.aggregate_varlen(h.h, tokens, offs, layers, OUT_LAYERS, prec, out=out, ws=ws)

    fl = varlen_flops(frames, P, model)
    est = fl / (args.assumed_tflops * 1e12)
    elapsed = time.perf_counter() - T_START
    steps, warmup = plan_steps(args.steps, args.warmup, est, args.wall_budget - elapsed - 10.0)
    log(f"estimated {est:.1f}s per step; running {warmup} warm-up + {steps} timed step(s)")
    sec, tm, peak = run_forward(h.h, tokens, layers, prec, out, ws, steps, warmup, "varlen bf16", draw, fwd=fwd)
    h.close()
    ga = tm["attn_global"]
    ga_tf = attn_rate(tm)
    res = {
        "metric": "frames/sec + global-attn TFLOP/s, 12-scene varlen batch (BF16), peak HBM GB",
        "value": S * steps / sec,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": sec / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"bf16": "bf16", "fp8pv": "bf16 scores, e4m3 P V", "fp8": "e4m3"}[head],
        "data": "synthetic (tokens N(0,1) drawn on the device with a fixed seed before every forward; "
                "weights N(0,0.02), seeded)",
        "config": {"workload": f"vggt_l_varlen{len(frames)}_bf16", "scene_frames": list(frames), "frames": S,
                   "tokens_per_frame": P, "global_tokens": S * P, "depth": model.depth,
                   "out_layers": list(OUT_LAYERS), "attn_schedule": args.schedule},
        "forward_tflops": fl / (sec / steps) / 1e12,
        "global_attn_tflops": ga_tf,
        "global_attn_frac_of_peak": ga_tf / PEAK_TFLOPS["bf16"] if ga_tf else None,
        "global_attn_launches": ga["launches"],
        "peak_hbm_gb": peak,
        "kernel_time_ms": {k: v["ms"] for k, v in tm.items() if isinstance(v, dict)},
    }
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--frames", type=int, default=1000)
    ap.add_argument("--wall-budget", type=float, default=500.0,
                    help="seconds from process start within which the run should end; timed steps beyond the "
                         "first, warm-up steps and the extra legs are cut to fit (the counts run are reported)")
    ap.add_argument("--reserve", type=float, default=45.0,
                    help="seconds of the budget kept for the float32 leg, the accuracy check and the CPU baseline")
    ap.add_argument("--assumed-tflops", type=float, default=1000.0,
                    help="forward rate assumed when planning steps before any has run")
    ap.add_argument("--no-extra", action="store_true", help="skip the FP8 forwards, the FP32 rate and the accuracy check")
    ap.add_argument("--headline", choices=["bf16", "fp8pv", "fp8"], default="bf16",
                    help="precision of the timed forward (the others run as extra legs); bf16 is the headline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the run, copy 2 GiB device to device (calibrates HBM byte counters)")
    ap.add_argument("--stage", choices=["aggregator", "varlen", "embed", "ga", "heads"], default="aggregator",
                    help="aggregator (default): the aggregator forward; varlen: the 12-scene batch in one varlen "
                         "forward; embed: the patch-embedding front end; ga: camera global alignment; heads: "
                         "head-input packing")
    ap.add_argument("--cameras", type=int, default=1000, help="--stage ga: number of cameras")
    ap.add_argument("--schedule", choices=["queue", "grid"], default="queue",
                    help="global attention work distribution (queue: work counter, longest scene first; grid: one "
                         "workgroup per item)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              f"(the multi-GPU sharding of the path is a design, not an implementation).", file=sys.stderr)
        sys.exit(2)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.stage == "embed":
        bench_embed(args, dev)
    elif args.stage == "ga":
        bench_ga(args, dev)
    elif args.stage == "heads":
        bench_heads(args, dev)
    elif args.stage == "varlen":
        bench_varlen(args, dev)
    else:
        bench_aggregator(args, dev)


if __name__ == "__main__":
    main()
