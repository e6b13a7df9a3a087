"""Parity at the full VGGT-L shapes (C=1024, 16 heads x 64, MLP 4096, P=1374).

* 24-layer aggregator at S=32 frames (43,968 global tokens, BF16) and at
  S=200 frames (274,800 global tokens, FP8 global attention): every
  requested layer's global half is checked on 256 sampled rows against the
  FP64 global block fed with the GPU's own frame-block output of that layer
  (teacher forcing); the frame half on 4 frames against the FP64 frame block
  fed with the previous layer's global output.  This measures each layer's
  local error; the whole-network drift is covered at small sizes.
* The S=200 configuration in BF16 (the precision the configuration states;
  its 128-frame chunks also cover the multi-chunk path at this width).
* Layer 0 of the S=1000 configuration (1,374,000 global tokens, FP8 global
  attention), teacher-forced the same way.
* The whole 24-layer network, not teacher forced, at S=2 frames (2,748
  tokens) in BF16 and FP8: layers 4/11/17/23 against the FP64 forward of the
  same input, so the drift over 24 bfloat16 layers is measured.
* The 12-scene varlen batch (frame counts drawn from 16..300, about 1,900
  frames, 2.6 M tokens) through the aggregator in BF16, teacher-forced on
  sampled rows and frames of its longest and shortest scene.
* Global attention at S=1000 frames (1,374,000 tokens) in BF16 and FP8, and
  over the 12-scene varlen batch, in the launch configuration the benchmark
  times; the oracle evaluates sampled query rows against all keys.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import DEV, max_abs_rel, to_dev

vg = pytest.importorskip("paper_2509_25191_amd.vggtx")
pytestmark = pytest.mark.gpu

P = 1374


def _bf16_weights_dev(layers):
    return [{part: {k: torch.from_numpy(v).to(DEV).to(torch.bfloat16) for k, v in blk.items()}
             for part, blk in l.items()} for l in layers]


def _teacher_forced(S, prec, keep, tol_frame, tol_global, seed):
    m = synth.ModelConfig()
    N = S * P
    tokens, layers = synth.gen_problem(m, S, P, seed=seed, bf16=True)
    req = sorted(set(keep) | {l - 1 for l in keep})
    h = vg.Handle(0, dim=m.dim, heads=m.heads, mlp_hidden=m.mlp_hidden)
    out = vg.aggregate(h.h, to_dev(tokens, torch.float32), _bf16_weights_dev(layers), req, prec,
                       out_dtype=vg.OUT_F32)
    torch.cuda.synchronize()
    del tokens
    C = m.dim
    rows = synth.sample_rows(seed, N, 256, P)
    frames = [0, S - 1, 7, 19]
    for l in keep:
        i, ip = req.index(l), req.index(l - 1)
        fo = out[i, :, :, :C].reshape(N, C).cpu().numpy().astype(np.float64)
        go_rows = out[i, :, :, C:].reshape(N, C)[torch.from_numpy(rows).to(DEV)].cpu().numpy()
        ref_g = oracle.global_block_rows(fo, layers[l]["global"], rows, m.heads, m.ln_eps)
        del fo
        eg = max_abs_rel(go_rows, ref_g)
        prev = out[ip, :, :, C:].reshape(N, C)[: (max(frames) + 1) * P].cpu().numpy().astype(np.float64)
        ref_f = oracle.frame_block_frames(prev, layers[l]["frame"], frames, P, m.heads, m.ln_eps)
        got_f = out[i, frames, :, :C].cpu().numpy()
        ef = max_abs_rel(got_f, ref_f)
        print(f"S={S} prec={prec} layer {l}: frame half {ef:.3e}  global half {eg:.3e}", flush=True)
        assert ef < tol_frame and eg < tol_global
    h.close()


def test_aggregate_vggt_l_s32_teacher_forced():
    _teacher_forced(32, vg.BF16, [4, 11, 17, 23], 2e-2, 2e-2, seed=0)


def test_aggregate_vggt_l_s200_fp8_teacher_forced():
    """The S=200 configuration with FP8 global attention (frame blocks BF16)."""
    _teacher_forced(200, vg.FP8_E4M3, [4, 23], 2e-2, 6e-2, seed=200)


@pytest.mark.timeout(600)
def test_aggregate_vggt_l_s200_bf16_teacher_forced():
    """The S=200 configuration as stated: BF16 operands, FP32 accumulation."""
    _teacher_forced(200, vg.BF16, [4, 11, 17, 23], 2e-2, 2e-2, seed=201)


_E2E = {}


def _e2e_problem():
    """Depth-24 VGGT-L weights, S=2 frames of P tokens, and the FP64 forward (computed once)."""
    if not _E2E:
        m = synth.ModelConfig()
        tokens, layers = synth.gen_problem(m, 2, P, seed=24, bf16=True)
        ref = oracle.aggregate(tokens, layers, [4, 11, 17, 23], m.heads, m.ln_eps)
        _E2E.update(m=m, tokens=tokens, layers=layers, ref=ref)
    return _E2E


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec,tol", [(vg.BF16, 2e-2), (vg.FP8_E4M3, 6e-2), (vg.FP8_PV, 6e-2)])
def test_aggregate_vggt_l_depth24_end_to_end(prec, tol):
    """All 24 layers at C=1024, H=16, F=4096, P=1374, S=2, with no teacher
    forcing: the GPU output of layers 4/11/17/23 against the FP64 forward."""
    pr = _e2e_problem()
    m, layers, ref = pr["m"], pr["layers"], pr["ref"]
    h = vg.Handle(0, dim=m.dim, heads=m.heads, mlp_hidden=m.mlp_hidden)
    out = vg.aggregate(h.h, to_dev(pr["tokens"], torch.float32), _bf16_weights_dev(layers), [4, 11, 17, 23], prec,
                       out_dtype=vg.OUT_F32)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    h.close()
    C = m.dim
    worst = 0.0
    for i, l in enumerate((4, 11, 17, 23)):
        ef = max_abs_rel(got[i, ..., :C], ref[i, ..., :C])
        eg = max_abs_rel(got[i, ..., C:], ref[i, ..., C:])
        print(f"depth-24 end-to-end S=2 prec={prec} layer {l}: frame half {ef:.3e}  global half {eg:.3e}",
              flush=True)
        worst = max(worst, ef, eg)
    assert worst < tol


@pytest.mark.timeout(900)
def test_aggregate_varlen_12_scenes_bf16_teacher_forced():
    """12 scenes with frame counts drawn from 16..300 in one aggregator call
    (BF16, layer 0): for the longest and the shortest scene, the frame half
    of two frames against the FP64 frame block of the input tokens and the
    global half of 128 sampled rows against the FP64 global block of that
    scene, fed with the GPU's frame output."""
    m = synth.ModelConfig()
    C = m.dim
    frames = synth.varlen_scene_frames()
    foff = np.concatenate([[0], np.cumsum(frames)]).astype(np.int64)
    S = int(foff[-1])
    g = torch.Generator(device=DEV)
    g.manual_seed(12)
    tokens = torch.empty((S, P, C), device=DEV).normal_(0, 1, generator=g)
    rng = np.random.default_rng(12)
    lw = {"frame": synth.gen_block(rng, C, m.mlp_hidden, bf16=True),
          "global": synth.gen_block(rng, C, m.mlp_hidden, bf16=True)}
    h = vg.Handle(0, dim=C, heads=m.heads, mlp_hidden=m.mlp_hidden)
    out = vg.aggregate_varlen(h.h, tokens, foff.tolist(), _bf16_weights_dev([lw]), [0], vg.BF16,
                              out_dtype=vg.OUT_F32)
    torch.cuda.synchronize()
    print(f"varlen aggregator: scenes {list(frames)} ({S} frames, {S * P} tokens)", flush=True)
    for sc in (int(np.argmax(frames)), int(np.argmin(frames))):
        a, b = int(foff[sc]), int(foff[sc + 1])
        fr = [a, b - 1]
        x_in = tokens[fr].reshape(-1, C).cpu().numpy().astype(np.float64)
        ref_f = oracle.frame_block_frames(x_in, lw["frame"], [0, 1], P, m.heads, m.ln_eps)
        ef = max_abs_rel(out[0, fr, :, :C].cpu().numpy(), ref_f)
        n = (b - a) * P
        rows = synth.sample_rows(sc, n, 128, P)
        fo = out[0, a:b, :, :C].reshape(n, C).cpu().numpy()
        go = out[0, a:b, :, C:].reshape(n, C)[torch.from_numpy(rows).to(DEV)].cpu().numpy()
        ref_g = oracle.global_block_rows(fo, lw["global"], rows, m.heads, m.ln_eps)
        del fo
        eg = max_abs_rel(go, ref_g)
        print(f"varlen scene {sc} ({b - a} frames): frame half {ef:.3e}  global half {eg:.3e}", flush=True)
        assert ef < 2e-2 and eg < 2e-2
    h.close()


def _dev_qkv(N, H, seed, std_qk=0.64):
    g = torch.Generator(device=DEV)
    g.manual_seed(seed)
    q = torch.empty((N, H, 64), device=DEV).normal_(0, std_qk, generator=g).to(torch.bfloat16)
    k = torch.empty((N, H, 64), device=DEV).normal_(0, std_qk, generator=g).to(torch.bfloat16)
    v = torch.empty((N, H, 64), device=DEV).normal_(0, 1.0, generator=g).to(torch.bfloat16)
    return q, k, v


def _check_rows(q, k, v, o, seq_start, seq_end, rows, heads):
    """Oracle attention of the given rows (absolute indices inside [seq_start, seq_end))."""
    errs = []
    for hh in heads:
        kk = k[seq_start:seq_end, hh].float().cpu().numpy()[None]
        vv = v[seq_start:seq_end, hh].float().cpu().numpy()[None]
        qq = q[rows, hh].float().cpu().numpy()[None]
        ref = oracle.attention(qq, kk, vv)[0]
        got = o[rows, hh].float().cpu().numpy()
        errs.append(max_abs_rel(got, ref))
    return max(errs)


@pytest.mark.parametrize("prec,tol", [(vg.BF16, 2e-2), (vg.FP8_E4M3, 6e-2), (vg.FP8_PV, 6e-2)])
def test_attn_global_s1000_sampled_rows(prec, tol):
    S, H = 1000, 16
    N = S * P
    h = vg.Handle(0, dim=1024, heads=16, mlp_hidden=4096)
    q, k, v = _dev_qkv(N, H, seed=1000 + prec)
    o = torch.empty_like(q)
    vg.attn_global(h.h, q, k, v, o, [0, N], prec)
    torch.cuda.synchronize()
    rows = torch.from_numpy(synth.sample_rows(1000, N, 64, P)).to(DEV)
    e = _check_rows(q, k, v, o, 0, N, rows, heads=[0, 7, 15])
    print(f"S=1000 global attention prec={prec}: max_abs_rel on 64 rows x 3 heads = {e:.3e}")
    assert e < tol
    h.close()


def test_attn_global_varlen_12_scenes_sampled_rows():
    H = 16
    frames = synth.varlen_scene_frames()
    offs = np.concatenate([[0], np.cumsum(frames)]) * P
    N = int(offs[-1])
    h = vg.Handle(0, dim=1024, heads=16, mlp_hidden=4096)
    q, k, v = _dev_qkv(N, H, seed=12)
    o = torch.empty_like(q)
    vg.attn_global(h.h, q, k, v, o, offs.tolist(), vg.BF16)
    torch.cuda.synchronize()
    worst = 0.0
    rng = np.random.default_rng(12)
    for i in range(len(frames)):
        a, b = int(offs[i]), int(offs[i + 1])
        rows = np.unique(np.concatenate([[a, b - 1], rng.integers(a, b, 6)]))
        worst = max(worst, _check_rows(q, k, v, o, a, b, torch.from_numpy(rows).to(DEV), heads=[int(rng.integers(0, H))]))
    print(f"varlen 12 scenes ({frames}) max_abs_rel = {worst:.3e}")
    assert worst < 2e-2
    h.close()


def test_aggregate_vggt_l_s1000_layer0_fp8():
    """Layer 0 of the S=1000 configuration (1,374,000 global tokens) with FP8
    global attention, in the benchmark's launch configuration: the global half
    on 256 sampled rows against the FP64 global block fed with the GPU's frame
    output, the frame half on 4 frames against the FP64 frame block of the
    input tokens."""
    m = synth.ModelConfig()
    S = 1000
    N = S * P
    C = m.dim
    rng = np.random.default_rng(1000)
    tokens = rng.standard_normal((S, P, C), dtype=np.float32)
    lw = {"frame": synth.gen_block(rng, C, m.mlp_hidden, bf16=True),
          "global": synth.gen_block(rng, C, m.mlp_hidden, bf16=True)}
    h = vg.Handle(0, dim=C, heads=m.heads, mlp_hidden=m.mlp_hidden)
    out = vg.aggregate(h.h, to_dev(tokens, torch.float32), _bf16_weights_dev([lw]), [0], vg.FP8_E4M3,
                       out_dtype=vg.OUT_F32)
    torch.cuda.synchronize()
    frames = [0, S - 1, 7, 519]
    got_f = out[0, frames, :, :C].cpu().numpy()
    ref_f = oracle.frame_block_frames(tokens.reshape(N, C)[: (max(frames) + 1) * P].astype(np.float64),
                                      lw["frame"], frames, P, m.heads, m.ln_eps)
    ef = max_abs_rel(got_f, ref_f)
    del ref_f
    rows = synth.sample_rows(1000, N, 256, P)
    go_rows = out[0, :, :, C:].reshape(N, C)[torch.from_numpy(rows).to(DEV)].cpu().numpy()
    fo = out[0, :, :, :C].reshape(N, C).cpu().numpy()
    del out
    h.close()
    ref_g = oracle.global_block_rows(fo, lw["global"], rows, m.heads, m.ln_eps)
    eg = max_abs_rel(go_rows, ref_g)
    print(f"S=1000 FP8 layer 0: frame half {ef:.3e}  global half {eg:.3e}", flush=True)
    assert ef < 2e-2 and eg < 6e-2
