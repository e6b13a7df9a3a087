"""Parity of the HIP patch-embedding front end (Sec. 3.2: per-frame DINO-based
patch embedding, processed in frame chunks) with the FP64 oracle, its chunking
invariance, its host-side validation, and the images -> features pipeline
(front end, then aggregator)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import DEV, max_abs_rel, to_dev, weights_to_dev

vg = pytest.importorskip("paper_2509_25191_amd.vggtx")
pytestmark = pytest.mark.gpu

SMALL = synth.ModelConfig(dim=256, heads=4, head_dim=64, mlp_hidden=1024, depth=1)
E_INVALID, E_WORKSPACE = 1, 3


def _handle(m, chunk=128):
    return vg.Handle(0, dim=m.dim, heads=m.heads, head_dim=m.head_dim, mlp_hidden=m.mlp_hidden,
                     ln_eps=m.ln_eps, frame_chunk=chunk)


def _dt(prec):
    return torch.float32 if prec == vg.F32 else torch.bfloat16


def _embed_to_dev(w, dtype):
    d = {k: to_dev(w[k], dtype) for k in vg.EMBED_FIELDS}
    d["blocks"] = [{k: to_dev(v, dtype) for k, v in b.items()} for b in w["blocks"]]
    return d


def _problem(m, S, hw, depth, seed, bf16, std=0.02):
    rng = np.random.default_rng(seed)
    img = synth.gen_images(rng, S, *hw)
    w = synth.gen_embed(rng, m, hw[0], hw[1], depth, std=std, bf16=bf16)
    return img, w


def _check_special(got, w, scenes):
    firsts = set(np.concatenate([[0], np.cumsum(scenes)[:-1]]).tolist())
    for f in range(got.shape[0]):
        s = 0 if f in firsts else 1
        np.testing.assert_array_equal(got[f, 0], np.asarray(w["cam"][s], np.float32))
        np.testing.assert_array_equal(got[f, 1:5], np.asarray(w["agg_reg"][s], np.float32))


@pytest.mark.parametrize("prec,tol", [(vg.F32, 1e-4), (vg.BF16, 2e-2)])
@pytest.mark.parametrize("std", [0.02, 0.15])
def test_embed_parity_small(prec, tol, std):
    """C=256, 42x56 images (12 patches, 17 tokens), 2 blocks, scenes of 2, 1
    and 2 frames, chunks of 2 frames (chunks straddle scene boundaries)."""
    m, scenes = SMALL, [2, 1, 2]
    img, w = _problem(m, sum(scenes), (42, 56), 2, seed=21, bf16=prec != vg.F32, std=std)
    ref = oracle.embed(img, w, m.heads, m.ln_eps, scene_frames=scenes)
    h = _handle(m, chunk=2)
    offs = np.concatenate([[0], np.cumsum(scenes)]).tolist()
    print(f"embed small prec={prec} std={std} scenes={scenes}", flush=True)
    out = vg.embed(h.h, to_dev(img, torch.float32), _embed_to_dev(w, _dt(prec)), prec, frame_offsets=offs)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    e = max_abs_rel(got[:, 5:], ref[:, 5:])
    print(f"  patch tokens max_abs_rel={e:.3e}")
    assert got.shape == ref.shape
    assert e < tol
    _check_special(got, w, scenes)
    h.close()


def test_embed_results_do_not_depend_on_chunk():
    m, scenes = SMALL, [3, 2]
    img, w = _problem(m, 5, (28, 42), 1, seed=22, bf16=True)
    wd = _embed_to_dev(w, torch.bfloat16)
    imgd = to_dev(img, torch.float32)
    outs = []
    for chunk in (1, 2, 5):
        h = _handle(m, chunk=chunk)
        outs.append(vg.embed(h.h, imgd, wd, vg.BF16, frame_offsets=[0, 3, 5]).clone())
        h.close()
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])


def test_embed_depth0_and_fp8_runs_as_bf16():
    """No blocks: patch embedding and final LayerNorm only; VGGTX_FP8_E4M3 gives
    the VGGTX_BF16 result bitwise (no global attention in the front end)."""
    m = SMALL
    img, w = _problem(m, 2, (14, 28), 0, seed=23, bf16=True)
    ref = oracle.embed(img, w, m.heads, m.ln_eps)
    h = _handle(m)
    wd = _embed_to_dev(w, torch.bfloat16)
    a = vg.embed(h.h, to_dev(img, torch.float32), wd, vg.BF16)
    b = vg.embed(h.h, to_dev(img, torch.float32), wd, vg.FP8_E4M3)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    e = max_abs_rel(a.cpu().numpy()[:, 5:], ref[:, 5:])
    print(f"embed depth 0 max_abs_rel={e:.3e}")
    assert e < 2e-2
    h.close()


def test_embed_dino_l_shape_sampled_frame():
    """ViT-L/14 shape at 518 x 518 (1369 patches, 1374 tokens, C=1024, 16 heads,
    F=4096, 24 blocks), 3 frames in one scene, BF16; the oracle recomputes
    frame 1 in full (the front end is per frame), the special rows of all."""
    m = synth.ModelConfig()
    img, w = _problem(m, 3, (518, 518), 24, seed=24, bf16=True)
    h = _handle(m)
    print("embed DINO-L 518x518 S=3 depth=24 bf16", flush=True)
    out = vg.embed(h.h, to_dev(img, torch.float32), _embed_to_dev(w, torch.bfloat16), vg.BF16)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert got.shape == (3, 1374, 1024)
    ref = oracle.embed(img, w, m.heads, m.ln_eps, frames=[1])
    e = max_abs_rel(got[1, 5:], ref[0, 5:])
    print(f"  frame 1 patch tokens max_abs_rel={e:.3e}")
    assert e < 2e-2
    _check_special(got, w, [3])
    h.close()


def test_embed_rejected_calls_write_nothing():
    m = SMALL
    img, w = _problem(m, 2, (28, 28), 1, seed=25, bf16=True)
    h = _handle(m)
    wd = _embed_to_dev(w, torch.bfloat16)
    imgd = to_dev(img, torch.float32)
    out = torch.full((2, 9, m.dim), 5.0, device=DEV)
    with pytest.raises(vg.VggtxError) as e:  # 30 is not a multiple of 14
        vg.embed(h.h, to_dev(np.zeros((2, 3, 28, 30), np.float32), torch.float32), wd, vg.BF16, out=out)
    assert e.value.status == E_INVALID
    small = torch.empty(1024, dtype=torch.uint8, device=DEV)
    with pytest.raises(vg.VggtxError) as e:
        vg.embed(h.h, imgd, wd, vg.BF16, out=out, ws=small)
    assert e.value.status == E_WORKSPACE
    with pytest.raises(vg.VggtxError) as e:  # offsets must start at 0
        vg.embed(h.h, imgd, wd, vg.BF16, frame_offsets=[1, 2], out=out)
    assert e.value.status == E_INVALID
    torch.cuda.synchronize()
    assert bool((out == 5.0).all())
    h.close()


@pytest.mark.parametrize("prec,tol", [(vg.F32, 1e-4), (vg.BF16, 2e-2)])
def test_images_to_features_pipeline(prec, tol):
    """Front end then aggregator (one layer pair), two scenes: the library's
    features against oracle.aggregate(oracle.embed(...))."""
    m, scenes = SMALL, [2, 2]
    img, w = _problem(m, 4, (28, 42), 1, seed=26, bf16=prec != vg.F32)
    rng = np.random.default_rng(27)
    layers = synth.gen_weights(rng, m, bf16=prec != vg.F32)
    tok_ref = oracle.embed(img, w, m.heads, m.ln_eps, scene_frames=scenes)
    ref = oracle.aggregate(tok_ref, layers, [0], m.heads, m.ln_eps, scene_frames=scenes)
    h = _handle(m, chunk=3)
    offs = [0, 2, 4]
    tok = vg.embed(h.h, to_dev(img, torch.float32), _embed_to_dev(w, _dt(prec)), prec, frame_offsets=offs)
    out = vg.aggregate_varlen(h.h, tok, offs, weights_to_dev(layers, _dt(prec)), [0], prec, out_dtype=vg.OUT_F32)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    C = m.dim
    ef = max_abs_rel(got[0, :, :, :C], ref[0, :, :, :C])
    eg = max_abs_rel(got[0, :, :, C:], ref[0, :, :, C:])
    print(f"pipeline prec={prec}: frame half {ef:.3e}, global half {eg:.3e}")
    assert ef < tol and eg < tol
    h.close()


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_pack_head_inputs_bit_exact(dtype):
    """Head inputs of the kept layers (patch tokens as channels-first maps)
    equal the oracle's layout change element for element; one case at the
    VGGT-L shape (37 x 37 patches, 2C = 2048) and one ragged small case."""
    from oracle import heads
    for (n_out, S, gh, gw, C) in ((4, 3, 37, 37, 1024), (2, 5, 3, 7, 256)):
        P = 5 + gh * gw
        rng = np.random.default_rng(gh)
        f = rng.normal(0, 1, (n_out, S, P, 2 * C)).astype(np.float32)
        if dtype == torch.bfloat16:
            f = synth.round_bf16(f)
        h = vg.Handle(0, dim=C, heads=C // 64, mlp_hidden=4 * C)
        got = vg.pack_head_inputs(h.h, to_dev(f, dtype), gh, gw)
        torch.cuda.synchronize()
        ref = heads.pack_head_inputs(f, gh, gw)
        assert np.array_equal(got.float().cpu().numpy(), ref)
        h.close()


def test_pack_head_inputs_rejects_misaligned_features():
    """The packing reads 16-byte granules: a feature pointer off a 16-byte
    boundary is refused before any launch and the output is left alone."""
    C, gh, gw = 256, 3, 7
    P = 5 + gh * gw
    h = vg.Handle(0, dim=C, heads=C // 64, mlp_hidden=4 * C)
    base = torch.zeros(2 * P * 2 * C + 8, dtype=torch.bfloat16, device=DEV)
    feats = base[1:1 + 2 * P * 2 * C].view(1, 2, P, 2 * C)  # 2 bytes past an aligned start
    out = torch.full((1, 2, 2 * C, gh, gw), 7.0, dtype=torch.bfloat16, device=DEV)
    with pytest.raises(vg.VggtxError) as e:
        vg.pack_head_inputs(h.h, feats, gh, gw, out=out)
    assert e.value.status == E_INVALID
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
    h.close()
