"""Pins of the front-end oracle (per-frame patch embedding, Sec. 3.2) against
library routines, brute force and the invariants of its definition."""
import numpy as np
import torch

import oracle
import synth


def _rng(seed):
    return np.random.default_rng(seed)


def _torch_layer(w, C, H, F, eps):
    layer = torch.nn.TransformerEncoderLayer(
        d_model=C, nhead=H, dim_feedforward=F, dropout=0.0, activation="gelu",
        layer_norm_eps=eps, batch_first=True, norm_first=True, dtype=torch.float64)
    sd = {
        "self_attn.in_proj_weight": w["w_qkv"], "self_attn.in_proj_bias": w["b_qkv"],
        "self_attn.out_proj.weight": w["w_o"], "self_attn.out_proj.bias": w["b_o"],
        "linear1.weight": w["w_fc1"], "linear1.bias": w["b_fc1"],
        "linear2.weight": w["w_fc2"], "linear2.bias": w["b_fc2"],
        "norm1.weight": w["ln1_g"], "norm1.bias": w["ln1_b"],
        "norm2.weight": w["ln2_g"], "norm2.bias": w["ln2_b"],
    }
    layer.load_state_dict({k: torch.from_numpy(np.asarray(v, np.float64)) for k, v in sd.items()})
    return layer.eval()


def _t(a):
    return torch.from_numpy(np.asarray(a, np.float64))


def test_patch_embedding_is_a_stride_14_conv2d():
    """patchify + linear == Conv2d(3, C, kernel 14, stride 14) (torch, float64),
    output channels read out row-major over the patch grid."""
    rng = _rng(1)
    C = 24
    img = rng.normal(0, 1, (2, 3, 42, 56))
    w = rng.normal(0, 1, (C, 3 * 14 * 14)); b = rng.normal(0, 1, C)
    ours = oracle.linear(oracle.patchify(img), w, b)
    ref = torch.nn.functional.conv2d(_t(img), _t(w).reshape(C, 3, 14, 14), _t(b), stride=14)
    ref = ref.reshape(2, C, -1).permute(0, 2, 1).numpy()
    assert ours.shape == (2, 12, C)
    np.testing.assert_allclose(ours, ref, rtol=0, atol=1e-11)


def test_patchify_brute_force():
    rng = _rng(2)
    img = rng.normal(0, 1, (1, 3, 28, 42))
    pt = oracle.patchify(img)
    for py in range(2):
        for px in range(3):
            for c in range(3):
                for ky in range(14):
                    for kx in range(14):
                        assert pt[0, py * 3 + px, c * 196 + ky * 14 + kx] == img[0, c, py * 14 + ky, px * 14 + kx]


def _small(depth, seed=3, hw=(28, 42)):
    m = synth.ModelConfig(dim=64, heads=2, head_dim=32, mlp_hidden=128, depth=depth)
    rng = _rng(seed)
    img = synth.gen_images(rng, 3, *hw)
    w = synth.gen_embed(rng, m, hw[0], hw[1], depth, std=0.2)
    return m, img, w


def test_depth0_front_end_closed_form():
    """Without blocks: patch rows = LayerNorm(conv(img) + pos), special rows are
    the camera / register tokens (first-frame set for frame 0 only)."""
    m, img, w = _small(0)
    out = oracle.embed(img, w, m.heads, m.ln_eps)
    C = m.dim
    conv = torch.nn.functional.conv2d(_t(img), _t(w["w_patch"]).reshape(C, 3, 14, 14), _t(w["b_patch"]), stride=14)
    z = conv.reshape(3, C, -1).permute(0, 2, 1) + _t(w["pos"])[1:]
    ref = torch.nn.functional.layer_norm(z, (C,), _t(w["norm_g"]), _t(w["norm_b"]), eps=m.ln_eps).numpy()
    assert out.shape == (3, 5 + 6, C)
    np.testing.assert_allclose(out[:, 5:], ref, rtol=0, atol=1e-11)
    for f in range(3):
        s = 0 if f == 0 else 1
        np.testing.assert_array_equal(out[f, 0], w["cam"][s])
        np.testing.assert_array_equal(out[f, 1:5], w["agg_reg"][s])


def test_front_end_matches_torch_vit():
    """Two pre-LN encoder layers of torch over [cls + pos0, registers, patches +
    pos], then torch layer_norm: the patch rows of the oracle's output."""
    m, img, w = _small(2)
    out = oracle.embed(img, w, m.heads, m.ln_eps)
    C = m.dim
    conv = torch.nn.functional.conv2d(_t(img), _t(w["w_patch"]).reshape(C, 3, 14, 14), _t(w["b_patch"]), stride=14)
    z = conv.reshape(3, C, -1).permute(0, 2, 1) + _t(w["pos"])[1:]
    cls = (_t(w["cls"]) + _t(w["pos"])[0]).expand(3, 1, C)
    x = torch.cat([cls, _t(w["reg"]).expand(3, 4, C), z], dim=1)
    with torch.no_grad():
        for bw in w["blocks"]:
            x = _torch_layer(bw, C, m.heads, m.mlp_hidden, m.ln_eps)(x)
        ref = torch.nn.functional.layer_norm(x, (C,), _t(w["norm_g"]), _t(w["norm_b"]), eps=m.ln_eps).numpy()
    np.testing.assert_allclose(out[:, 5:], ref[:, 5:], rtol=0, atol=1e-10)


def test_front_end_is_per_frame():
    """Permuting the frames of a scene permutes the patch rows; the first-frame
    tokens follow the scene starts; a frame subset equals the full result's rows."""
    m, img, w = _small(1, seed=4)
    full = oracle.embed(img, w, m.heads, m.ln_eps, scene_frames=[2, 1])
    perm = [1, 0, 2]
    pe = oracle.embed(img[perm], w, m.heads, m.ln_eps, scene_frames=[2, 1])
    np.testing.assert_array_equal(pe[:, 5:], full[perm, 5:])
    for f, s in zip(range(3), (0, 1, 0)):
        np.testing.assert_array_equal(full[f, 0], w["cam"][s])
        np.testing.assert_array_equal(full[f, 1:5], w["agg_reg"][s])
    sub = oracle.embed(img, w, m.heads, m.ln_eps, scene_frames=[2, 1], frames=[2, 1])
    np.testing.assert_array_equal(sub, full[[2, 1]])
