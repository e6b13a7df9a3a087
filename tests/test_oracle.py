"""Pins of the FP64 oracle against things other than itself: closed forms,
library routines (torch float64 on the CPU), brute force on tiny inputs and the
invariants the paper states for the memory-efficient aggregator (Sec. 3.2)."""
import math
import os

import numpy as np
import pytest
import torch

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed=0):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------- attention

def test_attention_closed_form_example():
    vals = {}
    for line in open(os.path.join(GOLDEN, "attention_closed_form.txt")):
        if line.startswith("#") or not line.strip():
            continue
        key, *nums = line.split()
        vals[key] = np.array([float(v) for v in nums])
    q = vals["q"][None, None, :]
    k = np.stack([vals["k0"], vals["k1"]])[None]
    v = np.stack([vals["v0"], vals["v1"]])[None]
    p = oracle.attention_probs(q, k)
    assert abs(p[0, 0, 0] - vals["p0"][0]) < 1e-15
    o = oracle.attention(q, k, v)
    np.testing.assert_allclose(o[0, 0], vals["o"], rtol=0, atol=1e-15)


def _naive_attention(q, k, v):
    """Triple loops with math.exp: the definition written out element by element."""
    H, nq, D = q.shape
    nk = k.shape[1]
    out = np.zeros((H, nq, v.shape[2]))
    for h in range(H):
        for i in range(nq):
            s = [sum(q[h, i, d] * k[h, j, d] for d in range(D)) / math.sqrt(D) for j in range(nk)]
            m = max(s)
            e = [math.exp(x - m) for x in s]
            z = sum(e)
            for c in range(v.shape[2]):
                out[h, i, c] = sum(e[j] / z * v[h, j, c] for j in range(nk))
    return out


def test_attention_brute_force_tiny():
    rng = _rng(1)
    q, k, v = (rng.normal(0, 1.5, (2, 6, 4)) for _ in range(3))
    np.testing.assert_allclose(oracle.attention(q, k, v), _naive_attention(q, k, v), rtol=0, atol=1e-12)


def test_attention_matches_torch_sdpa_float64():
    rng = _rng(2)
    q, k, v = (rng.normal(0, 2.0, (3, 700, 64)) for _ in range(3))
    ref = torch.nn.functional.scaled_dot_product_attention(
        torch.from_numpy(q)[None], torch.from_numpy(k)[None], torch.from_numpy(v)[None])[0].numpy()
    np.testing.assert_allclose(oracle.attention(q, k, v), ref, rtol=0, atol=1e-12)


def test_softmax_rows_sum_to_one_and_nonnegative():
    rng = _rng(3)
    q, k = rng.normal(0, 4, (2, 50, 16)), rng.normal(0, 4, (2, 80, 16))
    p = oracle.attention_probs(q, k)
    assert (p >= 0).all()
    np.testing.assert_allclose(p.sum(-1), 1.0, rtol=0, atol=1e-14)


def test_constant_values_give_that_row():
    rng = _rng(4)
    q, k = rng.normal(0, 3, (2, 40, 8)), rng.normal(0, 3, (2, 90, 8))
    row = rng.normal(0, 1, 8)
    v = np.broadcast_to(row, (2, 90, 8))
    o = oracle.attention(q, k, v)
    np.testing.assert_allclose(o, np.broadcast_to(row, o.shape), rtol=0, atol=1e-14)


def test_identical_keys_give_mean_of_values():
    rng = _rng(5)
    q = rng.normal(0, 3, (1, 10, 8))
    k = np.broadcast_to(rng.normal(0, 1, 8), (1, 30, 8))
    v = rng.normal(0, 1, (1, 30, 8))
    o = oracle.attention(q, k, v)
    np.testing.assert_allclose(o[0], np.broadcast_to(v[0].mean(0), (10, 8)), rtol=0, atol=1e-14)


def _streamed_attention(q, k, v, bn):
    """Online softmax over key tiles (running max m, running sum l, rescaled
    accumulator), written independently of the oracle to pin the identity the
    streamed GPU kernels rely on: it must equal the two-pass definition."""
    H, nq, D = q.shape
    out = np.zeros_like(q)
    for h in range(H):
        m = np.full(nq, -np.inf); l = np.zeros(nq); acc = np.zeros((nq, D))
        for j0 in range(0, k.shape[1], bn):
            s = q[h] @ k[h, j0:j0 + bn].T / math.sqrt(D)
            m_new = np.maximum(m, s.max(1))
            a = np.exp(m - m_new)
            p = np.exp(s - m_new[:, None])
            l = l * a + p.sum(1)
            acc = acc * a[:, None] + p @ v[h, j0:j0 + bn]
            m = m_new
        out[h] = acc / l[:, None]
    return out


@pytest.mark.parametrize("bn", [1, 7, 64, 1000])
def test_online_softmax_equals_two_pass(bn):
    rng = _rng(6)
    q, k, v = rng.normal(0, 2, (2, 33, 16)), rng.normal(0, 2, (2, 301, 16)), rng.normal(0, 1, (2, 301, 16))
    np.testing.assert_allclose(_streamed_attention(q, k, v, bn), oracle.attention(q, k, v), rtol=0, atol=1e-13)


# ---------------------------------------------------------------- LN / GELU / linear

def test_layer_norm_constant_row_gives_beta():
    g = np.linspace(0.5, 1.5, 32); b = np.linspace(-1, 1, 32)
    x = np.full((3, 32), 7.25)
    np.testing.assert_allclose(oracle.layer_norm(x, g, b, 1e-6), np.broadcast_to(b, (3, 32)), rtol=0, atol=1e-15)


@pytest.mark.parametrize("eps", [1e-6, 1e-5])
def test_layer_norm_matches_torch(eps):
    rng = _rng(7)
    x = rng.normal(0.3, 2.0, (50, 256)); g = rng.normal(1, 0.1, 256); b = rng.normal(0, 0.1, 256)
    ref = torch.nn.functional.layer_norm(torch.from_numpy(x), (256,), torch.from_numpy(g), torch.from_numpy(b), eps)
    np.testing.assert_allclose(oracle.layer_norm(x, g, b, eps), ref.numpy(), rtol=0, atol=1e-12)


def test_gelu_exact_erf():
    assert oracle.gelu(np.array([0.0]))[0] == 0.0
    u = np.linspace(-8, 8, 2001)
    ref = torch.nn.functional.gelu(torch.from_numpy(u)).numpy()
    np.testing.assert_allclose(oracle.gelu(u), ref, rtol=0, atol=1e-15)
    big = np.array([12.0, 30.0]); np.testing.assert_allclose(oracle.gelu(big), big, rtol=1e-15)
    assert abs(oracle.gelu(np.array([-30.0]))[0]) < 1e-100
    # GELU(1) = Phi(1) = 0.8413447460685429 (standard normal CDF at 1)
    assert abs(oracle.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15


def test_linear_matches_torch():
    rng = _rng(8)
    x, w, b = rng.normal(0, 1, (20, 64)), rng.normal(0, 1, (96, 64)), rng.normal(0, 1, 96)
    ref = torch.nn.functional.linear(torch.from_numpy(x), torch.from_numpy(w), torch.from_numpy(b)).numpy()
    np.testing.assert_allclose(oracle.linear(x, w, b), ref, rtol=0, atol=1e-12)


# ---------------------------------------------------------------- whole block

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


def test_block_matches_torch_pre_ln_encoder_layer():
    """torch.nn.TransformerEncoderLayer(norm_first=True, activation='gelu') is the
    same pre-LN block; it pins the q|k|v packing, the head split, LN and GELU."""
    C, H, F, P, eps = 128, 2, 512, 37, 1e-6
    rng = _rng(9)
    w = synth.gen_block(rng, C, F, std=0.2)
    x = rng.normal(0, 1, (3 * P, C))
    ours = oracle.block(x, w, oracle.frame_bounds(3, P), H, eps)
    layer = _torch_layer(w, C, H, F, eps)
    with torch.no_grad():
        ref = layer(torch.from_numpy(x).reshape(3, P, C)).reshape(3 * P, C).numpy()
    np.testing.assert_allclose(ours, ref, rtol=0, atol=1e-11)


# ---------------------------------------------------------------- invariants

def _tiny_model(depth=2):
    return synth.ModelConfig(dim=64, heads=2, head_dim=32, mlp_hidden=128, depth=depth)


def test_global_equals_frame_when_one_frame():
    m = _tiny_model(1)
    tokens, w = synth.gen_problem(m, 1, 19, seed=3)
    x = tokens.reshape(19, 64)
    a = oracle.block(x, w[0]["global"], oracle.scene_bounds([1], 19), m.heads, m.ln_eps)
    b = oracle.block(x, w[0]["global"], oracle.frame_bounds(1, 19), m.heads, m.ln_eps)
    np.testing.assert_array_equal(a, b)


def test_global_block_is_frame_permutation_equivariant():
    m = _tiny_model(1)
    S, P = 5, 11
    tokens, w = synth.gen_problem(m, S, P, seed=4)
    perm = np.array([3, 0, 4, 2, 1])
    x = tokens.reshape(S * P, 64)
    xp = tokens[perm].reshape(S * P, 64)
    y = oracle.block(x, w[0]["global"], [(0, S * P)], m.heads, m.ln_eps).reshape(S, P, 64)
    yp = oracle.block(xp, w[0]["global"], [(0, S * P)], m.heads, m.ln_eps).reshape(S, P, 64)
    np.testing.assert_allclose(yp, y[perm], rtol=0, atol=1e-12)


def test_frame_block_is_intra_frame():
    m = _tiny_model(1)
    S, P = 4, 9
    tokens, w = synth.gen_problem(m, S, P, seed=5)
    t2 = tokens.copy(); t2[2] += 1.0
    a = oracle.block(tokens.reshape(-1, 64), w[0]["frame"], oracle.frame_bounds(S, P), m.heads, m.ln_eps).reshape(S, P, 64)
    b = oracle.block(t2.reshape(-1, 64), w[0]["frame"], oracle.frame_bounds(S, P), m.heads, m.ln_eps).reshape(S, P, 64)
    np.testing.assert_array_equal(a[[0, 1, 3]], b[[0, 1, 3]])
    assert np.abs(a[2] - b[2]).max() > 1e-3


def test_out_layer_subset_is_slice_of_all():
    m = _tiny_model(3)
    tokens, w = synth.gen_problem(m, 3, 7, seed=6)
    full = oracle.aggregate(tokens, w, [0, 1, 2], m.heads, m.ln_eps)
    sub = oracle.aggregate(tokens, w, [1], m.heads, m.ln_eps)
    np.testing.assert_array_equal(sub[0], full[1])


def test_varlen_equals_each_scene_alone():
    m = _tiny_model(2)
    P = 6
    scenes = [2, 3, 1]
    tokens, w = synth.gen_problem(m, sum(scenes), P, seed=7)
    both = oracle.aggregate(tokens, w, [0, 1], m.heads, m.ln_eps, scene_frames=scenes)
    f0 = 0
    for s in scenes:
        alone = oracle.aggregate(tokens[f0:f0 + s], w, [0, 1], m.heads, m.ln_eps)
        np.testing.assert_allclose(both[:, f0:f0 + s], alone, rtol=0, atol=1e-13)
        f0 += s


def test_teacher_forced_rows_equal_full_block():
    m = _tiny_model(1)
    S, P = 3, 13
    tokens, w = synth.gen_problem(m, S, P, seed=8)
    x = tokens.reshape(S * P, 64)
    full = oracle.block(x, w[0]["global"], [(0, S * P)], m.heads, m.ln_eps)
    rows = [0, 5, 17, 38]
    np.testing.assert_allclose(oracle.global_block_rows(x, w[0]["global"], rows, m.heads, m.ln_eps),
                               full[rows], rtol=0, atol=1e-13)
    ff = oracle.block(x, w[0]["frame"], oracle.frame_bounds(S, P), m.heads, m.ln_eps).reshape(S, P, 64)
    np.testing.assert_allclose(oracle.frame_block_frames(x, w[0]["frame"], [2, 0], P, m.heads, m.ln_eps),
                               ff[[2, 0]], rtol=0, atol=1e-13)


def test_aggregate_small_matches_torch_layers():
    """Whole aggregate of the one-pair small workload against torch encoder
    layers applied per frame and then over all frames."""
    m = synth.ModelConfig(dim=256, heads=4, head_dim=64, mlp_hidden=1024, depth=1)
    S, P = 8, 86
    tokens, w = synth.gen_problem(m, S, P, seed=0)
    out = oracle.aggregate(tokens, w, [0], m.heads, m.ln_eps)
    fl = _torch_layer(w[0]["frame"], 256, 4, 1024, m.ln_eps)
    gl = _torch_layer(w[0]["global"], 256, 4, 1024, m.ln_eps)
    with torch.no_grad():
        x = torch.from_numpy(tokens.astype(np.float64))
        fo = fl(x)
        go = gl(fo.reshape(1, S * P, 256)).reshape(S, P, 256)
    np.testing.assert_allclose(out[0, :, :, :256], fo.numpy(), rtol=0, atol=1e-11)
    np.testing.assert_allclose(out[0, :, :, 256:], go.numpy(), rtol=0, atol=1e-11)


# ---------------------------------------------------------------- FP8 E4M3

def test_e4m3_golden_codes():
    for line in open(os.path.join(GOLDEN, "e4m3_codes.txt")):
        if line.startswith("#") or not line.strip():
            continue
        c, v = line.split()
        code = int(c, 16)
        got = oracle.e4m3_decode(np.array([code], np.uint8))[0]
        assert got == float(v) and np.signbit(got) == v.startswith("-"), (c, got, v)
        if code not in (0x80,):
            assert oracle.e4m3_encode(np.array([float(v)]))[0] == code


def test_e4m3_decode_all_codes_match_torch():
    codes = np.arange(256, dtype=np.uint8)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    ours = oracle.e4m3_decode(codes)
    assert np.array_equal(np.isnan(ours), np.isnan(ref))
    ok = ~np.isnan(ref)
    np.testing.assert_array_equal(ours[ok], ref[ok])
    assert np.isnan(ours).sum() == 2 and np.nanmax(ours) == 448.0


def test_e4m3_encode_roundtrip_and_matches_torch_in_range():
    codes = np.array([c for c in range(256) if (c & 0x7F) != 0x7F], dtype=np.uint8)
    vals = oracle.e4m3_decode(codes)
    enc = oracle.e4m3_encode(vals)
    # -0 and +0 both decode to zero; everything else round-trips exactly
    np.testing.assert_array_equal(enc[codes != 0x80], codes[codes != 0x80])
    rng = _rng(10)
    x = np.concatenate([rng.uniform(-448, 448, 5000), rng.normal(0, 1, 5000), rng.normal(0, 0.01, 2000),
                        vals, (vals[:-1] + vals[1:]) / 2])  # includes exact midpoints (ties)
    x = x[np.abs(x) <= 448]
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    ours = oracle.e4m3_encode(x)
    same = (ours == ref) | ((ours & 0x7F) == 0) & ((ref & 0x7F) == 0)
    assert same.all(), x[~same][:10]


def test_e4m3_ties_to_even_and_saturation():
    enc = lambda v: int(oracle.e4m3_encode(np.array([v]))[0])
    assert enc(1.0625) == 0x38          # tie between 1.0 (even) and 1.125
    assert enc(1.1875) == 0x3A          # tie between 1.125 and 1.25 (even)
    assert enc(464.0) == 0x7E and enc(1e9) == 0x7E and enc(-1e9) == 0xFE
    assert enc(2.0 ** -10) == 0x00      # tie between 0 (even) and 2^-9
    assert enc(3 * 2.0 ** -10) == 0x02  # tie between 2^-9 and 2^-8 (even)


def test_quantize_rows_scale_and_error_bound():
    rng = _rng(11)
    x = synth.round_bf16(rng.normal(0, 0.7, (300, 64)).astype(np.float32))
    x[130:140] *= 37.0  # a block with a larger amax
    starts = np.array([0, 128, 256]); ends = np.array([128, 256, 300])
    codes, scales = oracle.quantize_rows(x, starts, ends)
    for i, (a, e) in enumerate(zip(starts, ends)):
        amax = float(np.abs(x[a:e]).max())
        # the scale is the smallest power of two with amax <= 448 s
        ex = np.log2(float(scales[i]))
        assert ex == np.round(ex) and 224.0 * scales[i] < amax <= 448.0 * scales[i]
        # division by a power of two is exact: the codes are torch's own E4M3
        # conversion of x / s (independent implementation)
        ref = torch.from_numpy(x[a:e].astype(np.float64) / float(scales[i])).to(torch.float8_e4m3fn)
        np.testing.assert_array_equal(codes[a:e], ref.view(torch.uint8).numpy())
        deq = oracle.e4m3_decode(codes[a:e]) * scales[i]
        # relative rounding error of E4M3 normals is at most 2^-4 (3 mantissa bits, RNE)
        err = np.abs(deq - x[a:e])
        bound = np.maximum(np.abs(x[a:e]) * 2.0 ** -4, 2.0 ** -10 * scales[i]) * (1 + 1e-6)
        assert (err <= bound).all()
    z, s = oracle.quantize_rows(np.zeros((10, 4), np.float32), np.array([0]), np.array([10]))
    assert s[0] == 1.0 and (z == 0).all()
    # pre-multiplied input: the float32 product is what gets quantised
    c = oracle.logit_factor(64)
    assert abs(float(c) - np.log2(np.e) / 8) < 1e-8
    c1, s1 = oracle.quantize_rows(x, starts, ends, pre=c)
    c2, s2 = oracle.quantize_rows((x * np.float32(c)).astype(np.float32), starts, ends)
    np.testing.assert_array_equal(c1, c2)
    np.testing.assert_array_equal(s1, s2)


def test_block_exponent_edges():
    be = oracle.block_exponent
    assert be(448.0) == 0 and be(448.0 * 2.0 ** -3) == -3 and be(np.nextafter(np.float32(448), np.float32(1e9))) == 1
    assert be(224.0) == -1 and be(np.nextafter(np.float32(224), np.float32(1e9))) == 0
    assert be(1.0) == -8 and be(1.75) == -8 and be(np.nextafter(np.float32(1.75), np.float32(9))) == -7
    assert be(0.0) == 0
    assert be(1e-38) == -127            # clamped at the E8M0 minimum
    assert be(3e38) == 120              # 3e38 / 448 lies in (2^119, 2^120]


# ---------------------------------------------------------------- synth helpers

def test_round_bf16_matches_torch():
    rng = _rng(12)
    x = np.concatenate([rng.normal(0, 1, 10000), [1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 0.0, -0.0]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(synth.round_bf16(x), ref)


def test_sample_rows_forced_members():
    rows = synth.sample_rows(0, 10000, 256, 1374)
    assert len(rows) == 256 and rows[0] == 0 and rows[-1] == 9999 and len(set(rows.tolist())) == 256
    assert (rows >= (10000 // 128) * 128).any()


def test_fp8_emulation_constant_v_and_error_bound():
    rng = _rng(13)
    q, k = rng.normal(0, 0.7, (2, 300, 64)), rng.normal(0, 0.7, (2, 300, 64))
    row = synth.round_bf16(rng.normal(0, 1, 64).astype(np.float32)).astype(np.float64)
    # a constant V row quantises exactly only up to E4M3 rounding of each entry; the
    # output must equal the dequantised row (convex combination of identical rows)
    v = np.broadcast_to(row, (2, 300, 64)).copy()
    o = oracle.attention_fp8_emulated(q, k, v)
    st = np.array([0, 128, 256]); en = np.array([128, 256, 300])
    c, s = oracle.quantize_rows(v[0], st, en)
    deq = oracle.e4m3_decode(c[0]) * s[0]
    np.testing.assert_allclose(o, np.broadcast_to(deq, o.shape), rtol=0, atol=1e-12)
    # random operands: error against the exact definition stays within a few E4M3 half-ulps
    v = rng.normal(0, 1, (2, 300, 64))
    ref = oracle.attention(q, k, v)
    err = np.abs(oracle.attention_fp8_emulated(q, k, v) - ref).max() / np.abs(ref).max()
    assert 1e-3 < err < 0.1
