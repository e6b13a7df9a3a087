"""Plain float64 definition of the alternating-attention aggregator.

Paper anchors (arXiv 2509.25191):
  * Sec. 3.2: VGGT = per-frame patch embedding -> 24 alternating-attention (AA)
    layers, each a frame-wise attention block (attention restricted to the P
    tokens of one frame) and a global attention block (attention over the
    tokens of all frames) -> heads.  Only the outputs of layers 4, 11, 17 and 23
    feed the heads; the others are discarded ("VGGT-").
  * Sec. 3.2: frame-wise work is intra-frame, so frames may be processed in
    sequential chunks without changing the result ("VGGT--", chunk 128, Sec. 4.1).

Readings where the paper is silent (the block internals are not described):
  * Block = pre-LayerNorm transformer block: x += MHA(LN1(x)); x += MLP(LN2(x)),
    MLP = Linear(C, F) -> exact-erf GELU -> Linear(F, C); biases on every Linear;
    LN with biased variance and eps from the config (1e-6 by default).
  * QKV projection output is packed [q | k | v], each C wide; head h uses
    columns h*D ... h*D+D-1 of each part; attention scale 1/sqrt(D).
  * Within a layer the frame block runs first, then the global block; layers
    are indexed from 0 (23 = last).
  * The "output feature" of layer l is [frame_out_l | global_out_l] (2C wide).
  * No positional encoding, q/k normalisation or layer-scale (not mentioned).
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
from scipy.special import erf

Bounds = List[Tuple[int, int]]
_ROW_BLOCK = 512


def layer_norm(x: np.ndarray, g: np.ndarray, b: np.ndarray, eps: float) -> np.ndarray:
    """(x - mean) / sqrt(var + eps) * g + b over the last axis, biased variance."""
    x = np.asarray(x, dtype=np.float64)
    mu = x.mean(axis=-1, keepdims=True)
    var = ((x - mu) ** 2).mean(axis=-1, keepdims=True)
    return (x - mu) / np.sqrt(var + eps) * np.asarray(g, np.float64) + np.asarray(b, np.float64)


def gelu(u: np.ndarray) -> np.ndarray:
    """GELU(u) = u * Phi(u) with the exact Gaussian CDF Phi(u) = (1 + erf(u/sqrt 2)) / 2."""
    u = np.asarray(u, dtype=np.float64)
    return 0.5 * u * (1.0 + erf(u / math.sqrt(2.0)))


def linear(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y = x W^T + b with W stored [out, in] (row-major)."""
    return np.asarray(x, np.float64) @ np.asarray(w, np.float64).T + np.asarray(b, np.float64)


def split_heads(t: np.ndarray, H: int) -> np.ndarray:
    """[n, C] -> [H, n, D]; head h takes columns h*D ... h*D+D-1."""
    n, C = t.shape
    return t.reshape(n, H, C // H).transpose(1, 0, 2)


def merge_heads(t: np.ndarray) -> np.ndarray:
    """[H, n, D] -> [n, H*D]."""
    H, n, D = t.shape
    return t.transpose(1, 0, 2).reshape(n, H * D)


def softmax_rows(s: np.ndarray) -> np.ndarray:
    """Exact two-pass softmax along the last axis: subtract the row max, exponentiate, normalise."""
    m = s.max(axis=-1, keepdims=True)
    e = np.exp(s - m)
    return e / e.sum(axis=-1, keepdims=True)


def attention_probs(q: np.ndarray, k: np.ndarray) -> np.ndarray:
    """Full probability matrix softmax(q k^T / sqrt(D)) for small inputs: [H, nq, nk]."""
    q = np.asarray(q, np.float64); k = np.asarray(k, np.float64)
    D = q.shape[-1]
    return softmax_rows(q @ np.swapaxes(k, -1, -2) / math.sqrt(D))


def attention(q: np.ndarray, k: np.ndarray, v: np.ndarray) -> np.ndarray:
    """softmax(q k^T / sqrt(D)) v per head.  q [H, nq, D], k and v [H, nk, D].

    Query rows are taken a block at a time only to bound memory; every row is
    the exact definition (its own full score row, two-pass softmax)."""
    q = np.asarray(q, np.float64); k = np.asarray(k, np.float64); v = np.asarray(v, np.float64)
    H, nq, D = q.shape
    out = np.empty((H, nq, v.shape[-1]), dtype=np.float64)
    scale = 1.0 / math.sqrt(D)
    for h in range(H):
        kt = k[h].T
        for r0 in range(0, nq, _ROW_BLOCK):
            s = (q[h, r0:r0 + _ROW_BLOCK] @ kt) * scale
            out[h, r0:r0 + _ROW_BLOCK] = softmax_rows(s) @ v[h]
    return out


def _mlp(x1: np.ndarray, w: Dict[str, np.ndarray], eps: float) -> np.ndarray:
    h2 = layer_norm(x1, w["ln2_g"], w["ln2_b"], eps)
    return x1 + linear(gelu(linear(h2, w["w_fc1"], w["b_fc1"])), w["w_fc2"], w["b_fc2"])


def block(x: np.ndarray, w: Dict[str, np.ndarray], seqs: Bounds, H: int, eps: float) -> np.ndarray:
    """One pre-LN transformer block over rows x [n, C]; attention is restricted
    to each half-open row range in ``seqs`` (frames for the frame block,
    scenes for the global block)."""
    x = np.asarray(x, np.float64)
    C = x.shape[1]
    h = layer_norm(x, w["ln1_g"], w["ln1_b"], eps)
    qkv = linear(h, w["w_qkv"], w["b_qkv"])
    attn = np.empty_like(x)
    for (a, e) in seqs:
        q = split_heads(qkv[a:e, :C], H)
        k = split_heads(qkv[a:e, C:2 * C], H)
        v = split_heads(qkv[a:e, 2 * C:], H)
        attn[a:e] = merge_heads(attention(q, k, v))
    x1 = x + linear(attn, w["w_o"], w["b_o"])
    return _mlp(x1, w, eps)


def frame_bounds(S: int, P: int, first: int = 0) -> Bounds:
    return [(first + f * P, first + (f + 1) * P) for f in range(S)]


def scene_bounds(scene_frames: Sequence[int], P: int) -> Bounds:
    out, a = [], 0
    for s in scene_frames:
        out.append((a, a + s * P)); a += s * P
    return out


def aggregate(tokens: np.ndarray, weights: List[Dict[str, Dict[str, np.ndarray]]],
              out_layers: Sequence[int], H: int, eps: float = 1e-6,
              scene_frames: Optional[Sequence[int]] = None) -> np.ndarray:
    """Aggregator forward.  tokens [S, P, C]; weights[l] = {"frame": ..., "global": ...}.

    Returns [len(out_layers), S, P, 2C] holding [frame_out_l | global_out_l] for
    each requested layer (0-based), nothing else is kept (Sec. 3.2).
    ``scene_frames`` splits the S frames into independent scenes (global
    attention restricted to each scene); default: one scene."""
    S, P, C = tokens.shape
    scenes = list(scene_frames) if scene_frames is not None else [S]
    assert sum(scenes) == S
    x = np.asarray(tokens, np.float64).reshape(S * P, C)
    fr = frame_bounds(S, P)
    sc = scene_bounds(scenes, P)
    want = {l: i for i, l in enumerate(out_layers)}
    out = np.empty((len(out_layers), S, P, 2 * C), dtype=np.float64)
    for l, wl in enumerate(weights):
        if l > max(out_layers):
            break
        x = block(x, wl["frame"], fr, H, eps)
        if l in want:
            out[want[l], :, :, :C] = x.reshape(S, P, C)
        x = block(x, wl["global"], sc, H, eps)
        if l in want:
            out[want[l], :, :, C:] = x.reshape(S, P, C)
    return out


# --------------------------------------------------------------------------
# teacher-forced checks for sizes where a full float64 forward is too slow
# --------------------------------------------------------------------------

def global_block_rows(x_scene: np.ndarray, w: Dict[str, np.ndarray], rows: Sequence[int],
                      H: int, eps: float) -> np.ndarray:
    """Global-block output for the selected rows of one scene, given the block
    input x_scene [n, C] for every row of the scene (keys and values need all
    of them).  Equals ``block(x_scene, w, [(0, n)], H, eps)[rows]``."""
    x = np.asarray(x_scene, np.float64)
    C = x.shape[1]
    rows = np.asarray(rows, dtype=np.int64)
    h = layer_norm(x, w["ln1_g"], w["ln1_b"], eps)
    wqkv = np.asarray(w["w_qkv"], np.float64); bqkv = np.asarray(w["b_qkv"], np.float64)
    k = split_heads(h @ wqkv[C:2 * C].T + bqkv[C:2 * C], H)
    v = split_heads(h @ wqkv[2 * C:].T + bqkv[2 * C:], H)
    q = split_heads(h[rows] @ wqkv[:C].T + bqkv[:C], H)
    attn = merge_heads(attention(q, k, v))
    x1 = x[rows] + linear(attn, w["w_o"], w["b_o"])
    return _mlp(x1, w, eps)


def frame_block_frames(x: np.ndarray, w: Dict[str, np.ndarray], frames: Sequence[int], P: int,
                       H: int, eps: float) -> np.ndarray:
    """Frame-block output for the selected frames only: [len(frames), P, C]."""
    x = np.asarray(x, np.float64)
    outs = [block(x[f * P:(f + 1) * P], w, [(0, P)], H, eps) for f in frames]
    return np.stack(outs)
