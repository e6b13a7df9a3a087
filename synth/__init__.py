"""Seeded synthetic inputs shared by the FP64 oracle and the GPU library's tests.

This module holds no arithmetic of the aggregator: it only draws random numbers
and converts storage formats (round-to-nearest-even into bfloat16).  Both the
oracle and the HIP path receive exactly the arrays produced here.

Recipe (stands in for the MipNeRF360 / Tanks-and-Temples / CO3Dv2 scenes the
paper evaluates on, which are not available; their sequence lengths of up to
311 / 1106 / 202 frames motivate the frame counts used):

* tokens: float32 N(0, 1), shape [S, P, C]; P = 5 special tokens + (img/14)^2
  patch tokens (86 for a 126-pixel image, 1374 for a 518-pixel image).
* every Linear weight and bias: N(0, 0.02); LayerNorm gamma = 1 + N(0, 0.02),
  beta = N(0, 0.02).
* draw order: tokens first, then for every layer the frame block and then the
  global block, each block's parameters in the order of ``BLOCK_FIELDS``.
* bf16 configurations draw in float64, round to bfloat16 (RNE) and hand the
  rounded values to both sides, so the input rounding is not counted as error.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

BLOCK_FIELDS = (
    "ln1_g", "ln1_b", "w_qkv", "b_qkv", "w_o", "b_o",
    "ln2_g", "ln2_b", "w_fc1", "b_fc1", "w_fc2", "b_fc2",
)


@dataclasses.dataclass(frozen=True)
class ModelConfig:
    dim: int = 1024
    heads: int = 16
    head_dim: int = 64
    mlp_hidden: int = 4096
    depth: int = 24
    ln_eps: float = 1e-6
    frame_chunk: int = 128


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    model: ModelConfig
    frames: int                      # S (total over scenes for varlen)
    tokens_per_frame: int            # P
    out_layers: tuple
    prec: str                        # "f32" | "bf16" | "fp8"
    scene_frames: Optional[tuple] = None   # varlen: frames per scene


def varlen_scene_frames(seed: int = 0, n_scenes: int = 12, lo: int = 16, hi: int = 300) -> tuple:
    """Frame counts of the batched multi-scene workload: uniform on [lo, hi]."""
    return tuple(int(v) for v in np.random.default_rng(seed).integers(lo, hi + 1, size=n_scenes))


def workloads() -> Dict[str, Workload]:
    big = ModelConfig()
    small = ModelConfig(dim=256, heads=4, head_dim=64, mlp_hidden=1024, depth=1)
    full_out = (4, 11, 17, 23)
    return {
        "pair_s8_c256": Workload("pair_s8_c256", small, 8, 86, (0,), "f32"),
        "vggt_l_s32": Workload("vggt_l_s32", big, 32, 1374, full_out, "bf16"),
        "vggt_l_s200": Workload("vggt_l_s200", big, 200, 1374, full_out, "bf16"),
        "vggt_l_s1000": Workload("vggt_l_s1000", big, 1000, 1374, full_out, "fp8"),
        "vggt_l_varlen12": Workload("vggt_l_varlen12", big, sum(varlen_scene_frames()), 1374,
                                    full_out, "bf16", varlen_scene_frames()),
    }


def round_bf16(a: np.ndarray) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even); returns float32
    arrays holding exactly representable bf16 values.  NaN stays NaN."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    nan = np.isnan(f)
    if nan.any():
        out = out.copy()
        out[nan] = np.nan
    return out.reshape(np.shape(a))


def bf16_bits(a: np.ndarray) -> np.ndarray:
    """uint16 bit patterns of float32 values that are already bf16-representable."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def gen_tokens(rng: np.random.Generator, S: int, P: int, C: int) -> np.ndarray:
    return rng.standard_normal((S, P, C), dtype=np.float32)


def gen_block(rng: np.random.Generator, C: int, F: int, std: float = 0.02,
              bf16: bool = False) -> Dict[str, np.ndarray]:
    shapes = {
        "ln1_g": (C,), "ln1_b": (C,), "w_qkv": (3 * C, C), "b_qkv": (3 * C,),
        "w_o": (C, C), "b_o": (C,), "ln2_g": (C,), "ln2_b": (C,),
        "w_fc1": (F, C), "b_fc1": (F,), "w_fc2": (C, F), "b_fc2": (C,),
    }
    out = {}
    for name in BLOCK_FIELDS:
        v = rng.normal(0.0, std, size=shapes[name])
        if name in ("ln1_g", "ln2_g"):
            v = v + 1.0
        v = v.astype(np.float32)
        out[name] = round_bf16(v) if bf16 else v
    return out


def gen_weights(rng: np.random.Generator, model: ModelConfig, bf16: bool) -> List[Dict[str, Dict[str, np.ndarray]]]:
    """List over layers of {"frame": block, "global": block}."""
    layers = []
    for _ in range(model.depth):
        fr = gen_block(rng, model.dim, model.mlp_hidden, bf16=bf16)
        gl = gen_block(rng, model.dim, model.mlp_hidden, bf16=bf16)
        layers.append({"frame": fr, "global": gl})
    return layers


def gen_problem(model: ModelConfig, S: int, P: int, seed: int = 0, bf16: bool = False):
    """Tokens [S,P,C] float32 and weights for ``model.depth`` layers, drawn in order."""
    rng = np.random.default_rng(seed)
    tokens = gen_tokens(rng, S, P, model.dim)
    weights = gen_weights(rng, model, bf16)
    return tokens, weights


# --------------------------------------------------------------------------
# attention-only inputs (three logit regimes)
# --------------------------------------------------------------------------

def gen_qkv(rng: np.random.Generator, H: int, N: int, D: int, regime: str = "R0",
            frames: int = 1, bf16: bool = True):
    """Q, K, V as float32 arrays [H, N, D] (bf16-representable when ``bf16``).

    R0: element std 0.64 (logit std about 0.4, the random-init regime).
    R1: element std 0.64 * sqrt(3 / 0.41)  (logit std about 3).
    R2: peaked, multi-view-like: each token is a shared scene-point embedding
        (the same point appears once in every frame) plus small noise, and
        K = Q up to noise, so matched logits are large (about 20) against a
        competitor spread of a few units.
    """
    if regime == "R0":
        q = rng.normal(0, 0.64, (H, N, D)); k = rng.normal(0, 0.64, (H, N, D))
    elif regime == "R1":
        s = 0.64 * np.sqrt(3.0 / 0.41)
        q = rng.normal(0, s, (H, N, D)); k = rng.normal(0, s, (H, N, D))
    elif regime == "R2":
        per_frame = max(1, N // max(frames, 1))
        pts = rng.normal(0, 1.0, (H, per_frame, D))
        idx = np.arange(N) % per_frame
        base = pts[:, idx, :] * 2.6
        q = base + rng.normal(0, 0.3, (H, N, D))
        k = base + rng.normal(0, 0.3, (H, N, D))
    else:
        raise ValueError(regime)
    v = rng.normal(0, 1.0, (H, N, D))
    q, k, v = (a.astype(np.float32) for a in (q, k, v))
    if bf16:
        q, k, v = round_bf16(q), round_bf16(k), round_bf16(v)
    return q, k, v


def sample_rows(seed: int, n_rows: int, n_sample: int, P: int, extra: Sequence[int] = ()) -> np.ndarray:
    """Seeded query-row sample: forced rows (0, last, the special tokens 0..4 of
    one frame, a row in the last partial 128-row block) plus uniform draws."""
    rng = np.random.default_rng(seed + 1)
    forced = {0, n_rows - 1}
    f = int(rng.integers(0, max(1, n_rows // P)))
    forced.update(min(n_rows - 1, f * P + t) for t in range(5))
    tail_start = (n_rows // 128) * 128
    if tail_start < n_rows:
        forced.add(int(rng.integers(tail_start, n_rows)))
    forced.update(int(e) for e in extra if 0 <= e < n_rows)
    forced = sorted(forced)
    need = max(0, n_sample - len(forced))
    pool = np.setdiff1d(np.arange(n_rows), forced)
    draw = rng.choice(pool, size=min(need, len(pool)), replace=False) if need else np.array([], int)
    return np.sort(np.concatenate([np.array(forced, dtype=np.int64), draw.astype(np.int64)]))


# --------------------------------------------------------------------------
# patch-embedding front end (images -> aggregator input tokens)
# --------------------------------------------------------------------------

EMBED_PATCH = 14      # patch side in pixels
EMBED_SPECIAL = 5     # 1 class / camera token + 4 register tokens per frame


def gen_images(rng: np.random.Generator, S: int, height: int, width: int) -> np.ndarray:
    """Normalised images, float32 N(0, 1), shape [S, 3, height, width]."""
    return rng.standard_normal((S, 3, height, width), dtype=np.float32)


def gen_embed(rng: np.random.Generator, model: ModelConfig, height: int, width: int, depth: int,
              std: float = 0.02, bf16: bool = False) -> Dict[str, object]:
    """Front-end parameters, drawn in this order: w_patch [C, 3*14*14] (the
    Conv2d weight [C, 3, 14, 14] flattened), b_patch [C], pos [1 + n_patches, C],
    cls [C], reg [4, C], then ``depth`` blocks (``gen_block``), norm_g, norm_b
    [C], cam [2, C], agg_reg [2, 4, C].  All N(0, std) except norm_g = 1 + N(0, std)."""
    C = model.dim
    n_patch = (height // EMBED_PATCH) * (width // EMBED_PATCH)
    def draw(shape, one=False):
        v = rng.normal(0.0, std, size=shape) + (1.0 if one else 0.0)
        v = v.astype(np.float32)
        return round_bf16(v) if bf16 else v
    w: Dict[str, object] = {}
    w["w_patch"] = draw((C, 3 * EMBED_PATCH * EMBED_PATCH))
    w["b_patch"] = draw((C,))
    w["pos"] = draw((1 + n_patch, C))
    w["cls"] = draw((C,))
    w["reg"] = draw((EMBED_SPECIAL - 1, C))
    w["blocks"] = [gen_block(rng, C, model.mlp_hidden, std=std, bf16=bf16) for _ in range(depth)]
    w["norm_g"] = draw((C,), one=True)
    w["norm_b"] = draw((C,))
    w["cam"] = draw((2, C))
    w["agg_reg"] = draw((2, EMBED_SPECIAL - 1, C))
    return w


# --------------------------------------------------------------------------
# global alignment: cameras and correspondences
# --------------------------------------------------------------------------

def _look_at_origin(C: np.ndarray) -> np.ndarray:
    """World-to-camera rotation whose optical axis (third row) points from C to the origin."""
    z = -C / np.linalg.norm(C)
    x = np.cross(np.array([0.0, 1.0, 0.0]), z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    return np.stack([x, y, z])


def _small_rotation(v: np.ndarray) -> np.ndarray:
    """Rotation by the axis-angle vector v (Rodrigues)."""
    a = float(np.linalg.norm(v))
    if a == 0.0:
        return np.eye(3)
    k = v / a
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + math.sin(a) * K + (1 - math.cos(a)) * (K @ K)


def gen_ga_cameras(rng: np.random.Generator, n_cams: int, arc_deg: float = 360.0, radius: float = 4.0,
                   focal: float = 500.0, size: int = 518, rot_noise_deg: float = 1.0, trans_noise: float = 0.05,
                   focal_noise: float = 0.02):
    """True cameras on a horizontal arc of `arc_deg` degrees (radius `radius`,
    small random height), all looking at the origin, focal `focal`, principal
    point at the image centre; and the predicted (initial) cameras: the true
    ones with a random rotation of std rot_noise_deg per axis, centre noise of
    std trans_noise and relative focal noise of std focal_noise.  Returns two
    dicts with R [N,3,3], t [N,3], f [N], c [N,2] (float64)."""
    yaw = np.radians(np.linspace(0.0, arc_deg, n_cams, endpoint=arc_deg < 360.0))
    height = rng.normal(0.0, 0.3, n_cams)
    true = {"R": np.empty((n_cams, 3, 3)), "t": np.empty((n_cams, 3)), "f": np.full(n_cams, float(focal)),
            "c": np.full((n_cams, 2), size / 2.0)}
    init = {"R": np.empty((n_cams, 3, 3)), "t": np.empty((n_cams, 3)), "f": np.empty(n_cams),
            "c": np.full((n_cams, 2), size / 2.0)}
    for n in range(n_cams):
        C = np.array([radius * math.sin(yaw[n]), height[n], -radius * math.cos(yaw[n])])
        R = _look_at_origin(C)
        true["R"][n], true["t"][n] = R, -R @ C
        Ri = _small_rotation(rng.normal(0.0, math.radians(rot_noise_deg), 3)) @ R
        Ci = C + rng.normal(0.0, trans_noise, 3)
        init["R"][n], init["t"][n] = Ri, -Ri @ Ci
        init["f"][n] = focal * (1.0 + rng.normal(0.0, focal_noise))
    return true, init


def gen_ga_corr(rng: np.random.Generator, cams: Dict[str, np.ndarray], pairs: np.ndarray, per_pair,
                noise_px: float = 0.5, outlier_frac: float = 0.2, size: int = 518, spread: float = 0.7):
    """Correspondences of the pairs: scene points N(0, spread^2) per axis
    projected into both true cameras, pixel noise of std noise_px, and a
    fraction outlier_frac whose second point is replaced by a uniform random
    pixel.  per_pair: int or a sequence with one count per pair.  Returns
    (corr float32 [K, 4] = (u, v, u', v'), offsets int64 [n_pairs + 1])."""
    counts = np.full(len(pairs), per_pair) if np.isscalar(per_pair) else np.asarray(per_pair)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    corr = np.empty((offsets[-1], 4), np.float32)
    R, t, f, c = cams["R"], cams["t"], cams["f"], cams["c"]
    for m, (i, j) in enumerate(pairs):
        n = int(counts[m])
        X = rng.normal(0.0, spread, (n, 3))
        uv = []
        for cam in (i, j):
            Xc = X @ R[cam].T + t[cam]
            uv.append(np.stack([f[cam] * Xc[:, 0] / Xc[:, 2] + c[cam, 0], f[cam] * Xc[:, 1] / Xc[:, 2] + c[cam, 1]], 1))
        a = np.concatenate(uv, 1) + rng.normal(0.0, noise_px, (n, 4))
        bad = rng.random(n) < outlier_frac
        a[bad, 2:] = rng.uniform(0.0, size, (int(bad.sum()), 2))
        corr[offsets[m]:offsets[m + 1]] = a
    return corr, offsets
