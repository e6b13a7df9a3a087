"""Plain float64 definition of the per-frame patch-embedding front end.

Paper anchor (arXiv 2509.25191, Sec. 3.2): the network starts with a per-frame
DINO-based patch-embedding extractor; like frame-wise attention it involves
only intra-frame computation, so frames can be processed in sequential chunks
without changing the result.

Readings where the paper is silent (it does not describe the extractor):
  * Patch embedding: non-overlapping 14 x 14 patches, a linear map of the 588
    pixel values (channel-major, then row, then column inside the patch, the
    flattening of a Conv2d weight [C, 3, 14, 14]) plus a bias; patches are
    numbered row-major over the patch grid.
  * DINO-style token sequence per frame: [class token, 4 register tokens,
    patch tokens]; a learned position embedding (row 0 for the class token,
    row 1 + i for patch i) is added to the class and patch tokens, the
    registers get none.
  * The ViT blocks are the pre-LN block of the aggregator (``block``), with
    attention over the tokens of one frame; a final LayerNorm follows.
  * Output (the aggregator input): per frame [camera token, 4 register tokens,
    the final-normalised patch tokens].  The camera and register tokens are
    learned, with one set for the first frame of each scene and one for the
    other frames.
"""
from __future__ import annotations

from typing import Dict, Optional, Sequence

import numpy as np

from .aggregator import block, layer_norm, linear

PATCH = 14
N_SPECIAL = 5  # class (camera) token + 4 registers


def patchify(images: np.ndarray, patch: int = PATCH) -> np.ndarray:
    """[S, 3, Hi, Wi] -> [S, n_patches, 3 * patch * patch]: patch (py, px) is
    row py * (Wi / patch) + px; inside a patch the value of channel c at pixel
    (ky, kx) is column c * patch^2 + ky * patch + kx."""
    x = np.asarray(images, np.float64)
    S, ch, Hi, Wi = x.shape
    assert Hi % patch == 0 and Wi % patch == 0, "image sides must be multiples of the patch size"
    gh, gw = Hi // patch, Wi // patch
    x = x.reshape(S, ch, gh, patch, gw, patch)
    return x.transpose(0, 2, 4, 1, 3, 5).reshape(S, gh * gw, ch * patch * patch)


def frame_tokens(patches: np.ndarray, w: Dict[str, object]) -> np.ndarray:
    """DINO input of one frame: [cls + pos_0, reg_1..4, W_patch x_i + b + pos_(1+i)]."""
    pos = np.asarray(w["pos"], np.float64)
    z = linear(patches, w["w_patch"], w["b_patch"]) + pos[1:]
    cls = np.asarray(w["cls"], np.float64)[None, :] + pos[:1]
    return np.concatenate([cls, np.asarray(w["reg"], np.float64), z], axis=0)


def embed(images: np.ndarray, w: Dict[str, object], H: int, eps: float = 1e-6,
          scene_frames: Optional[Sequence[int]] = None, frames: Optional[Sequence[int]] = None) -> np.ndarray:
    """Front end: images [S, 3, Hi, Wi] -> aggregator tokens [S, 5 + n_patches, C].

    ``scene_frames`` splits the S frames into scenes (the first frame of each
    gets the first-frame camera and register tokens); ``frames`` restricts the
    computation to those frame indices (the result then has len(frames) rows
    of frames, in that order)."""
    S = images.shape[0]
    scenes = list(scene_frames) if scene_frames is not None else [S]
    assert sum(scenes) == S
    firsts = set(np.concatenate([[0], np.cumsum(scenes)[:-1]]).astype(int).tolist())
    idx = list(range(S)) if frames is None else list(frames)
    pt = patchify(images[idx])
    cam = np.asarray(w["cam"], np.float64)
    agg_reg = np.asarray(w["agg_reg"], np.float64)
    outs = []
    for j, f in enumerate(idx):
        x = frame_tokens(pt[j], w)
        n = x.shape[0]
        for bw in w["blocks"]:
            x = block(x, bw, [(0, n)], H, eps)
        x = layer_norm(x, w["norm_g"], w["norm_b"], eps)
        s = 0 if f in firsts else 1
        outs.append(np.concatenate([cam[s][None, :], agg_reg[s], x[N_SPECIAL:]], axis=0))
    return np.stack(outs)
