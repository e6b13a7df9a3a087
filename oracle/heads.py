"""Plain definition of the prediction-head input packing (arXiv 2509.25191,
Sec. 3.2: the dense-prediction heads consume the outputs of layers 4, 11, 17
and 23).

Reading (the heads are not described beyond that): for every kept layer and
frame, the head input is the feature map of the patch tokens, channels first:
out[l, s, c, y, x] = feats[l, s, 5 + y * gw + x, c] for the 2C channels of
the layer's [frame | global] feature, dropping the 5 special tokens (camera
and registers), with the patch grid gh x gw in row-major token order."""
from __future__ import annotations

import numpy as np

N_SPECIAL = 5


def pack_head_inputs(feats: np.ndarray, gh: int, gw: int) -> np.ndarray:
    """feats [n_out, S, P, 2C] with P = 5 + gh * gw -> [n_out, S, 2C, gh, gw]."""
    n_out, S, P, C2 = feats.shape
    assert P == N_SPECIAL + gh * gw
    return np.ascontiguousarray(feats[:, :, N_SPECIAL:, :].reshape(n_out, S, gh, gw, C2).transpose(0, 1, 4, 2, 3))
