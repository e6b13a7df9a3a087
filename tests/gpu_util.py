"""Helpers shared by the GPU parity tests (no aggregator arithmetic here)."""
import numpy as np
import torch

import synth

DEV = "cuda:0"


def max_abs_rel(got, ref) -> float:
    """max |g - r| / max |r| (the parity metric of every float comparison)."""
    got = np.asarray(got, np.float64); ref = np.asarray(ref, np.float64)
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV).to(dtype)


def weights_to_dev(layers, dtype):
    return [{part: {k: to_dev(v, dtype) for k, v in blk.items()} for part, blk in l.items()} for l in layers]


def head_major_to_tokens(a):
    """[H, N, D] -> [N, H, D] (contiguous)."""
    return np.ascontiguousarray(np.transpose(a, (1, 0, 2)))
