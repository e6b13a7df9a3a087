"""CPU pins of the kernel-consistency diagnostic (tests/fp8_stream_emulation.py):
the float64 emulation of the FP8 kernel's tile-by-tile probability placement
with headroom and overflow fallback."""
import numpy as np

import oracle
import synth
from fp8_stream_emulation import attention_fp8_streamed


def _rising(n, step_binades, H=1, D=64, seed=5):
    """Queries along one direction u (norm 8); key tile j (64 keys) at
    step * j binades of base-2 logit, plus small noise."""
    rng = np.random.default_rng(seed)
    u = rng.normal(0, 1, (H, 1, D))
    u /= np.linalg.norm(u, axis=-1, keepdims=True)
    q = 8.0 * u + rng.normal(0, 0.02, (H, n, D))
    tile = (np.arange(n) // 64)[None, :, None]
    k = (step_binades * np.log(2.0)) * tile * u + rng.normal(0, 0.02, (H, n, D))
    v = rng.normal(0, 1, (H, n, D))
    return q, k, v


def test_single_tile_equals_the_two_pass_emulation():
    """One (partial) key tile: the first tile places the row maximum two
    binades below 448 instead of at 448, a power-of-two shift that E4M3
    rounding commutes with while the probabilities stay normal numbers."""
    rng = np.random.default_rng(3)
    q, k, v = (rng.normal(0, s, (2, 50, 64)) for s in (0.5, 0.5, 1.0))
    got, fb = attention_fp8_streamed(q, k, v)
    ref = oracle.attention_fp8_emulated(q, k, v)
    assert fb == 0
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-14)


def test_constant_v_survives_rescales():
    """A constant value row comes back exactly (the output is a convex
    combination of value rows) across many tiles, fallbacks and rescales;
    a rescale applied to the output but not to the row sum would break it."""
    q, k, _ = _rising(700, 3.0)
    rng = np.random.default_rng(8)
    row = synth.round_bf16(rng.normal(0, 1, 64).astype(np.float32)).astype(np.float64)
    v = np.broadcast_to(row, q.shape).copy()
    got, fb = attention_fp8_streamed(q, k, v)
    assert fb > 0
    st = np.arange(0, 700, 128)
    c, s = oracle.quantize_rows(v[0], st, np.minimum(st + 128, 700))
    deq = oracle.e4m3_decode(c[0]) * s[0]
    np.testing.assert_allclose(got, np.broadcast_to(deq, got.shape), rtol=0, atol=1e-12)


def test_rising_keys_fall_back_on_every_full_tile():
    """Keys rising 3 binades per tile overflow the two-binade headroom on
    every full tile after the first, in every 32-row group: 900 keys give 14
    full tiles and a partial one (which always takes the exact step), 900
    queries give 29 groups, so 29 * 13 fallbacks.  The result stays within
    one E4M3 step of the two-pass emulation (the two round each probability
    against a different offset, so single probabilities may differ by a step,
    and here four top keys carry a third of the weight)."""
    q, k, v = _rising(900, 3.0)
    got, fb = attention_fp8_streamed(q, k, v)
    assert fb == 29 * 13
    ref = oracle.attention_fp8_emulated(q, k, v)
    assert np.abs(got - ref).max() / np.abs(ref).max() < 0.0625
    # more headroom than the rise: no fallback at all
    _, fb_wide = attention_fp8_streamed(q, k, v, headroom=40.0)
    assert fb_wide == 0


def test_slow_rise_falls_back_on_about_every_other_tile():
    """1.2 binades per tile: a placed maximum at 448/4 absorbs one rise
    (2^1.2 < 4.14) and overflows on the second."""
    q, k, v = _rising(64 * 21, 1.2)
    _, fb = attention_fp8_streamed(q, k, v)
    groups, full_after_first = 64 * 21 // 32, 20
    assert fb == groups * (full_after_first // 2)
