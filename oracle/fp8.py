"""OCP FP8 E4M3 (the "E4M3FN" encoding) and per-row-block quantisation.

The paper runs in bfloat16 (Sec. 3.2); the FP8 global-attention variant is an
extension of the library.  Its quantiser reading:
  * format: OCP 8-bit floating point, E4M3: 1 sign, 4 exponent (bias 7) and
    3 mantissa bits; exponent field 0 encodes subnormals m/8 * 2^-6; the codes
    S.1111.111 are NaN; the largest finite magnitude is 1.75 * 2^8 = 448; no
    infinities.
  * encode: round to nearest, ties to even mantissa, saturate to +-448.
  * block scale over a block of rows: s = amax / 448 (s = 1 when amax = 0),
    codes = encode(x * (448 / amax)), all in float32 arithmetic.
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0


def e4m3_decode(codes: np.ndarray) -> np.ndarray:
    """Decode uint8 E4M3 codes to float64 following the OCP definition."""
    c = np.asarray(codes, dtype=np.uint8).astype(np.int64)
    sign = np.where(c & 0x80, -1.0, 1.0)
    e = (c >> 3) & 0xF
    m = c & 0x7
    val = np.where(e == 0, m / 8.0 * 2.0 ** -6, (1.0 + m / 8.0) * np.exp2(e - 7.0))
    val = sign * val
    return np.where((e == 15) & (m == 7), np.nan, val)


def e4m3_encode(x: np.ndarray) -> np.ndarray:
    """Encode float values as E4M3 codes: round to nearest even, saturate at 448.

    For |x| in binade [2^e, 2^(e+1)) (e >= -6) the spacing of representable
    values is 2^(e-3); below 2^-6 (subnormals) it is 2^-9.  The magnitude is
    divided by that spacing, rounded half-to-even (exact: power-of-two scaling),
    and re-assembled into exponent and mantissa fields."""
    x = np.asarray(x, dtype=np.float64)
    if np.isnan(x).any():
        raise ValueError("NaN has no defined E4M3 encoding in this library")
    neg = np.signbit(x)
    a = np.abs(x)
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    e = np.clip(e, -6, 8)
    # guard against log2 rounding at exact binade edges
    e = np.where(a >= np.exp2(e + 1), e + 1, e)
    e = np.where((a < np.exp2(e)) & (e > -6), e - 1, e)
    e = np.clip(e, -6, 8)
    step = np.exp2(e - 3)
    k = np.rint(a / step)                      # half-to-even
    mag = k * step                             # rounded magnitude (may reach next binade)
    mag = np.minimum(mag, E4M3_MAX)            # saturate
    # re-derive fields from the rounded magnitude
    with np.errstate(divide="ignore"):
        e2 = np.floor(np.log2(np.where(mag > 0, mag, 1.0)))
    e2 = np.where(mag >= np.exp2(e2 + 1), e2 + 1, e2)
    sub = mag < 2.0 ** -6
    exp_field = np.where(sub, 0, e2 + 7).astype(np.int64)
    man_field = np.where(sub, np.rint(mag / 2.0 ** -9), np.rint((mag / np.exp2(e2) - 1.0) * 8)).astype(np.int64)
    code = (exp_field << 3) | man_field
    code = np.where(mag == 0, 0, code)
    code = code | np.where(neg, 0x80, 0)
    return code.astype(np.uint8)


def quantize_rows(x: np.ndarray, block_starts: np.ndarray, block_ends: np.ndarray):
    """Quantise rows of x [rows, D] in row blocks [start_i, end_i).

    Returns (codes [rows, D] uint8, scales [n_blocks] float32) with
    s_i = amax_i / 448 and codes = encode(x * (448 / amax_i)) in float32."""
    x32 = np.asarray(x, dtype=np.float32)
    codes = np.zeros(x32.shape, dtype=np.uint8)
    scales = np.ones(len(block_starts), dtype=np.float32)
    for i, (a, e) in enumerate(zip(block_starts, block_ends)):
        blk = x32[a:e]
        amax = np.float32(np.abs(blk).max()) if blk.size else np.float32(0)
        if amax == 0:
            codes[a:e] = e4m3_encode(blk.astype(np.float64))
            scales[i] = np.float32(1.0)
            continue
        inv = np.float32(np.float32(E4M3_MAX) / amax)
        scales[i] = np.float32(amax / np.float32(E4M3_MAX))
        codes[a:e] = e4m3_encode((blk * inv).astype(np.float32).astype(np.float64))
    return codes, scales


def attention_fp8_emulated(q: np.ndarray, k: np.ndarray, v: np.ndarray, block: int = 128) -> np.ndarray:
    """What FP8 E4M3 global attention computes, emulated in float64 for one
    sequence: q, k, v [H, n, D] are quantised per (head, 128-row block)
    (``quantize_rows``); logits use the dequantised Q and K; the V block scale
    is folded into the probabilities, A_j = p_j * 448 * s_v(b_j) / max_b s_v,
    which are rounded to E4M3; the output is sum_j A_j V8_j / sum_j A_j / r_j
    times max_b s_v / 448 (the row sum taken from the rounded A).  The
    softmax here uses the final row maximum (two-pass); a streamed kernel
    rounds against its running maximum instead, so the two differ by
    rounding only.  Used to tell the error of the format from kernel error."""
    q = np.asarray(q, np.float64); k = np.asarray(k, np.float64); v = np.asarray(v, np.float64)
    H, n, D = q.shape
    starts = np.arange(0, n, block); ends = np.minimum(starts + block, n)
    rows = ends - starts
    out = np.empty((H, n, D))
    for h in range(H):
        qc, qs = quantize_rows(q[h], starts, ends)
        kc, ks = quantize_rows(k[h], starts, ends)
        vc, vs = quantize_rows(v[h], starts, ends)
        qd = e4m3_decode(qc) * np.repeat(qs, rows)[:, None]
        kd = e4m3_decode(kc) * np.repeat(ks, rows)[:, None]
        v8 = e4m3_decode(vc)
        s = qd @ kd.T / np.sqrt(D)
        p = np.exp(s - s.max(axis=1, keepdims=True))
        vmax = vs.astype(np.float64).max()
        r = E4M3_MAX * np.repeat(vs, rows).astype(np.float64) / vmax
        a = e4m3_decode(e4m3_encode(p * r[None, :]))
        out[h] = (a @ v8) * (vmax / E4M3_MAX) / (a / r[None, :]).sum(axis=1, keepdims=True)
    return out
