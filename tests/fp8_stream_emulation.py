"""Kernel-consistency diagnostic for the FP8 global attention (test code, not
part of the oracle).

A float64 emulation of the FP8 kernel's own tile-by-tile probability
placement: it follows the kernel's 32-row query groups, 64-key tiles, two
binades of placement headroom and the overflow fallback, so it shares the
kernel's design choices and cannot vouch for them.  The accuracy gates of
the FP8 path compare with the float64 definition (``oracle.attention``) or
the two-pass format emulation (``oracle.attention_fp8_emulated``); this
module only serves a printed diagnostic of how closely the kernel follows
its stated placement rule, and its own CPU pins.
"""
import numpy as np

from oracle.fp8 import E4M3_MAX, e4m3_decode, e4m3_encode, logit_factor, quantize_rows

E4M3_NAN_ABOVE = 464.0  # the hardware conversion rounds (448, 464] to 448 and larger values to NaN


def attention_fp8_streamed(q: np.ndarray, k: np.ndarray, v: np.ndarray, block: int = 128, tile: int = 64,
                           group: int = 32, headroom: float = 2.0):
    """The streamed FP8 global attention's arithmetic, emulated in float64 for
    one sequence (reading of the FP8 variant; the paper fixes no FP8 kernel):
    Q, K, V quantised as in ``attention_fp8_emulated``; per group of 32 query
    rows (starting at the sequence start) the keys are visited in tiles of
    64.  Each row keeps an offset m: probabilities are E4M3(2^(t - m + log2
    448)).  The first tile and the partial last tile take the exact step; any
    other tile first tries the current m and takes the exact step only when
    some row of the group would exceed 464 before rounding (the hardware turns
    that into the E4M3 NaN code).  The exact step finds each row's tile
    maximum x (in units of the current offset); on the first tile every row,
    later only rows with x > log2 448, move m so that their maximum lands
    ``headroom`` binades below 448, and the running sum and output are
    rescaled by 2^(old m - new m).  Returns (output [H, n, D], number of
    (head, group, tile) steps that fell back to the exact step after a
    failed try)."""
    q = np.asarray(q, np.float64); k = np.asarray(k, np.float64); v = np.asarray(v, np.float64)
    H, n, D = q.shape
    starts = np.arange(0, n, block); ends = np.minimum(starts + block, n)
    rows = ends - starts
    c2 = logit_factor(D)
    L = np.log2(E4M3_MAX)
    place = L - headroom
    out = np.empty((H, n, D))
    fallbacks = 0
    for h in range(H):
        qc, qs = quantize_rows(q[h], starts, ends, pre=c2)
        kc, ks = quantize_rows(k[h], starts, ends)
        vc, vs = quantize_rows(v[h], starts, ends)
        qd = e4m3_decode(qc) * np.repeat(qs, rows)[:, None]
        kd = e4m3_decode(kc) * np.repeat(ks, rows)[:, None]
        vd = e4m3_decode(vc) * np.repeat(vs, rows)[:, None]
        t = qd @ kd.T  # base-2 logits
        for r0 in range(0, n, group):
            tr = t[r0:r0 + group]
            R = tr.shape[0]
            m = np.full(R, L)  # offset: x = t + (log2 448 - m)
            l = np.zeros(R)
            o = np.zeros((R, D))
            for j0 in range(0, n, tile):
                x = tr[:, j0:j0 + tile] + (L - m)[:, None]
                first = j0 == 0
                exact = first or j0 + tile > n
                if not exact and (np.exp2(x) > E4M3_NAN_ABOVE).any():
                    exact = True
                    fallbacks += 1
                if exact:
                    xmax = x.max(axis=1)
                    if first or (xmax > L).any():
                        delta = xmax - place if first else np.where(xmax > L, xmax - place, 0.0)
                        alpha = np.zeros(R) if first else np.exp2(-delta)
                        l *= alpha
                        o *= alpha[:, None]
                        m += delta
                        x = x - delta[:, None]
                p = e4m3_decode(e4m3_encode(np.exp2(x)))  # saturating: (448, 464] -> 448
                l += p.sum(axis=1)
                o += p @ vd[j0:j0 + tile]
            out[h, r0:r0 + R] = o / l[:, None]
    return out, fallbacks
