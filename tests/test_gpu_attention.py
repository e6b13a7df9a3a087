"""Parity of the HIP attention kernels and the FP8 quantiser with the FP64 oracle.

Attention outputs are compared head by head, element by element, in three
logit regimes (random-init, logit std ~3, peaked multi-view-like)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import DEV, max_abs_rel, to_dev, head_major_to_tokens

vg = pytest.importorskip("paper_2509_25191_amd.vggtx")
pytestmark = pytest.mark.gpu

TOL = {vg.F32: 1e-4, vg.BF16: 2e-2, vg.FP8_E4M3: 6e-2, vg.FP8_PV: 6e-2}


@pytest.fixture(scope="module")
def handle():
    h = vg.Handle(0, dim=256, heads=4, mlp_hidden=1024)
    yield h.h
    h.close()


def _qkv(H, N, D, regime, seed, frames=1, bf16=True):
    rng = np.random.default_rng(seed)
    return synth.gen_qkv(rng, H, N, D, regime, frames=frames, bf16=bf16)


def _dev_tokens(a, prec):
    return to_dev(head_major_to_tokens(a), torch.float32 if prec == vg.F32 else torch.bfloat16)


def _oracle_seqs(q, k, v, offs, rows=None):
    out = np.zeros(q.shape)
    for a, b in zip(offs[:-1], offs[1:]):
        if b > a:
            out[:, a:b] = oracle.attention(q[:, a:b], k[:, a:b], v[:, a:b])
    return out


def _run_global(handle, q, k, v, offs, prec):
    H, N, D = q.shape
    qd, kd, vd = (_dev_tokens(a, prec) for a in (q, k, v))
    o = torch.zeros_like(qd)
    vg.attn_global(handle, qd, kd, vd, o, offs, prec)
    torch.cuda.synchronize()
    return o.float().cpu().numpy().transpose(1, 0, 2)


def _fp8_large_logits(got, ref, q, k, v, offs, what):
    """FP8 E4M3 Q and K at large logits.  The gate is the two-pass emulation
    of the format (E4M3 Q, K, V and probabilities, exact softmax): the kernel
    must stay within 6e-2 of it.  Against the float64 definition the result
    is only reported: E4M3 rounds Q and K to 3 mantissa bits, so at a logit
    std of about 3 the logits move by about 0.15 and the weights by about
    15%, more than the 6e-2 the FP8 path is held to (xfail when above it)."""
    emu = np.zeros(q.shape)
    for a, b in zip(offs[:-1], offs[1:]):
        if b > a:
            emu[:, a:b] = oracle.attention_fp8_emulated(q[:, a:b], k[:, a:b], v[:, a:b])
    e, e_emu, e_fmt = max_abs_rel(got, ref), max_abs_rel(got, emu), max_abs_rel(emu, ref)
    print(f"   FP8 {what}: vs definition {e:.3e}, vs two-pass E4M3 emulation {e_emu:.3e}, "
          f"format alone {e_fmt:.3e}")
    assert e_emu < TOL[vg.FP8_E4M3]
    if e >= TOL[vg.FP8_E4M3]:
        pytest.xfail(f"FP8 E4M3 Q/K, {what}: {e:.3e} against the float64 definition "
                     f"(the format alone gives {e_fmt:.3e}) exceeds 6e-2")


@pytest.mark.parametrize("prec", [vg.F32, vg.BF16, vg.FP8_E4M3])
@pytest.mark.parametrize("regime", ["R0", "R1", "R2"])
def test_attn_global_small(handle, prec, regime):
    H, S, P, D = 4, 8, 86, 64
    q, k, v = _qkv(H, S * P, D, regime, seed=1, frames=S, bf16=prec != vg.F32)
    got = _run_global(handle, q, k, v, [0, S * P], prec)
    ref = _oracle_seqs(q, k, v, [0, S * P])
    e = max_abs_rel(got, ref)
    print(f"attn_global prec={prec} regime={regime} max_abs_rel={e:.3e}")
    if prec == vg.FP8_E4M3 and regime != "R0":
        _fp8_large_logits(got, ref, q, k, v, [0, S * P], f"regime {regime}")
    assert e < TOL[prec]


@pytest.mark.parametrize("prec", [vg.F32, vg.BF16, vg.FP8_E4M3])
def test_attn_global_varlen_ragged(handle, prec):
    H, D = 4, 64
    offs = [0, 200, 201, 201, 718, 845]  # includes a 1-token and an empty sequence
    q, k, v = _qkv(H, offs[-1], D, "R1", seed=2, bf16=prec != vg.F32)
    got = _run_global(handle, q, k, v, offs, prec)
    ref = _oracle_seqs(q, k, v, offs)
    e = max_abs_rel(got, ref)
    print(f"varlen prec={prec} max_abs_rel={e:.3e}")
    if prec == vg.FP8_E4M3:
        _fp8_large_logits(got, ref, q, k, v, offs, "varlen, logit std 3")
    assert e < TOL[prec]


@pytest.mark.parametrize("prec", [vg.F32, vg.BF16, vg.FP8_E4M3])
def test_attn_global_single_key_tails(handle, prec):
    """Sequences of 64k + 1 tokens: the last key tile holds one valid key and
    the last query tile one valid row (waves with a single live query)."""
    H, D = 4, 64
    offs = [0, 65, 194, 387]
    q, k, v = _qkv(H, offs[-1], D, "R0", seed=10, bf16=prec != vg.F32)
    got = _run_global(handle, q, k, v, offs, prec)
    ref = _oracle_seqs(q, k, v, offs)
    e = max_abs_rel(got, ref)
    print(f"single-key tails prec={prec} max_abs_rel={e:.3e}")
    assert e < TOL[prec]


def _far_below_case():
    """Sequences whose first 128 keys point against every query (logits near
    -96, -138 in base 2) before ordinary keys follow."""
    H, D = 2, 64
    offs = [0, 300, 520]
    rng = np.random.default_rng(41)
    u = rng.normal(0, 1, (H, 1, D))
    u /= np.linalg.norm(u, axis=-1, keepdims=True)
    n = offs[-1]
    q = 16.0 * u + rng.normal(0, 0.05, (H, n, D))
    k = rng.normal(0, 0.1, (H, n, D))
    for a in offs[:-1]:
        k[:, a:a + 128] = -48.0 * u + rng.normal(0, 0.05, (H, 128, D))
    v = rng.normal(0, 1, (H, n, D))
    return q, k, v, offs


def _rising_case():
    """Keys that line up with the queries more and more: every 64-key tile
    raises the row maximum by 3 binades in one sequence and by 1.2 in the
    other."""
    H, D = 2, 64
    offs = [0, 900, 1500]
    rng = np.random.default_rng(43)
    u = rng.normal(0, 1, (H, 1, D))
    u /= np.linalg.norm(u, axis=-1, keepdims=True)
    n = offs[-1]
    q = 8.0 * u + rng.normal(0, 0.05, (H, n, D))
    k = np.empty((H, n, D))
    for (a, b), step in zip(zip(offs[:-1], offs[1:]), (3.0, 1.2)):
        tile = (np.arange(b - a) // 64)[None, :, None]
        # q.k / sqrt(D) = level in natural units, i.e. step * tile binades
        k[:, a:b] = (step * np.log(2.0)) * tile * u + rng.normal(0, 0.05, (H, b - a, D))
    v = rng.normal(0, 1, (H, n, D))
    return q, k, v, offs


@pytest.mark.parametrize("prec", [vg.F32, vg.BF16, vg.FP8_E4M3])
def test_attn_global_first_tile_far_below_max(handle, prec):
    """The first 128 keys of each sequence (two key tiles, one FP8 scale
    block) point against every query (logits near -96, i.e. -138 in base 2)
    and the later keys give ordinary logits: the first tiles' weights vanish
    against the row maximum found later, with no overflow in the streamed
    rescale on the way."""
    q, k, v, offs = _far_below_case()
    if prec != vg.F32:
        q, k, v = (synth.round_bf16(x.astype(np.float32)) for x in (q, k, v))
    got = _run_global(handle, q, k, v, offs, prec)
    ref = _oracle_seqs(q, k, v, offs)
    e = max_abs_rel(got, ref)
    print(f"first tile far below max prec={prec} max_abs_rel={e:.3e} finite={np.isfinite(got).all()}")
    assert np.isfinite(got).all() and e < TOL[prec]


def _e4m3_rounded(x, offs, pre=None):
    """x [H, n, D] as the FP8 path sees it: E4M3 codes times the power-of-two
    scale of their 128-row block (blocks start at every sequence start),
    quantised after multiplication by ``pre`` and divided by it again."""
    from oracle import fp8
    st = np.concatenate([np.arange(a, b, 128) for a, b in zip(offs[:-1], offs[1:])])
    en = np.concatenate([np.minimum(np.arange(a, b, 128) + 128, b) for a, b in zip(offs[:-1], offs[1:])])
    out = np.empty(x.shape)
    for h in range(x.shape[0]):
        codes, sc = fp8.quantize_rows(x[h], st, en, pre)
        for i, (a, b) in enumerate(zip(st, en)):
            out[h, a:b] = fp8.e4m3_decode(codes[a:b]) * np.float64(sc[i])
    return out / np.float64(pre) if pre is not None else out


@pytest.mark.parametrize("prec", [vg.F32, vg.BF16, vg.FP8_E4M3])
def test_attn_global_rising_maximum(handle, prec):
    """Keys that line up with the queries more and more, tile by tile: in one
    sequence every 64-key tile raises the row maximum by 3 binades (base-2
    logits), in the other by 1.2, so in FP8 every tile of the first and every
    other tile of the second overflow the probability placement and take the
    recompute-and-rescale path.  FP8 is compared with the oracle on the
    E4M3-rounded Q, K and V, so that only the rounding of the probabilities
    and the rescaling are measured."""
    q, k, v, offs = _rising_case()
    D = q.shape[-1]
    if prec != vg.F32:
        q, k, v = (synth.round_bf16(x.astype(np.float32)) for x in (q, k, v))
    got = _run_global(handle, q, k, v, offs, prec)
    if prec == vg.FP8_E4M3:
        from oracle import fp8
        q, k, v = _e4m3_rounded(q, offs, fp8.logit_factor(D)), _e4m3_rounded(k, offs), _e4m3_rounded(v, offs)
    ref = _oracle_seqs(q, k, v, offs)
    e = max_abs_rel(got, ref)
    print(f"rising maximum prec={prec} max_abs_rel={e:.3e}")
    assert np.isfinite(got).all() and e < TOL[prec]


@pytest.mark.parametrize("prec", [vg.F32, vg.BF16])
@pytest.mark.parametrize("S,P", [(8, 86), (3, 1374), (5, 1)])
def test_attn_frame(handle, prec, S, P):
    H, D = 4, 64
    q, k, v = _qkv(H, S * P, D, "R1", seed=3, bf16=prec != vg.F32)
    qd, kd, vd = (_dev_tokens(a, prec) for a in (q, k, v))
    o = torch.zeros_like(qd)
    vg.attn_frame(handle, qd, kd, vd, o, S, P, prec)
    torch.cuda.synchronize()
    got = o.float().cpu().numpy().transpose(1, 0, 2)
    ref = _oracle_seqs(q, k, v, [f * P for f in range(S + 1)])
    e = max_abs_rel(got, ref)
    print(f"attn_frame prec={prec} S={S} P={P} max_abs_rel={e:.3e}")
    assert e < TOL[prec]


@pytest.mark.parametrize("prec", [vg.F32, vg.BF16])
def test_global_equals_frame_for_one_frame(handle, prec):
    H, P, D = 4, 300, 64
    q, k, v = _qkv(H, P, D, "R1", seed=4, bf16=prec != vg.F32)
    qd, kd, vd = (_dev_tokens(a, prec) for a in (q, k, v))
    o1 = torch.zeros_like(qd); o2 = torch.zeros_like(qd)
    vg.attn_frame(handle, qd, kd, vd, o1, 1, P, prec)
    vg.attn_global(handle, qd, kd, vd, o2, [0, P], prec)
    torch.cuda.synchronize()
    assert torch.equal(o1, o2)


def test_attn_global_strided_layouts(handle):
    """q/k/v as slices of a packed [N, 3, H, D] tensor and O into a [N, H*D] buffer."""
    H, N, D = 4, 517, 64
    q, k, v = _qkv(H, N, D, "R1", seed=5)
    packed = torch.zeros((N, 3, H, D), dtype=torch.bfloat16, device=DEV)
    for i, a in enumerate((q, k, v)):
        packed[:, i] = to_dev(head_major_to_tokens(a), torch.bfloat16)
    o = torch.zeros((N, H * D), dtype=torch.bfloat16, device=DEV)
    vg.attn_global(handle, packed[:, 0], packed[:, 1], packed[:, 2], o.view(N, H, D), [0, N], vg.BF16)
    torch.cuda.synchronize()
    got = o.float().cpu().numpy().reshape(N, H, D).transpose(1, 0, 2)
    assert max_abs_rel(got, oracle.attention(q, k, v)) < 2e-2


def test_attn_global_sampled_rows_large(handle):
    """N = 43,968 (32 frames of 1374 tokens); oracle on 256 sampled query rows."""
    H, S, P, D = 2, 32, 1374, 64
    N = S * P
    q, k, v = _qkv(H, N, D, "R2", seed=6, frames=S)
    got = _run_global(handle, q, k, v, [0, N], vg.BF16)
    rows = synth.sample_rows(6, N, 256, P)
    ref = oracle.attention(q[:, rows], k, v)
    e = max_abs_rel(got[:, rows], ref)
    print(f"large sampled max_abs_rel={e:.3e}")
    assert e < 2e-2


def test_quantize_fp8_bit_exact(handle):
    H, D = 4, 64
    offs = [0, 300, 301, 688]
    rng = np.random.default_rng(7)
    x = synth.round_bf16(rng.normal(0, 0.8, (offs[-1], H, D)).astype(np.float32))
    x[5:9, 1] *= 40.0  # a block with a large amax
    x[300, :] = 0.0    # the one-token sequence is all zero: scale 1, codes 0
    x = synth.round_bf16(x)  # the device holds bf16: give the oracle the same values
    xd = to_dev(x, torch.bfloat16)
    codes, scales = vg.quantize_fp8(handle, xd, offs)
    torch.cuda.synchronize()
    codes = codes.cpu().numpy(); scales = scales.cpu().numpy()
    blk = 0
    for a, b in zip(offs[:-1], offs[1:]):
        starts = np.arange(a, b, 128); ends = np.minimum(starts + 128, b)
        for h in range(H):
            rc, rs = oracle.quantize_rows(x[:, h], starts, ends)
            np.testing.assert_array_equal(codes[h, a:b], rc[a:b])
            np.testing.assert_array_equal(scales[h, blk:blk + len(starts)], rs)
        blk += len(starts)


def _handle_with(env):
    import os
    old = {k: os.environ.get(k) for k in env}
    os.environ.update({k: str(v) for k, v in env.items()})
    try:
        return vg.Handle(0, dim=1024, heads=16, mlp_hidden=4096)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


@pytest.mark.parametrize("prec,key,values", [(vg.FP8_E4M3, "VGGTX_FP8_VARIANT", [0, 1, 2, 3]),
                                             (vg.BF16, "VGGTX_BF16_VARIANT", [0, 1, 2])])
def test_tile_variants_are_bitwise_identical(prec, key, values):
    """Every tile variant computes each query row with the same arithmetic in the same order."""
    H, D = 16, 64
    offs = [0, 700, 701, 1500, 3100]
    q, k, v = _qkv(H, offs[-1], D, "R1", seed=8)
    qd, kd, vd = (_dev_tokens(a, prec) for a in (q, k, v))
    outs = []
    for val in values:
        h = _handle_with({key: val})
        o = torch.zeros_like(qd)
        vg.attn_global(h.h, qd, kd, vd, o, offs, prec)
        torch.cuda.synchronize()
        outs.append(o)
        h.close()
    for o in outs[1:]:
        assert torch.equal(o, outs[0])


@pytest.mark.parametrize("prec", [vg.BF16, vg.FP8_PV, vg.FP8_E4M3])
def test_queue_and_grid_schedules_agree(prec):
    """Queue mode (work items taken from a counter, longest scene first,
    head by head) and the plain grid compute every (row, head) with the same
    arithmetic: bitwise equal outputs on uneven scenes, empty ones and a
    one-token scene included, twice in a row on one handle (the counter is
    reset before every launch)."""
    H, D = 16, 64
    offs = [0, 700, 701, 701, 1500, 3100, 3229]
    q, k, v = _qkv(H, offs[-1], D, "R1", seed=12)
    qd, kd, vd = (_dev_tokens(a, prec) for a in (q, k, v))
    outs = []
    for sched in (vg.SCHEDULE_GRID, vg.SCHEDULE_QUEUE):
        h = vg.Handle(0, dim=1024, heads=16, mlp_hidden=4096, attn_schedule=sched)
        for _ in range(2):
            o = torch.full_like(qd, float("nan"))
            vg.attn_global(h.h, qd, kd, vd, o, offs, prec)
            torch.cuda.synchronize()
            outs.append(o)
        h.close()
    assert torch.isfinite(outs[0].float()).all()
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    if prec != vg.FP8_E4M3:  # (all-E4M3 at logit std 3 is format-bound, gated elsewhere)
        ref = _oracle_seqs(q, k, v, offs)
        assert max_abs_rel(outs[-1].float().cpu().numpy().transpose(1, 0, 2), ref) < TOL[prec]


def test_autotune_picks_a_variant_and_caches_it(tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("VGGTX_AUTOTUNE_CACHE", str(cache))
    h = vg.Handle(0, dim=1024, heads=16, mlp_hidden=4096)
    v8 = vg.autotune(h.h, vg.FP8_E4M3, n_tokens=8192)
    vb = vg.autotune(h.h, vg.BF16, n_tokens=8192)
    assert 0 <= v8 < 4 and 0 <= vb < 3
    lines = cache.read_text().split()
    assert len(lines) == 8  # two records of (arch, prec, variant, ms)
    # a second handle reuses the cached choice without timing
    h2 = vg.Handle(0, dim=1024, heads=16, mlp_hidden=4096)
    assert vg.autotune(h2.h, vg.FP8_E4M3, n_tokens=8192) == v8
    # results after tuning still match the oracle
    H, D, N = 16, 64, 900
    q, k, v = _qkv(H, N, D, "R0", seed=9)
    qd, kd, vd = (_dev_tokens(a, vg.FP8_E4M3) for a in (q, k, v))
    o = torch.zeros_like(qd)
    vg.attn_global(h.h, qd, kd, vd, o, [0, N], vg.FP8_E4M3)
    torch.cuda.synchronize()
    assert max_abs_rel(o.float().cpu().numpy().transpose(1, 0, 2), oracle.attention(q, k, v)) < 6e-2
    h.close(); h2.close()


def _rising_keys(steps, offs, seed=43, H=2, D=64):
    rng = np.random.default_rng(seed)
    n = offs[-1]
    u = rng.normal(0, 1, (H, 1, D))
    u /= np.linalg.norm(u, axis=-1, keepdims=True)
    q = 8.0 * u + rng.normal(0, 0.05, (H, n, D))
    k = np.empty((H, n, D))
    for (a, b), step in zip(zip(offs[:-1], offs[1:]), steps):
        tile = (np.arange(b - a) // 64)[None, :, None]
        k[:, a:b] = (step * np.log(2.0)) * tile * u + rng.normal(0, 0.05, (H, b - a, D))
    v = rng.normal(0, 1, (H, n, D))
    return tuple(synth.round_bf16(x.astype(np.float32)).astype(np.float64) for x in (q, k, v))


@pytest.mark.parametrize("case", ["R0", "R1", "R2", "varlen", "rising"])
def test_attn_global_fp8_streamed_placement_diagnostic(handle, case):
    """Diagnostic only (no gate): how closely the FP8 kernel follows its own
    placement rule, compared with a float64 emulation of that rule
    (tests/fp8_stream_emulation.py), which shares the kernel's tiling and so
    cannot serve as an accuracy reference."""
    from fp8_stream_emulation import attention_fp8_streamed
    if case in ("R0", "R1", "R2"):
        q, k, v = _qkv(4, 8 * 86, 64, case, seed=1, frames=8)
        offs = [0, 8 * 86]
    elif case == "varlen":
        q, k, v = _qkv(4, 845, 64, "R1", seed=2)
        offs = [0, 200, 201, 201, 718, 845]
    else:
        offs = [0, 900, 1500]
        q, k, v = _rising_keys((3.0, 1.2), offs)
    got = _run_global(handle, q, k, v, offs, vg.FP8_E4M3)
    emu = np.zeros(q.shape)
    for a, b in zip(offs[:-1], offs[1:]):
        if b > a:
            emu[:, a:b] = attention_fp8_streamed(q[:, a:b], k[:, a:b], v[:, a:b])[0]
    print(f"fp8 kernel vs its placement-rule emulation, {case}: max_abs_rel={max_abs_rel(got, emu):.3e}")
    assert np.isfinite(got).all()


@pytest.mark.parametrize("case", ["R0", "R1", "R2", "varlen", "tails", "far_below", "rising"])
def test_attn_global_fp8pv_meets_fp8_gate(handle, case):
    """Scores in bfloat16, P and V in E4M3 (VGGTX_FP8_PV): within the FP8
    gate of the float64 definition in every logit regime, since Q and K keep
    8 mantissa bits (their E4M3 rounding is what moves large logits), on
    ragged and one-key tails, and through the overflow fallback of the
    probability placement (keys rising 3 and 1.2 binades per tile, a first
    tile far below the row maximum)."""
    if case in ("R0", "R1", "R2"):
        q, k, v = _qkv(4, 8 * 86, 64, case, seed=1, frames=8)
        offs = [0, 8 * 86]
    elif case == "varlen":
        offs = [0, 200, 201, 201, 718, 845]
        q, k, v = _qkv(4, offs[-1], 64, "R1", seed=2)
    elif case == "tails":
        offs = [0, 65, 194, 387]
        q, k, v = _qkv(4, offs[-1], 64, "R0", seed=10)
    else:
        q, k, v, offs = _far_below_case() if case == "far_below" else _rising_case()
        q, k, v = (synth.round_bf16(x.astype(np.float32)) for x in (q, k, v))
    got = _run_global(handle, q, k, v, offs, vg.FP8_PV)
    ref = _oracle_seqs(q, k, v, offs)
    e = max_abs_rel(got, ref)
    print(f"fp8pv {case}: max_abs_rel={e:.3e}")
    assert np.isfinite(got).all() and e < TOL[vg.FP8_PV]


@pytest.mark.parametrize("key,values", [("VGGTX_BF16_VARIANT", [0, 1, 2])])
def test_fp8pv_tile_variants_are_bitwise_identical(key, values):
    H, D = 16, 64
    offs = [0, 700, 701, 1500, 3100]
    q, k, v = _qkv(H, offs[-1], D, "R1", seed=8)
    qd, kd, vd = (_dev_tokens(a, vg.FP8_PV) for a in (q, k, v))
    outs = []
    for val in values:
        h = _handle_with({key: val})
        o = torch.zeros_like(qd)
        vg.attn_global(h.h, qd, kd, vd, o, offs, vg.FP8_PV)
        torch.cuda.synchronize()
        outs.append(o)
        h.close()
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
