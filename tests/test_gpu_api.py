"""The C ABI on a GPU: one call spanning more sequences than a launch carries
in its arguments, and calls that must fail host-side validation without
enqueueing any work (the contract of include/vggtx.h)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import DEV, head_major_to_tokens, max_abs_rel, to_dev

vg = pytest.importorskip("paper_2509_25191_amd.vggtx")
pytestmark = pytest.mark.gpu

E_INVALID, E_UNSUPPORTED, E_WORKSPACE = 1, 2, 3


@pytest.mark.parametrize("prec,tol", [(vg.BF16, 2e-2), (vg.FP8_E4M3, 6e-2)])
def test_global_attention_over_more_sequences_than_one_launch_holds(prec, tol):
    """100 sequences (a launch carries at most 64; longest-first groups),
    including empty and one-token sequences."""
    H, D = 2, 64
    rng = np.random.default_rng(31)
    lens = rng.integers(0, 160, size=100)
    lens[[3, 50, 99]] = 0
    lens[[10, 64]] = 1
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(int).tolist()
    q, k, v = synth.gen_qkv(rng, H, offs[-1], D, "R0")
    qd, kd, vd = (to_dev(head_major_to_tokens(a), torch.bfloat16) for a in (q, k, v))
    o = torch.zeros_like(qd)
    h = vg.Handle(0, dim=H * D, heads=H, mlp_hidden=4 * H * D)
    vg.attn_global(h.h, qd, kd, vd, o, offs, prec)
    torch.cuda.synchronize()
    got = o.float().cpu().numpy().transpose(1, 0, 2)
    ref = np.zeros(q.shape)
    for a, b in zip(offs[:-1], offs[1:]):
        if b > a:
            ref[:, a:b] = oracle.attention(q[:, a:b], k[:, a:b], v[:, a:b])
    e = max_abs_rel(got, ref)
    print(f"100 sequences prec={prec} max_abs_rel={e:.3e}")
    assert e < tol
    h.close()


def _qkv(N=300, H=2, D=64):
    g = torch.Generator(device=DEV)
    g.manual_seed(5)
    return [torch.empty((N, H, D), device=DEV).normal_(0, 0.6, generator=g).to(torch.bfloat16) for _ in range(3)]


def _expect(status, fn):
    with pytest.raises(vg.VggtxError) as e:
        fn()
    assert e.value.status == status, str(e.value)
    assert vg.last_error() != ""


def test_rejected_attention_calls_write_nothing():
    h = vg.Handle(0, dim=128, heads=2, mlp_hidden=256)
    q, k, v = _qkv()
    o = torch.full_like(q, 7.0)
    need = vg.attn_workspace_size(h.h, [0, 300], 2, 64, vg.FP8_E4M3)
    small = torch.empty(need // 2, dtype=torch.uint8, device=DEV)
    _expect(E_WORKSPACE, lambda: vg.attn_global(h.h, q, k, v, o, [0, 300], vg.FP8_E4M3, ws=small))
    _expect(E_INVALID, lambda: vg.attn_global(h.h, q, k, v, o, [0, 200, 100, 300], vg.BF16))  # decreasing
    q32 = torch.zeros((300, 2, 32), device=DEV, dtype=torch.bfloat16)
    _expect(E_UNSUPPORTED, lambda: vg.attn_global(h.h, q32, q32, q32, q32.clone(), [0, 300], vg.BF16))
    base = torch.zeros(300 * 2 * 64 + 8, device=DEV, dtype=torch.bfloat16)
    q_mis = base[1:1 + 300 * 2 * 64].view(300, 2, 64)  # 2-byte offset: not 16-byte aligned
    _expect(E_INVALID, lambda: vg.attn_global(h.h, q_mis, k, v, o, [0, 300], vg.BF16))
    torch.cuda.synchronize()
    assert bool((o == 7.0).all())
    h.close()


def test_rejected_aggregate_calls_write_nothing():
    m = synth.ModelConfig(dim=128, heads=2, head_dim=64, mlp_hidden=256, depth=2)
    S, P = 2, 20
    tokens, layers = synth.gen_problem(m, S, P, seed=3, bf16=True)
    ld = [{part: {kk: to_dev(vv, torch.bfloat16) for kk, vv in blk.items()} for part, blk in l.items()}
          for l in layers]
    h = vg.Handle(0, dim=m.dim, heads=m.heads, mlp_hidden=m.mlp_hidden)
    td = to_dev(tokens, torch.float32)
    out = torch.full((2, S, P, 2 * m.dim), 3.0, device=DEV, dtype=torch.bfloat16)
    _expect(E_INVALID, lambda: vg.aggregate(h.h, td, ld, [1, 0], vg.BF16, out=out))  # not increasing
    _expect(E_INVALID, lambda: vg.aggregate(h.h, td, ld, [0, 2], vg.BF16, out=out))  # layer >= depth
    ws = torch.empty(256, dtype=torch.uint8, device=DEV)
    _expect(E_WORKSPACE, lambda: vg.aggregate(h.h, td, ld, [0, 1], vg.BF16, out=out, ws=ws))
    torch.cuda.synchronize()
    assert bool((out == 3.0).all())
    # a valid call on the same handle still works after the rejected ones
    vg.aggregate(h.h, td, ld, [0, 1], vg.BF16, out=out)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out.float()).all()) and not bool((out == 3.0).all())
    h.close()
