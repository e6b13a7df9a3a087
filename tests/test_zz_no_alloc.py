"""vggtx_attn_global_noalloc, the entry point that allocates nothing (for
callers that cannot call hipMalloc: graph capture, serving loops), against
vggtx_attn_global with a caller workspace: the same kernels and arithmetic,
so the outputs agree bitwise.  Two calls in a row per precision, the second
on fewer tokens (the fixed scratch keeps the first call's contents), and a
call that needs more scratch than the library holds is rejected before any
work is enqueued."""
import numpy as np
import pytest
import torch

from gpu_util import DEV

vg = pytest.importorskip("paper_2509_25191_amd.vggtx")
pytestmark = pytest.mark.gpu

E_WORKSPACE = 3


def _qkv(N, H, seed):
    g = torch.Generator(device=DEV)
    g.manual_seed(seed)
    return [torch.empty((N, H, 64), device=DEV).normal_(0, 0.8, generator=g).to(torch.bfloat16) for _ in range(3)]


@pytest.mark.parametrize("prec", [1, 2])
def test_noalloc_matches_workspace_entry_point(prec):
    H = 16
    h = vg.Handle(0, dim=H * 64, heads=H, mlp_hidden=4 * H * 64)
    # first call: three ragged scenes, 6,000 tokens; second call: fewer tokens, other scenes
    for offs, seed in (([0, 1374, 4122, 6000], 1), ([0, 700, 701, 2049], 2)):
        q, k, v = _qkv(offs[-1], H, seed)
        ref = torch.full_like(q, float("nan"))
        got = torch.full_like(q, float("nan"))
        vg.attn_global(h.h, q, k, v, ref, offs, prec)
        vg.attn_global_noalloc(h.h, q, k, v, got, offs, prec)
        torch.cuda.synchronize()
        assert torch.isfinite(got.float()).all()
        print(f"noalloc prec={prec} tokens={offs[-1]}: max |diff| "
              f"{(got.float() - ref.float()).abs().max().item():.3e}", flush=True)
        assert torch.equal(got.view(torch.int16), ref.view(torch.int16))
    h.close()


def test_noalloc_rejects_more_than_its_scratch():
    H = 16
    h = vg.Handle(0, dim=H * 64, heads=H, mlp_hidden=4 * H * 64)
    n = 40000  # BF16 needs 16 * 64 * 40,000 * 2 bytes of transposed V, above 64 MiB
    assert vg.attn_workspace_size(h.h, [0, n], H, 64, vg.BF16) > 64 << 20
    q, k, v = _qkv(n, H, 3)
    o = torch.zeros_like(q)
    with pytest.raises(vg.VggtxError) as e:
        vg.attn_global_noalloc(h.h, q, k, v, o, [0, n], vg.BF16)
    assert e.value.status == E_WORKSPACE
    torch.cuda.synchronize()
    assert not o.any()
    h.close()
