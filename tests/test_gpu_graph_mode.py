"""Graph mode of the aggregate entry points: a forward recorded once and
replayed as a HIP graph gives the direct call's result bitwise, follows
reallocated buffers by updating node arguments (no rebuild), and builds a new
graph only for a new structure."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import to_dev, weights_to_dev

vg = pytest.importorskip("paper_2509_25191_amd.vggtx")
pytestmark = pytest.mark.gpu

M = synth.ModelConfig(dim=256, heads=4, head_dim=64, mlp_hidden=1024, depth=3)


def _handle(chunk=2):
    return vg.Handle(0, dim=M.dim, heads=M.heads, head_dim=M.head_dim, mlp_hidden=M.mlp_hidden, ln_eps=M.ln_eps,
                     frame_chunk=chunk)


def _direct(tokens, offs, layers, out_layers, prec):
    h = _handle()
    out = vg.aggregate_varlen(h.h, tokens, offs, layers, out_layers, prec)
    torch.cuda.synchronize()
    h.close()
    return out


@pytest.mark.parametrize("prec", [vg.BF16, vg.FP8_PV, vg.F32])
def test_graph_replay_follows_reallocated_buffers(prec):
    dt = torch.float32 if prec == vg.F32 else torch.bfloat16
    offs = [0, 3, 3, 8]  # three scenes, one empty
    P, out_layers = 86, [0, 2]
    tokens, layers = synth.gen_problem(M, offs[-1], P, seed=5, bf16=prec != vg.F32)
    td = to_dev(tokens, torch.float32)
    ld = weights_to_dev(layers, dt)
    ref = _direct(td, offs, ld, out_layers, prec)

    h = _handle()
    vg.graph_mode(h.h, True)
    ws = torch.empty(vg.workspace_size(h.h, offs[-1], P, prec), dtype=torch.uint8, device=td.device)
    out = vg.aggregate_varlen(h.h, td, offs, ld, out_layers, prec, ws=ws)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    st = vg.graph_stats(h.h)
    assert st["graphs"] == 1 and st["builds"] == 1 and st["launches"] == 1

    # every buffer reallocated (tokens, weights, outputs, workspace), new
    # token values, eager work on the device in between
    for rep in range(3):
        td2 = (td * (0.5 + 0.25 * rep)).contiguous()
        ld2 = weights_to_dev(layers, dt)
        ws2 = torch.empty_like(ws)
        junk = torch.randn(1 << 20, device=td.device).cumsum(0)
        out2 = vg.aggregate_varlen(h.h, td2, offs, ld2, out_layers, prec, ws=ws2)
        torch.cuda.synchronize()
        ref2 = _direct(td2, offs, ld2, out_layers, prec)
        assert torch.equal(out2, ref2), f"replay {rep}"
        del junk
    st = vg.graph_stats(h.h)
    assert st["builds"] == 1 and st["launches"] == 4 and st["node_updates"] > 0

    # a new structure (fewer tokens: other GEMM grids) builds a second graph;
    # the first is still replayable.  (Other scene splits of the same tokens
    # may map to the same launches, and then share a graph.)
    offs3 = [0, 4, 7]
    td3 = td[:7].contiguous()
    out3 = vg.aggregate_varlen(h.h, td3, offs3, ld, out_layers, prec, ws=ws)
    torch.cuda.synchronize()
    assert torch.equal(out3, _direct(td3, offs3, ld, out_layers, prec))
    out4 = vg.aggregate_varlen(h.h, td, offs, ld, out_layers, prec, ws=ws)
    torch.cuda.synchronize()
    assert torch.equal(out4, ref)
    st = vg.graph_stats(h.h)
    assert st["graphs"] == 2 and st["builds"] == 2 and st["launches"] == 6
    vg.graph_mode(h.h, False)
    assert vg.graph_stats(h.h)["graphs"] == 0
    h.close()


def test_graph_mode_errors_enqueue_nothing():
    """A call that fails validation in graph mode records and enqueues
    nothing and leaves the cache as it was."""
    tokens, layers = synth.gen_problem(M, 4, 86, seed=6, bf16=True)
    td = to_dev(tokens, torch.float32)
    ld = weights_to_dev(layers, torch.bfloat16)
    h = _handle()
    vg.graph_mode(h.h, True)
    with pytest.raises(vg.VggtxError):
        vg.aggregate(h.h, td, ld, [2, 1], vg.BF16)  # out_layers not increasing
    assert vg.graph_stats(h.h) == {"graphs": 0, "builds": 0, "node_updates": 0, "launches": 0}
    h.close()
