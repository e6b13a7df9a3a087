"""The whole layer loop captured into one HIP graph (stream capture of
vggtx_aggregate), replayed several times with eager work in between; every
replay must equal the eager result bitwise."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import DEV, to_dev, weights_to_dev

vg = pytest.importorskip("paper_2509_25191_amd.vggtx")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", [vg.BF16, vg.FP8_E4M3])
def test_aggregate_graph_replay_matches_eager(prec):
    m = synth.ModelConfig(dim=128, heads=2, head_dim=64, mlp_hidden=256, depth=2)
    S, P = 6, 90
    scenes = [0, 2, 6]
    tokens, layers = synth.gen_problem(m, S, P, seed=21, bf16=True)
    ld = weights_to_dev(layers, torch.bfloat16)
    h = vg.Handle(0, dim=m.dim, heads=m.heads, mlp_hidden=m.mlp_hidden, frame_chunk=4)
    td = to_dev(tokens, torch.float32)
    ws = torch.empty(vg.workspace_size(h.h, S, P, prec), dtype=torch.uint8, device=DEV)
    eager = vg.aggregate_varlen(h.h, td, scenes, ld, [0, 1], prec, ws=ws)
    torch.cuda.synchronize()
    out = torch.zeros_like(eager)
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(graph, stream=stream):
            vg.aggregate_varlen(h.h, td, scenes, ld, [0, 1], prec, out=out, ws=ws, stream=stream)
    torch.cuda.synchronize()
    for i in range(3):
        out.zero_()
        ws.fill_(0xAB)           # scribble over the workspace between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), f"replay {i} differs"
    h.close()


def test_images_to_features_graph_replay_matches_eager():
    """Front end and aggregator captured together into one HIP graph (images
    in, features out), replayed with scribbled workspaces in between."""
    m = synth.ModelConfig(dim=128, heads=2, head_dim=64, mlp_hidden=256, depth=1)
    rng = np.random.default_rng(22)
    img = synth.gen_images(rng, 4, 28, 42)
    w = synth.gen_embed(rng, m, 28, 42, 2, bf16=True)
    layers = synth.gen_weights(rng, m, bf16=True)
    wd = {k: to_dev(w[k], torch.bfloat16) for k in vg.EMBED_FIELDS}
    wd["blocks"] = [{k: to_dev(v, torch.bfloat16) for k, v in b.items()} for b in w["blocks"]]
    ld = weights_to_dev(layers, torch.bfloat16)
    h = vg.Handle(0, dim=m.dim, heads=m.heads, mlp_hidden=m.mlp_hidden, frame_chunk=3)
    imgd = to_dev(img, torch.float32)
    offs = [0, 1, 4]
    P = 5 + 2 * 3
    ws_e = torch.empty(vg.embed_workspace_size(h.h, 4, 28, 42, vg.BF16), dtype=torch.uint8, device=DEV)
    ws_a = torch.empty(vg.workspace_size(h.h, 4, P, vg.FP8_E4M3), dtype=torch.uint8, device=DEV)
    tok = torch.empty((4, P, m.dim), dtype=torch.float32, device=DEV)
    vg.embed(h.h, imgd, wd, vg.BF16, frame_offsets=offs, out=tok, ws=ws_e)
    eager = vg.aggregate_varlen(h.h, tok, offs, ld, [0], vg.FP8_E4M3, ws=ws_a).clone()
    torch.cuda.synchronize()
    out = torch.zeros_like(eager)
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(graph, stream=stream):
            vg.embed(h.h, imgd, wd, vg.BF16, frame_offsets=offs, out=tok, ws=ws_e, stream=stream)
            vg.aggregate_varlen(h.h, tok, offs, ld, [0], vg.FP8_E4M3, out=out, ws=ws_a, stream=stream)
    torch.cuda.synchronize()
    for i in range(3):
        out.zero_()
        tok.fill_(-1.0)
        ws_e.fill_(0xCD)
        ws_a.fill_(0xAB)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), f"replay {i} differs"
    h.close()
