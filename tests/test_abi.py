"""Host-side checks of the C-ABI library: it loads, exports every entry point
the public header declares, and rejects bad calls before touching a device."""
import ctypes
import os
import re

import pytest

import paper_2509_25191_amd.vggtx as vg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vggtx.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vggtx_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = vg.load()
    names = _declared_functions()
    assert "vggtx_aggregate" in names and "vggtx_attn_global" in names and "vggtx_attn_frame" in names
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_every_entry_point():
    for n in _declared_functions():
        assert hasattr(vg, n[len("vggtx_"):]), n


def test_status_strings():
    assert vg.status_str(0) == "ok"
    assert vg.status_str(3) == "workspace too small"
    assert vg.status_str(99) == "unknown status"


def test_null_handle_is_rejected_without_device():
    lib = vg.load()
    n = ctypes.c_size_t()
    assert lib.vggtx_workspace_size(None, 8, 86, vg.BF16, ctypes.byref(n)) == 1
    assert "null" in vg.last_error()
    ol = (ctypes.c_int32 * 1)(0)
    assert lib.vggtx_aggregate(None, None, 8, 86, None, 1, ol, 1, None, 1, 1, None, 0, None) == 1
    assert lib.vggtx_timing_enable(None, 1) == 1


def test_create_validates_config_before_device():
    lib = vg.load()
    h = ctypes.c_void_p()
    bad_d = vg.Config(256, 4, 32, 1024, 1e-6, 128)     # head_dim 32 unsupported
    assert lib.vggtx_create(ctypes.byref(h), 0, ctypes.byref(bad_d)) == 2
    bad_c = vg.Config(192, 3, 64, 768, 1e-6, 128)      # dim not a multiple of 128
    assert lib.vggtx_create(ctypes.byref(h), 0, ctypes.byref(bad_c)) == 2
    bad_h = vg.Config(256, 3, 64, 1024, 1e-6, 128)     # dim != heads * head_dim
    assert lib.vggtx_create(ctypes.byref(h), 0, ctypes.byref(bad_h)) == 1
    bad_eps = vg.Config(256, 4, 64, 1024, 0.0, 128)
    assert lib.vggtx_create(ctypes.byref(h), 0, ctypes.byref(bad_eps)) == 1
    bad_inplace = vg.Config(256, 4, 64, 1024, 1e-6, 128, 2)  # tokens_inplace is a 0/1 flag
    assert lib.vggtx_create(ctypes.byref(h), 0, ctypes.byref(bad_inplace)) == 1
    bad_sched = vg.Config(256, 4, 64, 1024, 1e-6, 128, 0, 2)  # attn_schedule is 0 (queue) or 1 (grid)
    assert lib.vggtx_create(ctypes.byref(h), 0, ctypes.byref(bad_sched)) == 1
    assert h.value is None


def test_no_device_reports_nodevice():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = vg.load()
    h = ctypes.c_void_p()
    ok = vg.Config(256, 4, 64, 1024, 1e-6, 128)
    assert lib.vggtx_create(ctypes.byref(h), 0, ctypes.byref(ok)) == 5


def test_front_end_rejects_bad_calls_without_device():
    lib = vg.load()
    n = ctypes.c_size_t()
    assert lib.vggtx_embed_workspace_size(None, 4, 518, 518, vg.BF16, ctypes.byref(n)) == 1
    off = (ctypes.c_int32 * 2)(0, 4)
    assert lib.vggtx_embed(None, None, 518, 518, off, 1, None, None, vg.BF16, None, 0, None) == 1
    assert "null" in vg.last_error()


def test_ga_pair_selection_is_host_side_and_matches_oracle():
    """vggtx_ga_select_pairs runs on the host (no device needed)."""
    import numpy as np
    import synth
    from oracle import ga
    rng = np.random.default_rng(3)
    _, init = synth.gen_ga_cameras(rng, 40, arc_deg=300.0, rot_noise_deg=3.0)
    got = vg.ga_select_pairs(init["R"], 30.0)
    want = [tuple(p) for p in ga.select_pairs(init["R"], 30.0).tolist()]
    assert got == want and len(got) > 40
    lib = vg.load()
    n = ctypes.c_int()
    small = (ctypes.c_int32 * 2)()
    Rh = np.ascontiguousarray(init["R"])
    assert lib.vggtx_ga_select_pairs(Rh.ctypes.data_as(ctypes.c_void_p), 40, 30.0, small, 1, ctypes.byref(n)) == 1
    cfg = vg.ga_config_default()
    assert cfg.iterations == 300 and list(cfg.lr) == [5e-4, 1e-3, 1e-2] and list(cfg.bounds) == [2.5, 7.5]
