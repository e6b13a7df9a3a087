"""Thin ctypes binding of the vggtx C-ABI (include/vggtx.h).

Argument marshalling only: every step of the aggregator runs in the HIP
library.  PyTorch provides device memory and the current stream.  Function
names follow the C entry points without the ``vggtx_`` prefix.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence

import torch

__all__ = [
    "F32", "BF16", "FP8_E4M3", "FP8_PV", "OUT_F32", "OUT_BF16", "VggtxError", "library_path", "load",
    "Config", "BlockW", "PairW", "Layout", "Handle", "create", "destroy", "workspace_size",
    "aggregate", "aggregate_varlen", "block", "attn_workspace_size", "attn_frame", "attn_global",
    "quantize_fp8", "status_str", "last_error", "BLOCK_FIELDS", "timing_enable", "timing_read", "timing_poll",
    "autotune_workspace_size", "autotune", "EmbedW", "EMBED_FIELDS", "embed_workspace_size", "embed",
    "GaConfig", "ga_config_default", "ga_select_pairs", "ga_workspace_size", "ga_align", "auc30",
    "pack_head_inputs", "SCHEDULE_QUEUE", "SCHEDULE_GRID", "graph_mode", "graph_stats",
    "K_ATTN_GLOBAL", "K_ATTN_FRAME", "K_GEMM", "K_OTHER",
]

F32, BF16, FP8_E4M3, FP8_PV = 0, 1, 2, 3
K_ATTN_GLOBAL, K_ATTN_FRAME, K_GEMM, K_OTHER = 0, 1, 2, 3
OUT_F32, OUT_BF16 = 0, 1
BLOCK_FIELDS = ("ln1_g", "ln1_b", "w_qkv", "b_qkv", "w_o", "b_o",
                "ln2_g", "ln2_b", "w_fc1", "b_fc1", "w_fc2", "b_fc2")

_LIB_NAME = "libvggtx.so"
_lib = None


def library_path() -> str:
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), _LIB_NAME)


class VggtxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"vggtx status {status} ({status_str(status)}): {msg}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("heads", ctypes.c_int), ("head_dim", ctypes.c_int),
                ("mlp_hidden", ctypes.c_int), ("ln_eps", ctypes.c_float), ("frame_chunk", ctypes.c_int),
                ("tokens_inplace", ctypes.c_int), ("attn_schedule", ctypes.c_int)]

# Config.attn_schedule
SCHEDULE_QUEUE, SCHEDULE_GRID = 0, 1


class BlockW(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in BLOCK_FIELDS]


class PairW(ctypes.Structure):
    _fields_ = [("frame", BlockW), ("global_", BlockW)]


EMBED_FIELDS = ("w_patch", "b_patch", "pos", "cls", "reg", "norm_g", "norm_b", "cam", "agg_reg")


class EmbedW(ctypes.Structure):
    _fields_ = [("w_patch", ctypes.c_void_p), ("b_patch", ctypes.c_void_p), ("pos", ctypes.c_void_p),
                ("cls", ctypes.c_void_p), ("reg", ctypes.c_void_p), ("blocks", ctypes.POINTER(BlockW)),
                ("depth", ctypes.c_int), ("norm_g", ctypes.c_void_p), ("norm_b", ctypes.c_void_p),
                ("cam", ctypes.c_void_p), ("agg_reg", ctypes.c_void_p)]


class GaConfig(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("lr", ctypes.c_double * 3), ("bounds", ctypes.c_double * 2),
                ("alpha", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double)]


class Layout(ctypes.Structure):
    _fields_ = [("token_stride", ctypes.c_int64), ("head_stride", ctypes.c_int64)]


class Timing(ctypes.Structure):
    _fields_ = [("total_ms", ctypes.c_double), ("launches", ctypes.c_int64), ("flops", ctypes.c_double)]


def load():
    """Load libvggtx.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2509_25191_amd.build`")
    L = ctypes.CDLL(path)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
    P_i32 = ctypes.POINTER(ctypes.c_int32)
    sig = {
        "vggtx_create": [ctypes.POINTER(vp), i32, ctypes.POINTER(Config)],
        "vggtx_destroy": [vp],
        "vggtx_workspace_size": [vp, i32, i32, i32, ctypes.POINTER(sz)],
        "vggtx_aggregate": [vp, vp, i32, i32, ctypes.POINTER(PairW), i32, P_i32, i32, vp, i32, i32, vp, sz, vp],
        "vggtx_aggregate_varlen": [vp, vp, P_i32, i32, i32, ctypes.POINTER(PairW), i32, P_i32, i32, vp, i32, i32,
                                   vp, sz, vp],
        "vggtx_block": [vp, vp, vp, P_i32, i32, ctypes.POINTER(BlockW), i32, vp, sz, vp],
        "vggtx_attn_workspace_size": [vp, P_i32, i32, i32, i32, i32, ctypes.POINTER(sz)],
        "vggtx_attn_frame": [vp, vp, vp, vp, vp, i32, i32, i32, i32, Layout, Layout, i32, vp, sz, vp],
        "vggtx_attn_global": [vp, vp, vp, vp, vp, P_i32, i32, i32, i32, Layout, Layout, i32, vp, sz, vp],
        "vggtx_attn_global_noalloc": [vp, vp, vp, vp, vp, P_i32, i32, i32, i32, Layout, Layout, i32, vp],
        "vggtx_quantize_fp8": [vp, vp, Layout, P_i32, i32, i32, i32, vp, vp, vp],
        "vggtx_autotune_workspace_size": [vp, i32, ctypes.POINTER(sz)],
        "vggtx_autotune": [vp, i32, i32, vp, sz, vp, ctypes.POINTER(i32)],
        "vggtx_embed_workspace_size": [vp, i32, i32, i32, i32, ctypes.POINTER(sz)],
        "vggtx_embed": [vp, vp, i32, i32, P_i32, i32, ctypes.POINTER(EmbedW), vp, i32, vp, sz, vp],
        "vggtx_ga_config_default": [ctypes.POINTER(GaConfig)],
        "vggtx_ga_select_pairs": [vp, i32, ctypes.c_double, P_i32, i32, ctypes.POINTER(i32)],
        "vggtx_ga_workspace_size": [vp, i32, i32, i64, ctypes.POINTER(sz)],
        "vggtx_ga_align": [vp, ctypes.POINTER(GaConfig), i32, vp, vp, vp, vp, P_i32, i32,
                           ctypes.POINTER(ctypes.c_int64), vp, vp, vp, vp, vp, vp, vp, sz, vp],
        "vggtx_auc30": [vp, vp, vp, vp, vp, i32, i32, vp, vp, vp],
        "vggtx_pack_head_inputs": [vp, vp, i32, i32, i32, i32, i32, i32, vp, vp],
        "vggtx_graph_mode": [vp, i32],
        "vggtx_graph_stats": [vp, ctypes.POINTER(ctypes.c_int64)],
        "vggtx_timing_enable": [vp, i32],
        "vggtx_timing_read": [vp, ctypes.POINTER(Timing), ctypes.POINTER(ctypes.c_int64)],
        "vggtx_timing_poll": [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                              ctypes.POINTER(ctypes.c_int64)],
        "vggtx_status_str": [i32],
        "vggtx_last_error": [],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name in ("vggtx_status_str", "vggtx_last_error") else ctypes.c_int
    L.vggtx_ga_config_default.restype = None
    _lib = L
    return L


def status_str(s: int) -> str:
    return load().vggtx_status_str(int(s)).decode()


def last_error() -> str:
    return load().vggtx_last_error().decode()


def _check(status: int):
    if status != 0:
        raise VggtxError(status, last_error())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    if isinstance(stream, torch.cuda.Stream):
        stream = stream.cuda_stream
    return ctypes.c_void_p(int(stream))


def _i32_array(vals: Sequence[int]):
    arr = (ctypes.c_int32 * max(1, len(vals)))(*[int(v) for v in vals])
    return arr


def create(device: int, dim: int, heads: int, head_dim: int = 64, mlp_hidden: Optional[int] = None,
           ln_eps: float = 1e-6, frame_chunk: int = 128, tokens_inplace: bool = False,
           attn_schedule: int = SCHEDULE_QUEUE) -> ctypes.c_void_p:
    cfg = Config(dim, heads, head_dim, mlp_hidden if mlp_hidden is not None else 4 * dim, ln_eps, frame_chunk,
                 1 if tokens_inplace else 0, int(attn_schedule))
    h = ctypes.c_void_p()
    _check(load().vggtx_create(ctypes.byref(h), int(device), ctypes.byref(cfg)))
    return h


def destroy(h) -> None:
    _check(load().vggtx_destroy(h))


def workspace_size(h, total_frames: int, P: int, prec: int) -> int:
    n = ctypes.c_size_t()
    _check(load().vggtx_workspace_size(h, int(total_frames), int(P), int(prec), ctypes.byref(n)))
    return n.value


def block_w(params: Dict[str, torch.Tensor]) -> BlockW:
    return BlockW(*[ctypes.c_void_p(params[n].data_ptr()) for n in BLOCK_FIELDS])


def pair_array(layers: List[Dict[str, Dict[str, torch.Tensor]]]):
    arr = (PairW * len(layers))()
    for i, l in enumerate(layers):
        arr[i].frame = block_w(l["frame"])
        arr[i].global_ = block_w(l["global"])
    return arr


def _alloc_ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def aggregate(h, tokens: torch.Tensor, layers, out_layers: Sequence[int], prec: int, out: Optional[torch.Tensor] = None,
              out_dtype: int = OUT_BF16, ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """tokens [S, P, C] float32 on the device; layers: list of {"frame": {...}, "global": {...}}."""
    S, P, C = tokens.shape
    return aggregate_varlen(h, tokens, [0, S], layers, out_layers, prec, out, out_dtype, ws, stream, _single=True)


def aggregate_varlen(h, tokens: torch.Tensor, frame_offsets: Sequence[int], layers, out_layers: Sequence[int],
                     prec: int, out: Optional[torch.Tensor] = None, out_dtype: int = OUT_BF16,
                     ws: Optional[torch.Tensor] = None, stream=None, _single: bool = False) -> torch.Tensor:
    S, P, C = tokens.shape
    if out is None:
        out = torch.empty((len(out_layers), S, P, 2 * C), device=tokens.device,
                          dtype=torch.float32 if out_dtype == OUT_F32 else torch.bfloat16)
    if ws is None:
        ws = _alloc_ws(workspace_size(h, S, P, prec), tokens.device)
    pw = pair_array(layers)
    ol = _i32_array(out_layers)
    if _single:
        st = load().vggtx_aggregate(h, _ptr(tokens), S, P, pw, len(layers), ol, len(out_layers), _ptr(out),
                                    out_dtype, prec, _ptr(ws), ws.numel(), _stream(stream))
    else:
        fo = _i32_array(frame_offsets)
        st = load().vggtx_aggregate_varlen(h, _ptr(tokens), fo, len(frame_offsets) - 1, P, pw, len(layers), ol,
                                           len(out_layers), _ptr(out), out_dtype, prec, _ptr(ws), ws.numel(),
                                           _stream(stream))
    _check(st)
    return out


def block(h, x_in: torch.Tensor, x_out: torch.Tensor, seq_offsets: Sequence[int], params: Dict[str, torch.Tensor],
          prec: int, ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    if ws is None:
        lmax = max(b - a for a, b in zip(seq_offsets[:-1], seq_offsets[1:])) if len(seq_offsets) > 1 else 1
        ws = _alloc_ws(workspace_size(h, len(seq_offsets) - 1, max(1, lmax), prec), x_in.device)
    bw = block_w(params)
    _check(load().vggtx_block(h, _ptr(x_in), _ptr(x_out), _i32_array(seq_offsets), len(seq_offsets) - 1,
                              ctypes.byref(bw), prec, _ptr(ws), ws.numel(), _stream(stream)))
    return x_out


def attn_workspace_size(h, seq_offsets: Sequence[int], H: int, D: int, prec: int) -> int:
    n = ctypes.c_size_t()
    _check(load().vggtx_attn_workspace_size(h, _i32_array(seq_offsets), len(seq_offsets) - 1, H, D, prec,
                                            ctypes.byref(n)))
    return n.value


def _layout(t: torch.Tensor) -> Layout:
    # t viewed as [tokens, H, D]
    return Layout(t.stride(0), t.stride(1))


def attn_frame(h, q, k, v, o, S: int, P: int, prec: int, ws: Optional[torch.Tensor] = None, stream=None):
    """q, k, v, o: [S*P, H, D] views (any token / head strides, unit stride along D)."""
    H, D = q.shape[1], q.shape[2]
    if ws is None:
        ws = _alloc_ws(attn_workspace_size(h, [f * P for f in range(S + 1)], H, D, prec), q.device)
    _check(load().vggtx_attn_frame(h, _ptr(q), _ptr(k), _ptr(v), _ptr(o), S, P, H, D, _layout(q), _layout(o), prec,
                                   _ptr(ws), ws.numel(), _stream(stream)))
    return o


def attn_global(h, q, k, v, o, seq_offsets: Sequence[int], prec: int, ws: Optional[torch.Tensor] = None,
                stream=None):
    H, D = q.shape[1], q.shape[2]
    if ws is None:
        ws = _alloc_ws(attn_workspace_size(h, seq_offsets, H, D, prec), q.device)
    _check(load().vggtx_attn_global(h, _ptr(q), _ptr(k), _ptr(v), _ptr(o), _i32_array(seq_offsets),
                                    len(seq_offsets) - 1, H, D, _layout(q), _layout(o), prec, _ptr(ws), ws.numel(),
                                    _stream(stream)))
    return o


def attn_global_noalloc(h, q, k, v, o, seq_offsets: Sequence[int], prec: int, stream=None):
    """vggtx_attn_global with the library's fixed device scratch (no workspace)."""
    H, D = q.shape[1], q.shape[2]
    _check(load().vggtx_attn_global_noalloc(h, _ptr(q), _ptr(k), _ptr(v), _ptr(o), _i32_array(seq_offsets),
                                            len(seq_offsets) - 1, H, D, _layout(q), _layout(o), prec,
                                            _stream(stream)))
    return o


def quantize_fp8(h, x, seq_offsets: Sequence[int], codes=None, scales=None, stream=None):
    """x [N, H, D] bfloat16 -> codes uint8 [H, N, D], scales float32 [H, n_blocks]."""
    N, H, D = x.shape
    nblk = sum((b - a + 127) // 128 for a, b in zip(seq_offsets[:-1], seq_offsets[1:]))
    if codes is None:
        codes = torch.empty((H, N, D), dtype=torch.uint8, device=x.device)
    if scales is None:
        scales = torch.empty((H, max(1, nblk)), dtype=torch.float32, device=x.device)
    _check(load().vggtx_quantize_fp8(h, _ptr(x), _layout(x), _i32_array(seq_offsets), len(seq_offsets) - 1, H, D,
                                     _ptr(codes), _ptr(scales), _stream(stream)))
    return codes, scales


def autotune_workspace_size(h, n_tokens: int) -> int:
    n = ctypes.c_size_t()
    _check(load().vggtx_autotune_workspace_size(h, int(n_tokens), ctypes.byref(n)))
    return n.value


def autotune(h, prec: int, n_tokens: int = 32768, ws: Optional[torch.Tensor] = None, stream=None,
             device="cuda") -> int:
    """Pick the fastest attention tile variant for `prec`; returns its index."""
    if ws is None:
        ws = _alloc_ws(autotune_workspace_size(h, n_tokens), device)
    chosen = ctypes.c_int()
    _check(load().vggtx_autotune(h, int(prec), int(n_tokens), _ptr(ws), ws.numel(), _stream(stream),
                                 ctypes.byref(chosen)))
    return chosen.value


def embed_workspace_size(h, total_frames: int, height: int, width: int, prec: int) -> int:
    n = ctypes.c_size_t()
    _check(load().vggtx_embed_workspace_size(h, int(total_frames), int(height), int(width), int(prec),
                                             ctypes.byref(n)))
    return n.value


def embed(h, images: torch.Tensor, params: Dict[str, object], prec: int, frame_offsets: Optional[Sequence[int]] = None,
          out: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Front end: images [S, 3, height, width] float32 -> aggregator tokens [S, 5 + n_patches, C] float32.
    params: the EMBED_FIELDS tensors plus "blocks" (a list of block parameter dicts)."""
    S, _, height, width = images.shape
    C = params["norm_g"].shape[0]
    P = 5 + (height // 14) * (width // 14)
    if frame_offsets is None:
        frame_offsets = [0, S]
    if out is None:
        out = torch.empty((S, P, C), dtype=torch.float32, device=images.device)
    if ws is None:
        ws = _alloc_ws(embed_workspace_size(h, S, height, width, prec), images.device)
    blocks = params["blocks"]
    barr = (BlockW * max(1, len(blocks)))(*[block_w(b) for b in blocks])
    ew = EmbedW(*[ctypes.c_void_p(params[n].data_ptr()) for n in EMBED_FIELDS[:5]],
                ctypes.cast(barr, ctypes.POINTER(BlockW)), len(blocks),
                *[ctypes.c_void_p(params[n].data_ptr()) for n in EMBED_FIELDS[5:]])
    _check(load().vggtx_embed(h, _ptr(images), height, width, _i32_array(frame_offsets), len(frame_offsets) - 1,
                              ctypes.byref(ew), _ptr(out), int(prec), _ptr(ws), ws.numel(), _stream(stream)))
    return out


def ga_config_default() -> GaConfig:
    cfg = GaConfig()
    load().vggtx_ga_config_default(ctypes.byref(cfg))
    return cfg


def ga_select_pairs(R, max_angle_deg: float = 30.0):
    """R: host float64 array-like [N, 3, 3] -> list of (i, j) pairs (host-side rule)."""
    import numpy as np
    Rh = np.ascontiguousarray(np.asarray(R, dtype=np.float64))
    n = ctypes.c_int()
    _check(load().vggtx_ga_select_pairs(Rh.ctypes.data_as(ctypes.c_void_p), len(Rh), float(max_angle_deg), None, 0,
                                        ctypes.byref(n)))
    buf = (ctypes.c_int32 * max(1, 2 * n.value))()
    _check(load().vggtx_ga_select_pairs(Rh.ctypes.data_as(ctypes.c_void_p), len(Rh), float(max_angle_deg), buf,
                                        n.value, ctypes.byref(n)))
    return [(buf[2 * k], buf[2 * k + 1]) for k in range(n.value)]


def ga_workspace_size(h, n_cams: int, n_pairs: int, n_corr: int) -> int:
    n = ctypes.c_size_t()
    _check(load().vggtx_ga_workspace_size(h, int(n_cams), int(n_pairs), int(n_corr), ctypes.byref(n)))
    return n.value


def ga_align(h, R0: torch.Tensor, t0: torch.Tensor, f0: torch.Tensor, pp: torch.Tensor, pairs: Sequence,
             corr_offsets: Sequence[int], corr: torch.Tensor, cfg: Optional[GaConfig] = None, weights: bool = True,
             losses: bool = True, ws: Optional[torch.Tensor] = None, stream=None):
    """Global alignment.  Camera tensors float64 on the device, corr float32 [K, 4] on the device; pairs and
    corr_offsets on the host.  Returns (R, t, f, weights or None, losses or None)."""
    cfg = cfg if cfg is not None else ga_config_default()
    N, P = R0.shape[0], len(pairs)
    K = int(corr_offsets[-1]) if P else 0
    dev = R0.device
    R, t, f = torch.empty_like(R0), torch.empty_like(t0), torch.empty_like(f0)
    w = torch.empty(max(1, K), dtype=torch.float32, device=dev) if weights else None
    lo = torch.empty(cfg.iterations + 1, dtype=torch.float64, device=dev) if losses else None
    if ws is None:
        ws = _alloc_ws(ga_workspace_size(h, N, P, K), dev)
    pa = (ctypes.c_int32 * max(1, 2 * P))(*[int(v) for pr in pairs for v in pr])
    off = (ctypes.c_int64 * (P + 1))(*[int(v) for v in corr_offsets]) if P else None
    _check(load().vggtx_ga_align(h, ctypes.byref(cfg), N, _ptr(R0), _ptr(t0), _ptr(f0), _ptr(pp), pa, P, off,
                                 _ptr(corr), _ptr(R), _ptr(t), _ptr(f), _ptr(w), _ptr(lo), _ptr(ws), ws.numel(),
                                 _stream(stream)))
    return R, t, f, (w[:K] if w is not None else None), lo


def auc30(h, R_pred: torch.Tensor, t_pred: torch.Tensor, R_gt: torch.Tensor, t_gt: torch.Tensor,
          both_orders: bool = True, stream=None):
    """Pose AUC@30 on the device: returns (auc float64 [1], counts int32-viewed uint32 [31]) device tensors."""
    dev = R_pred.device
    counts = torch.empty(31, dtype=torch.int32, device=dev)
    auc = torch.empty(1, dtype=torch.float64, device=dev)
    _check(load().vggtx_auc30(h, _ptr(R_pred), _ptr(t_pred), _ptr(R_gt), _ptr(t_gt), R_pred.shape[0],
                              1 if both_orders else 0, _ptr(counts), _ptr(auc), _stream(stream)))
    return auc, counts


def pack_head_inputs(h, feats: torch.Tensor, grid_h: int, grid_w: int, out: Optional[torch.Tensor] = None,
                     stream=None) -> torch.Tensor:
    """feats [n_out, S, P, 2C] (float32 or bfloat16) -> [n_out, S, 2C, grid_h, grid_w]."""
    n_out, S, P, C2 = feats.shape
    if out is None:
        out = torch.empty((n_out, S, C2, grid_h, grid_w), dtype=feats.dtype, device=feats.device)
    dt = OUT_F32 if feats.dtype == torch.float32 else OUT_BF16
    _check(load().vggtx_pack_head_inputs(h, _ptr(feats), dt, n_out, S, P, grid_h, grid_w, _ptr(out),
                                         _stream(stream)))
    return out


def graph_mode(h, enable: bool = True) -> None:
    _check(load().vggtx_graph_mode(h, 1 if enable else 0))


def graph_stats(h) -> dict:
    """{"graphs", "builds", "node_updates", "launches"} of the handle's graph cache."""
    arr = (ctypes.c_int64 * 4)()
    _check(load().vggtx_graph_stats(h, arr))
    return dict(zip(("graphs", "builds", "node_updates", "launches"), list(arr)))


def timing_enable(h, enable: bool = True) -> None:
    _check(load().vggtx_timing_enable(h, 1 if enable else 0))


def timing_read(h) -> dict:
    """{class: {"ms", "launches", "flops"}} since the last enable/read, plus "dropped"."""
    arr = (Timing * 4)()
    dropped = ctypes.c_int64()
    _check(load().vggtx_timing_read(h, arr, ctypes.byref(dropped)))
    names = {K_ATTN_GLOBAL: "attn_global", K_ATTN_FRAME: "attn_frame", K_GEMM: "gemm", K_OTHER: "other"}
    out = {names[i]: {"ms": arr[i].total_ms, "launches": arr[i].launches, "flops": arr[i].flops} for i in range(4)}
    out["dropped"] = dropped.value
    return out


def timing_poll(h):
    """(finished launches, recorded launches, finished global-attention launches); non-blocking."""
    f, r, g = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load().vggtx_timing_poll(h, ctypes.byref(f), ctypes.byref(r), ctypes.byref(g)))
    return f.value, r.value, g.value


class Handle:
    """Owns a vggtx handle for one device and model shape."""

    def __init__(self, device: int = 0, dim: int = 1024, heads: int = 16, head_dim: int = 64,
                 mlp_hidden: Optional[int] = None, ln_eps: float = 1e-6, frame_chunk: int = 128,
                 tokens_inplace: bool = False, attn_schedule: int = SCHEDULE_QUEUE):
        self.h = create(device, dim, heads, head_dim, mlp_hidden, ln_eps, frame_chunk, tokens_inplace, attn_schedule)

    def close(self):
        if self.h is not None:
            destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
