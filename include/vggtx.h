/*
 * vggtx — MI355X (gfx950) library for the memory-efficient dense-view
 * aggregator of VGGT-X (arXiv 2509.25191, Sec. 3.2).
 *
 * The aggregator runs `depth` alternating-attention layers over S frames of P
 * tokens each.  Every layer is a frame block (attention restricted to the P
 * tokens of one frame) followed by a global block (attention over every token
 * of the scene).  Only the outputs of the requested layers are kept, all
 * other activations are overwritten in place (the paper's "VGGT-" change), and
 * token-local work is processed in chunks of `frame_chunk` frames (the
 * paper's "VGGT--" change, chunk 128 in Sec. 4.1).
 *
 * Block (a reading: the paper does not spell the block out): pre-LayerNorm
 * transformer block, x += MHA(LN1(x)); x += W2 GELU(W1 LN2(x) + b1) + b2, with
 * exact-erf GELU, biases on every Linear, packed [q | k | v] projection
 * (head h = columns h*D .. h*D+D-1 of each part), attention scale 1/sqrt(D).
 *
 * Conventions for every entry point:
 *   - All pointers named as device pointers must point to device memory of the
 *     device the handle was created on; the caller owns every buffer (inputs,
 *     outputs, weights, workspace).  The library never allocates device memory.
 *   - Host pointers (offset tables, weight tables, layer lists) are read before
 *     the call returns.
 *   - Work is enqueued on `stream` and the call returns without waiting; device
 *     pointers must stay valid until that work completes.
 *   - Arguments are validated on the host before anything is enqueued: a call
 *     that returns an error has enqueued nothing and written nothing.
 *   - Errors never abort the process; the returned status says what failed and
 *     vggtx_last_error() (thread-local) gives a message.
 *   - Linear weights are stored [out, in] row-major (y = x W^T + b).
 *   - Element types: VGGTX_F32 runs every step in float32 (weights, Q/K/V,
 *     attention, outputs float32).  VGGTX_BF16 takes bfloat16 weights and runs
 *     GEMMs and attention on bfloat16 operands with float32 accumulation, float32
 *     softmax statistics and a float32 residual stream.  VGGTX_FP8_E4M3 is
 *     VGGTX_BF16 with global attention computed on OCP FP8 E4M3 Q, K, V and
 *     probabilities, with one power-of-two (OCP E8M0) scale per 128-row block
 *     of each sequence (see vggtx_quantize_fp8).
 */
#ifndef VGGTX_H
#define VGGTX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VGGTX_OK = 0,
  VGGTX_E_INVALID = 1,     /* bad shape, null pointer, bad layer list, bad offsets */
  VGGTX_E_UNSUPPORTED = 2, /* head_dim != 64, dim or mlp_hidden not a multiple of 128, not gfx950 */
  VGGTX_E_WORKSPACE = 3,   /* workspace pointer null or smaller than required */
  VGGTX_E_HIP = 4,         /* a HIP call failed (message in vggtx_last_error) */
  VGGTX_E_NODEVICE = 5     /* no usable GPU / bad device ordinal */
} vggtx_status;

typedef enum { VGGTX_F32 = 0, VGGTX_BF16 = 1, VGGTX_FP8_E4M3 = 2, VGGTX_FP8_PV = 3 } vggtx_prec;

/* storage type of an output buffer */
typedef enum { VGGTX_OUT_F32 = 0, VGGTX_OUT_BF16 = 1 } vggtx_dtype;

typedef struct vggtx_ctx* vggtx_handle;

typedef struct {
  int dim;          /* C; multiple of 128 */
  int heads;        /* H; dim == heads * head_dim */
  int head_dim;     /* D; must be 64 */
  int mlp_hidden;   /* F; multiple of 128 */
  float ln_eps;     /* LayerNorm epsilon (1e-6 by default) */
  int frame_chunk;  /* frames per chunk for token-local work; results do not depend on it */
  int tokens_inplace; /* 1: vggtx_aggregate[_varlen] keep the residual stream in the caller's tokens
                         buffer (which must then be writable; it is overwritten) instead of a copy
                         in the workspace, whose size shrinks by S*P*C*4 bytes; 0: tokens are read only */
  int attn_schedule;  /* global attention work distribution (BF16, FP8_PV, FP8_E4M3; results are the same):
                         0: queue mode, as many workgroups as the GPU holds at once take (sequence, head,
                         query tile) items from a work counter in the workspace, longest sequence first;
                         1: one workgroup per item (plain grid) */
} vggtx_config;

/* Device pointers of one block's parameters: float32 for VGGTX_F32, bfloat16
 * otherwise.  Shapes: ln*_g/ln*_b [C]; w_qkv [3C, C]; b_qkv [3C]; w_o [C, C];
 * b_o [C]; w_fc1 [F, C]; b_fc1 [F]; w_fc2 [C, F]; b_fc2 [C]. */
typedef struct {
  const void *ln1_g, *ln1_b, *w_qkv, *b_qkv, *w_o, *b_o;
  const void *ln2_g, *ln2_b, *w_fc1, *b_fc1, *w_fc2, *b_fc2;
} vggtx_block_w;

/* One alternating-attention layer: frame block, then global block. */
typedef struct {
  vggtx_block_w frame;
  vggtx_block_w global;
} vggtx_pair_w;

/* Row layout of a [tokens, heads, head_dim] tensor: element (n, h, d) lives at
 * base + n * token_stride + h * head_stride + d (in elements). */
typedef struct {
  int64_t token_stride;
  int64_t head_stride;
} vggtx_layout;

/* Create a handle on `device` for model shape `cfg` (copied).  Fails with
 * VGGTX_E_NODEVICE when the device does not exist and VGGTX_E_UNSUPPORTED when
 * it is not gfx950 or the shape is outside what the kernels support. */
vggtx_status vggtx_create(vggtx_handle* h, int device, const vggtx_config* cfg);
vggtx_status vggtx_destroy(vggtx_handle h);

/* Workspace bytes that vggtx_aggregate / vggtx_aggregate_varlen / vggtx_block
 * need for `total_frames` frames of P tokens at precision `prec`. */
vggtx_status vggtx_workspace_size(vggtx_handle h, int total_frames, int P, vggtx_prec prec, size_t* bytes);

/* Aggregator forward over one scene (Sec. 3.2).
 *   tokens     device, float32 [S, P, C]; read only, unless the handle's
 *              config sets tokens_inplace: then the forward runs its residual
 *              stream in this buffer and leaves it holding the last computed
 *              layer's global-block output
 *   w          host array[depth] of per-layer weight pointers
 *   out_layers host int32 [n_out], strictly increasing, each in [0, depth)
 *   out        device [n_out, S, P, 2C] of `out_dtype`: out[i, s, p, 0:C] is the
 *              frame-block output and out[i, s, p, C:2C] the global-block output
 *              of layer out_layers[i]
 *   ws         device workspace of at least vggtx_workspace_size bytes
 * Layers after the last requested one are not run. */
vggtx_status vggtx_aggregate(vggtx_handle h, const float* tokens, int S, int P,
                             const vggtx_pair_w* w, int depth,
                             const int32_t* out_layers, int n_out,
                             void* out, vggtx_dtype out_dtype, vggtx_prec prec,
                             void* ws, size_t ws_bytes, void* stream);

/* Same over several independent scenes stored back to back: frames of scene i
 * are frame_offsets[i] .. frame_offsets[i+1]-1 (host int32 [n_scenes+1],
 * frame_offsets[0] == 0, non-decreasing; an empty scene contributes nothing).  Global attention of a token is
 * restricted to the tokens of its own scene; all scenes run in the same
 * launches. */
vggtx_status vggtx_aggregate_varlen(vggtx_handle h, const float* tokens,
                                    const int32_t* frame_offsets, int n_scenes, int P,
                                    const vggtx_pair_w* w, int depth,
                                    const int32_t* out_layers, int n_out,
                                    void* out, vggtx_dtype out_dtype, vggtx_prec prec,
                                    void* ws, size_t ws_bytes, void* stream);

/* Graph mode of vggtx_aggregate and vggtx_aggregate_varlen (Sec. 4.3 runs
 * the same forward shape over many scenes; graphs remove its per-launch host
 * cost).  With enable = 1, each call records its kernel launches on the host
 * instead of enqueueing them and runs them as one HIP graph held by the
 * handle: the first call of a given structure (the same kernels, launch
 * shapes and argument sizes in order: same frame counts, P, layer list,
 * precision and config) builds and instantiates the graph; later calls of
 * that structure update the arguments of the nodes whose arguments changed
 * (so reallocated tokens, weights, outputs or workspace are followed without
 * a rebuild) and launch it on `stream`.  Results are bitwise those of direct
 * calls.  At most 8 graphs are kept (least recently used evicted); enable = 0
 * destroys them.  Kernel timing (vggtx_timing_enable) does not see graph
 * launches.  Errors: VGGTX_E_INVALID for a null handle or enable not 0/1. */
vggtx_status vggtx_graph_mode(vggtx_handle h, int enable);
/* stats (host int64 [4]): graphs held, graphs built, node argument updates,
 * graph launches, counted since the handle was created. */
vggtx_status vggtx_graph_stats(vggtx_handle h, int64_t* stats);

/* One transformer block (the unit both halves of a layer are made of) over
 * `n_seq` sequences back to back; token offsets host int32 [n_seq+1]
 * (non-decreasing, offsets[0] == 0).  Attention of a token is restricted to its
 * own sequence.  x_in and x_out are device float32 [n_tokens, C] and may be the
 * same buffer.  The workspace must hold vggtx_workspace_size(h, n_seq,
 * longest sequence, prec) bytes. */
vggtx_status vggtx_block(vggtx_handle h, const float* x_in, float* x_out,
                         const int32_t* seq_offsets, int n_seq,
                         const vggtx_block_w* w, vggtx_prec prec,
                         void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes that vggtx_attn_global needs for the sequences
 * seq_offsets[0..n_seq] (host int32, token offsets) of H heads of dimension D
 * at precision `prec`; for vggtx_attn_frame pass the frame offsets f * P. */
vggtx_status vggtx_attn_workspace_size(vggtx_handle h, const int32_t* seq_offsets, int n_seq, int H, int D,
                                       vggtx_prec prec, size_t* bytes);

/* Frame attention (Sec. 3.2: attention restricted to the P tokens of each of S
 * frames): o = softmax(q k^T / sqrt(D)) v per frame and head.
 *   q, k, v  device [S*P, H, D] with layout `in_layout`: bfloat16 for
 *            VGGTX_BF16, float32 for VGGTX_F32 (VGGTX_FP8_E4M3 is not offered
 *            for frame attention)
 *   o        device, same element type, layout `out_layout`. */
vggtx_status vggtx_attn_frame(vggtx_handle h, const void* q, const void* k, const void* v, void* o,
                              int S, int P, int H, int D,
                              vggtx_layout in_layout, vggtx_layout out_layout, vggtx_prec prec,
                              void* ws, size_t ws_bytes, void* stream);

/* Global attention (Sec. 3.2: attention over all tokens of a scene), streamed:
 * no score matrix is stored.  Sequence i covers tokens seq_offsets[i] ..
 * seq_offsets[i+1]-1 (host int32 [n_seq+1], seq_offsets[0] == 0, non-
 * decreasing; empty sequences are skipped).  q, k, v: bfloat16 for VGGTX_BF16 and VGGTX_FP8_E4M3 (the
 * library quantises them into the workspace), float32 for VGGTX_F32; o has
 * the same element type as q. */
vggtx_status vggtx_attn_global(vggtx_handle h, const void* q, const void* k, const void* v, void* o,
                               const int32_t* seq_offsets, int n_seq, int H, int D,
                               vggtx_layout in_layout, vggtx_layout out_layout, vggtx_prec prec,
                               void* ws, size_t ws_bytes, void* stream);

/* Global attention for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation, arguments and results as vggtx_attn_global, with no
 * workspace argument.  The transposed V (VGGTX_BF16) or the E4M3 codes and
 * block scales (VGGTX_FP8_E4M3) go to a fixed device array of
 * VGGTX_NOALLOC_SCRATCH_BYTES bytes inside the library, one per device, held
 * until the process ends; the call itself allocates nothing (no hipMalloc,
 * hipFree or allocating library routine) and records no kernel timing.
 * Returns VGGTX_E_WORKSPACE, having enqueued nothing, when the sequences need
 * more scratch than that (vggtx_attn_workspace_size gives the need; 64 MiB
 * hold about 32,000 tokens of 16 heads in BF16 and 21,000 in FP8).  Every
 * call on one device shares that device's array and overwrites it entirely
 * before reading it (nothing in it needs to start at zero), so calls that
 * overlap in time on one device, from any stream or handle, race: the caller
 * orders them (one stream, or events between streams). */
#define VGGTX_NOALLOC_SCRATCH_BYTES (64u << 20)
vggtx_status vggtx_attn_global_noalloc(vggtx_handle h, const void* q, const void* k, const void* v, void* o,
                                       const int32_t* seq_offsets, int n_seq, int H, int D,
                                       vggtx_layout in_layout, vggtx_layout out_layout, vggtx_prec prec,
                                       void* stream);

/* FP8 E4M3 quantiser used by the FP8 global attention.  x: device bfloat16
 * [n_tokens, H, D] with layout `in_layout`.  For every head and every
 * 128-token block of every sequence (blocks start at each sequence start; the
 * last block of a sequence may be shorter): s = 2^e, e the smallest integer
 * with amax <= 448 * 2^e (clamped to [-127, 127]; s = 1 when amax == 0), and
 * codes = E4M3 round-to-nearest-even of x / s (exact scaling, so the E4M3
 * rounding is the only one).  s is an OCP E8M0 block scale.  The attention
 * path quantises Q after multiplying it by log2(e)/sqrt(D) in float32.
 *   codes  device uint8 [H, n_tokens, D]
 *   scales device float32 [H, n_blocks], n_blocks = sum_i ceil(len_i / 128),
 *          blocks numbered sequence by sequence. */
vggtx_status vggtx_quantize_fp8(vggtx_handle h, const void* x, vggtx_layout in_layout,
                                const int32_t* seq_offsets, int n_seq, int H, int D,
                                uint8_t* codes, float* scales, void* stream);

/* Attention autotuner.  Times every compiled tile variant of the attention
 * kernel for `prec` (VGGTX_BF16: variants 0..2 = (query blocks of 32 rows per
 * wave, waves per workgroup) (1,4), (2,4), (1,8); VGGTX_FP8_E4M3: variants 0..3 = (query blocks
 * per wave, waves per workgroup) (1,4), (2,4), (1,8), (2,8)) on synthetic
 * Q, K, V written into the
 * caller's workspace (one sequence of `n_tokens` tokens, 16 heads of 64; a
 * truncated problem of 8192 to 65536 tokens is representative since the kernels
 * are compute bound) and keeps the fastest in the handle for all later calls.
 * The workspace must hold vggtx_autotune_workspace_size() bytes; the call
 * synchronises `stream`.  *chosen receives the variant index.  If the
 * environment variable VGGTX_AUTOTUNE_CACHE names a file, a previously stored
 * choice for (device architecture, prec) is reused without timing, and a new
 * choice is appended to it.  Results never depend on the variant: every
 * variant computes each query row with the same arithmetic in the same order. */
vggtx_status vggtx_autotune_workspace_size(vggtx_handle h, int n_tokens, size_t* bytes);
vggtx_status vggtx_autotune(vggtx_handle h, vggtx_prec prec, int n_tokens, void* ws, size_t ws_bytes, void* stream,
                            int* chosen);

/* ---------------------------------------------------------------- front end
 * Per-frame patch embedding (Sec. 3.2: every frame first goes through a
 * DINO-based patch-embedding extractor; it is intra-frame, so frames are
 * processed in chunks of `frame_chunk`, at most 2048, without changing the
 * result).  The extractor is not described in the paper; the reading built
 * here is a DINO-style ViT:
 *   patches  non-overlapping 14 x 14 pixel patches, numbered row-major over
 *            the (height/14) x (width/14) grid; patch vector entry
 *            c*196 + ky*14 + kx = pixel (c, 14*py + ky, 14*px + kx)
 *   tokens   per frame [class + pos[0], reg[0..3], W_patch p_i + b_patch +
 *            pos[1 + i] for every patch i]  (Pd = 5 + n_patches tokens)
 *   blocks   `depth` blocks of the aggregator's kind, attention over the Pd
 *            tokens of one frame, then a final LayerNorm (norm_g, norm_b)
 *   output   the aggregator input: per frame [cam[s], agg_reg[s][0..3], the
 *            normalised patch tokens], s = 0 for the first frame of a scene
 *            and 1 for the others (P = Pd tokens per frame).
 * A LayerScale on a block's residual branches, if a model has one, is folded
 * into that block's w_o / b_o and w_fc2 / b_fc2 rows by the caller.
 *
 * Device pointers, float32 for VGGTX_F32 and bfloat16 otherwise:
 *   w_patch [C, 588] (a Conv2d weight [C, 3, 14, 14] flattened), b_patch [C],
 *   pos [1 + n_patches, C], cls [C], reg [4, C], norm_g / norm_b [C],
 *   cam [2, C], agg_reg [2, 4, C]; blocks: host array [depth] (may be null
 *   when depth == 0). */
typedef struct {
  const void *w_patch, *b_patch, *pos, *cls, *reg;
  const vggtx_block_w* blocks;
  int depth;
  const void *norm_g, *norm_b, *cam, *agg_reg;
} vggtx_embed_w;

/* Workspace bytes vggtx_embed needs for `total_frames` frames of
 * height x width pixels (it holds one chunk of frames, not all of them). */
vggtx_status vggtx_embed_workspace_size(vggtx_handle h, int total_frames, int height, int width, vggtx_prec prec,
                                        size_t* bytes);

/* Front end over the frames of n_scenes scenes stored back to back:
 *   images        device float32 [S, 3, height, width] (normalised pixels);
 *                 height and width positive multiples of 14
 *   frame_offsets host int32 [n_scenes + 1], frame_offsets[0] == 0,
 *                 non-decreasing, S = frame_offsets[n_scenes]
 *   tokens        device float32 [S, 5 + n_patches, C], written in full
 * VGGTX_BF16 runs the blocks as in the aggregator (bfloat16 operands, float32
 * residual); VGGTX_FP8_E4M3 behaves as VGGTX_BF16 here (the front end has no
 * global attention); VGGTX_F32 runs in float32. */
vggtx_status vggtx_embed(vggtx_handle h, const float* images, int height, int width,
                         const int32_t* frame_offsets, int n_scenes, const vggtx_embed_w* w,
                         float* tokens, vggtx_prec prec, void* ws, size_t ws_bytes, void* stream);

/* Prediction-head inputs (Sec. 3.2: the heads consume the kept layers'
 * outputs).  For every kept layer l and frame s: out[l, s, c, y, x] =
 * feats[l, s, 5 + y * grid_w + x, c], c < 2C: the patch tokens behind the 5
 * special tokens as a channels-first grid_h x grid_w map.
 *   feats  device [n_out, S, P, 2C] of `dtype` (the vggtx_aggregate output),
 *          P = 5 + grid_h * grid_w, 16-byte aligned
 *   out    device [n_out, S, 2C, grid_h, grid_w] of the same type
 * n_out * S must not exceed 65535. */
vggtx_status vggtx_pack_head_inputs(vggtx_handle h, const void* feats, vggtx_dtype dtype, int n_out, int S, int P,
                                    int grid_h, int grid_w, void* out, void* stream);

/* ---------------------------------------------------------------- global alignment
 * Camera global alignment (Sec. 3.3): refine every camera by minimising the
 * weighted mean epipolar residual of Eq. (epi) over the correspondences of
 * the image pairs, with the weights of Eq. (weight) and the learning-rate
 * rule of Eq. (lr).  The paper leaves the details open; the reading built
 * here (float64 throughout):
 *   camera     x_cam = R X + t; pixel = (f x/z + cx, f y/z + cy); the
 *              principal point is fixed, R, t and f are refined
 *   residual   e = |x'^T F x| / |(F x)_{0,1}|, the pixel distance of x' from
 *              the epipolar line of x; F = Kj^-T [t_ij]x R_ij Ki^-1 with
 *              R_ij = Rj Ri^T, t_ij = tj - R_ij ti for the pair (i, j)
 *   weights    from the residuals of the initial cameras: histogram of bins
 *              of 0.1 px over [0, 20) plus an overflow bin of density 0;
 *              f(b) = count_b / (K * 0.1), w = (f / Avg_k f(e_k))^alpha
 *              (all weights 1 when no residual is below 20 px)
 *   rate       the bin of the ceil(K/2)-th smallest initial residual picks
 *              lr[0] (median < bounds[0]), lr[1] (< bounds[1]) or lr[2]
 *   optimiser  Adam on (unnormalised quaternion, t, log f) per camera,
 *              `iterations` steps, weights and rate fixed
 * Degenerate pairs (coincident camera centres, F = 0) are not supported. */
typedef struct {
  int iterations;     /* 300 */
  double lr[3];       /* 5e-4, 1e-3, 1e-2 */
  double bounds[2];   /* 2.5, 7.5 pixels; multiples of 0.1 in [0, 20] */
  double alpha;       /* 0.5 */
  double beta1, beta2, eps;  /* Adam: 0.9, 0.999, 1e-8 */
} vggtx_ga_config;

/* The paper's settings (Sec. 4.1) and Adam's usual constants. */
void vggtx_ga_config_default(vggtx_ga_config* cfg);

/* Candidate pairs (Sec. 3.3: views that differ by less than max_angle_deg,
 * 30 in Sec. 4.1), the angle being that between the optical axes (third rows
 * of R).  Host-only: R is host float64 [n_cams, 3, 3]; pairs receives (i, j),
 * i < j, in row-major order of (i, j) when it is not null.  *n_pairs receives
 * the number of pairs; VGGTX_E_INVALID when pairs is not null and more than
 * max_pairs exist (nothing is written then). */
vggtx_status vggtx_ga_select_pairs(const double* R, int n_cams, double max_angle_deg, int32_t* pairs, int max_pairs,
                                   int* n_pairs);

/* Workspace bytes vggtx_ga_align needs. */
vggtx_status vggtx_ga_workspace_size(vggtx_handle h, int n_cams, int n_pairs, int64_t n_corr, size_t* bytes);

/* Global alignment.
 *   R0, t0, f0, pp  device float64 [n_cams,3,3], [n_cams,3], [n_cams], [n_cams,2]: the
 *                   predicted cameras (f0 > 0) and their principal points
 *   pairs           host int32 [n_pairs, 2], camera indices i != j
 *   corr_offsets    host int64 [n_pairs + 1], 0 = first, non-decreasing: the
 *                   correspondences of pair m are rows corr_offsets[m] ..
 *                   corr_offsets[m+1]-1 of corr
 *   corr            device float32 [n_corr, 4] = (u, v, u', v'): pixel x in
 *                   camera i and x' in camera j; 16-byte aligned
 *   R_out, t_out, f_out  device float64, the refined cameras (same shapes)
 *   weights_out     device float32 [n_corr] or null: w of every correspondence
 *   loss_out        device float64 [iterations + 1] or null: the loss before
 *                   each step and after the last one
 * The host tables are copied into the workspace and `stream` is synchronised
 * once before the kernels are enqueued, so the host arrays may be released
 * when the call returns; the alignment itself runs asynchronously. */
vggtx_status vggtx_ga_align(vggtx_handle h, const vggtx_ga_config* cfg, int n_cams, const double* R0,
                            const double* t0, const double* f0, const double* pp, const int32_t* pairs,
                            int n_pairs, const int64_t* corr_offsets, const float* corr, double* R_out,
                            double* t_out, double* f_out, float* weights_out, double* loss_out, void* ws,
                            size_t ws_bytes, void* stream);

/* Pose accuracy AUC@30 (the paper's appendix).  For every ordered pair (i, j),
 * i != j (both_orders != 0, the paper's permutation-equivariant form) or
 * i < j only (the conventional form): relative poses E_i^-1 E_j =
 * (R_i^T R_j, R_i^T (t_j - t_i)) of the prediction and the ground truth;
 * error = max(rotation angle of dR_pred^T dR_gt, angle between dt_pred and
 * dt_gt (0 if either is zero)) in degrees.  AUC@30 = mean over tau = 1..30
 * of the fraction of pairs with error < tau.
 *   R_pred, t_pred, R_gt, t_gt  device float64 [n,3,3], [n,3] (n*n < 2^31)
 *   counts  device uint32 [31]: errors in [b, b+1) degrees, counts[30] >= 30
 *   auc     device float64 [1] or null */
vggtx_status vggtx_auc30(vggtx_handle h, const double* R_pred, const double* t_pred, const double* R_gt,
                         const double* t_gt, int n, int both_orders, uint32_t* counts, double* auc, void* stream);

/* Kernel timing (tracing).  While enabled, every kernel launch of the classes
 * below is bracketed by a pair of HIP events recorded on its launch stream, and
 * vggtx_timing_read() waits for those events and returns, per class, the summed
 * elapsed time, the number of launches and the algorithmic work of those
 * launches (attention: 4 * D * H * sum of sequence length squared flops; GEMMs:
 * 2 * M * N * K flops).  At most 262144 launches are recorded between reads;
 * later ones are counted in `dropped`.  Enabling or reading clears the record.
 * The events are host-side objects of the handle; no device memory is
 * allocated. */
typedef enum {
  VGGTX_K_ATTN_GLOBAL = 0, /* global attention (any precision) */
  VGGTX_K_ATTN_FRAME = 1,  /* frame attention */
  VGGTX_K_GEMM = 2,        /* projection / MLP GEMMs with their fused epilogues */
  VGGTX_K_OTHER = 3,       /* LayerNorm, V transposition, FP8 quantisation, copies */
  VGGTX_K_COUNT = 4
} vggtx_kernel_class;

typedef struct {
  double total_ms;
  int64_t launches;
  double flops;
} vggtx_timing;

vggtx_status vggtx_timing_enable(vggtx_handle h, int enable);
vggtx_status vggtx_timing_read(vggtx_handle h, vggtx_timing out[VGGTX_K_COUNT], int64_t* dropped);
/* Non-blocking progress query: of the launches recorded since the last
 * enable/read, how many have finished (in issue order) and how many of those
 * were global-attention launches.  Does not wait and does not clear.  Unlike
 * the other entry points it may be called from a second thread while a call
 * on the same handle is still enqueueing work (a long forward can block its
 * caller inside the launch queue). */
vggtx_status vggtx_timing_poll(vggtx_handle h, int64_t* finished, int64_t* recorded, int64_t* finished_attn_global);

const char* vggtx_status_str(vggtx_status s);
/* Message of the last failing call on this thread ("" if none). */
const char* vggtx_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* VGGTX_H */
