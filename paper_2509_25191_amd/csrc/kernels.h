// Host-visible launchers of the vggtx HIP kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"
#include "launch.h"

namespace vggtx {

// Sequence structure of one attention launch.  Either `uniform` (n_seq
// sequences of `len` tokens back to back from token `base`) or an explicit
// list (at most kMaxSeqInline entries) in processing order; the list is
// ordered longest-first so that the biggest scenes start first.
struct SeqTable {
  int n_seq;
  int uniform;
  int len;             // uniform: tokens per sequence
  int base;            // uniform: first token
  int tiles_per_seq;   // uniform: query tiles per sequence
  int start[kMaxSeqInline];     // list: first token
  int end[kMaxSeqInline];       // list: one past the last token
  int vt_base[kMaxSeqInline];   // list: padded column of the first token in transposed V
  int blk_base[kMaxSeqInline];  // list: first FP8 scale block
  int tile_end[kMaxSeqInline];  // list: inclusive prefix sum of query tiles
};

struct AttnParams {
  const void* q; int64_t q_ts, q_hs;     // [tokens, H, D] strides in elements
  const void* k; int64_t k_ts, k_hs;
  const void* v; int64_t v_ts, v_hs;     // key-major V (float32 kernel)
  const void* vt; int64_t vt_hs, vt_ds;  // transposed, padded V: (h, d, col) at h*vt_hs + d*vt_ds + col
  void* o; int64_t o_ts, o_hs;
  // FP8 scales: [H, n_blocks] (per-head stride sc_hs)
  const float* sq; const float* sk; const float* sv; int64_t sc_hs;
  const float* vmax;                     // FP8: per-head max of the V scales
  const int* kinfo;                      // FP8: per (head, key block) E8M0 codes, 2 ints each (launch_scale_max)
  float scale_log2;                      // log2(e) / sqrt(D)
  int n_items;                           // query tiles per head
  // Queue mode (BF16, FP8 P V and FP8 kernels): queue != null points at a
  // work counter in device memory; the launcher zeroes it, and each of the
  // n_heads * n_items workgroups takes its work item from it when it starts
  // (longest sequence first, see take_work).  Null: workgroup (x, y) runs
  // item x of head y.
  int* queue;
  int n_heads;
  SeqTable seqs;
};

// ---- attention (attention.hip)
// BF16 variants: (query blocks of 32 rows per wave, waves) 0 = (1, 4), 1 = (2, 4), 2 = (1, 8)
hipError_t launch_attn_bf16(const AttnParams& p, int H, int variant, hipStream_t s);
// Global attention with bfloat16 scores and E4M3 P V (same tile variants as BF16)
hipError_t launch_attn_fp8pv(const AttnParams& p, int H, int variant, hipStream_t s);
hipError_t launch_attn_f32(const AttnParams& p, int H, hipStream_t s);
// FP8 variants: 0 = (1 query block per wave, 4 waves), 1 = (2, 4), 2 = (1, 8), 3 = (2, 8)
hipError_t launch_attn_fp8(const AttnParams& p, int H, int variant, hipStream_t s);
int attn_n_variants(int prec);              // kernel variants of a precision (1 = BF16, 2 = FP8)
int attn_block_rows(int prec, int variant);  // query rows per work item of a kernel variant

// Transposed, zero-padded copy of V: v [tokens, H, D] (bf16 or u8 codes) ->
// vt [H, D, padded tokens].
hipError_t launch_v_transpose_bf16(const bf16* v, int64_t v_ts, int64_t v_hs, bf16* vt, int64_t vt_hs,
                                   int64_t vt_ds, const SeqTable& seqs, int n_tiles, int H, hipStream_t s);

// FP8 quantiser: x [tokens, H, D] bf16, times the float32 factor `pre`, ->
// codes and per-(head, 128-row block) power-of-two scales.
// transposed == false: codes [H, tokens, D] (row-major, c_hs = tokens*D);
//   token t of the table lands in code row out_row0 + t
// transposed == true:  codes [H, D, padded tokens] like vt above (zero padding).
hipError_t launch_quant_fp8(const bf16* x, int64_t x_ts, int64_t x_hs, float pre, uint8_t* codes, int64_t c_hs,
                            int64_t c_ds, bool transposed, int64_t out_row0, float* scales, int64_t sc_hs,
                            const SeqTable& seqs, int n_blocks, int H, hipStream_t s);
// Per-head max of the V block scales -> vmax[H], then per key block b the
// E8M0 codes kinfo[h][b] = {E8M0(s_k(b)), E8M0(s_v(b) / vmax[h])}.
hipError_t launch_scale_max(const float* sk, const float* sv, int64_t sc_hs, int n_blocks, float* vmax, int* kinfo,
                            int H, hipStream_t s);

// ---- GEMMs (gemm.hip): C[M, N] = A[M, K] W[N, K]^T + bias, then an epilogue
enum Epi { EPI_QKV = 0, EPI_RESID = 1, EPI_GELU = 2, EPI_EMBED = 3 };

struct GemmParams {
  const void* a; int64_t lda;      // A rows (bf16 or f32), row-major with leading dimension lda, or
  int64_t a_hs;                    // when a_hs != 0: head-major, A(m, k) at a[(k / 64) * a_hs + m * 64 + k % 64]
  const void* w;                   // W [N, K] row-major (bf16 or f32)
  const void* bias;                // [N] (bf16 or f32)
  int M, N, K;
  int row0;                        // global token index of A's first row
  // EPI_QKV: part j of [q | k | v] (C = H*D columns each), head h, A's row r,
  // dimension d goes to qkv[j][h * qkv_hs[j] + r * D + d] (bf16 or f32); the q
  // part is multiplied by q_scale before it is stored
  void* qkv[3]; int64_t qkv_hs[3]; int C; float q_scale;
  // EPI_RESID: x[row0 + r, c] += result (float32, leading dim ldx); optional copy to out
  float* x; int64_t ldx;
  void* out; int64_t ldo; int out_f32;
  // EPI_GELU: hid[r, c] = gelu(result)
  void* hid; int64_t ldh;
  // EPI_RESID with stats != null: the epilogue also writes, for every row it
  // updates, the (mean, M2) pair of the new residual over its 128-column
  // output slice, at stats[((row0 + r) * N / 128 + n0 / 128) * 2]
  // (ln_apply_kernel combines the pairs of a row into its LayerNorm).
  float* stats;
  // EPI_EMBED: A row m is patch i = m % emb_np of frame f = m / emb_np;
  // x[f * emb_pd + kEmbedSpecial + i, c] = result + pos[1 + i, c] (pos [.., N], bias type)
  const void* pos; int emb_np, emb_pd;
};

hipError_t launch_gemm_bf16(const GemmParams& p, Epi epi, hipStream_t s);
hipError_t launch_gemm_f32(const GemmParams& p, Epi epi, hipStream_t s);

// ---- LayerNorm (elementwise.hip): h[r] = LN(x[row0 + r]) for r < rows
hipError_t launch_layernorm(const float* x, int64_t ldx, const void* g, const void* b, float eps, void* h,
                            int64_t ldh, int rows, int C, bool bf16_io, hipStream_t s);
hipError_t launch_copy_f32(const float* src, float* dst, int64_t n, hipStream_t s);
// Per-row (mean, M2) of every 128-column slice of x [rows, C] -> stats [rows, C / 128, 2]
hipError_t launch_row_stats(const float* x, int64_t ldx, int rows, int C, float* stats, hipStream_t s);
// h[r] = bf16 LayerNorm of x[r] from the slice statistics of row srow0 + r (g, b bf16)
hipError_t launch_ln_apply(const float* x, int64_t ldx, const float* stats, int64_t srow0, const void* g, const void* b,
                           float eps, void* h, int64_t ldh, int rows, int C, hipStream_t s);

// ---- patch-embedding front end (embed.hip)
constexpr int kEmbedPatch = 14;                          // patch side in pixels
constexpr int kEmbedSpecial = 5;                         // class / camera token + 4 registers per frame
constexpr int kEmbedK = 3 * kEmbedPatch * kEmbedPatch;   // 588 values per patch
constexpr int kEmbedKp = 640;                            // kEmbedK padded to the GEMM's k-step (64)
constexpr int kEmbedMaxChunk = 2048;                     // frames per front-end chunk (bits of FirstMask)
struct FirstMask {
  uint32_t w[kEmbedMaxChunk / 32];  // bit f: chunk frame f is the first frame of a scene
};
hipError_t launch_pad_cols(const void* w, void* wp, int rows, int K, int Kp, bool bf16_io, hipStream_t s);
hipError_t launch_patchify(const float* img, int height, int width, int64_t f0, int n_frames, void* a, int Kp,
                           bool bf16_io, hipStream_t s);
hipError_t launch_embed_special(const void* pos, const void* cls, const void* reg, float* x, int n_frames, int Pd,
                                int C, bool bf16_io, hipStream_t s);
hipError_t launch_pack_heads(const void* feats, bool bf16_io, int n_ls, int P, int C2, int n_patch, void* out,
                             hipStream_t s);
hipError_t launch_embed_finish(const float* x, int Pd, const void* g, const void* b, float eps, const void* cam,
                               const void* agg_reg, float* out, int64_t f0, int n_frames, const FirstMask& first,
                               int C, bool bf16_io, hipStream_t s);
hipError_t launch_fill_hash_bf16(bf16* x, int64_t n, uint64_t seed, float scale, hipStream_t s);

// ---- camera global alignment (ga.hip)
constexpr int kGaBins = 200;               // residual histogram: bins of 1/kGaBinsPerPixel px over [0, 20)
constexpr double kGaBinsPerPixel = 10.0;   // (+1 overflow bin for e >= 20 px)
enum GaMode { GA_MODE_BINS = 0, GA_MODE_GRAD = 1, GA_MODE_LOSS = 2 };
struct GaParams {
  const int* pairs;         // [n_pairs, 2] camera indices (i, j)
  const int64_t* offsets;   // [n_pairs + 1] correspondence offsets
  const float* corr;        // [n_corr, 4] (u, v, u', v'), 16-byte aligned
  const double* f0;         // [n_cams] initial focal lengths
  const double* pp;         // [n_cams, 2] principal points
  double* p;                // [n_cams, 8] parameters (q, t, phi)
  double* adam;             // [n_cams, 16] first / second moments
  uint8_t* bins;            // [n_corr] histogram bin of the initial residual
  uint32_t* hist;           // [kGaBins + 1] bin counts
  const double* table;      // [kGaBins + 1] weight of a bin
  double* scal;             // [0] learning rate, [1] total weight W, [2] median bin
  double* pair_gf;          // [n_pairs, 9] sum_k w_k de_k/dF
  double* pair_grad;        // [n_pairs, 16] gradient w.r.t. (camera i, camera j) parameters
  double* pair_loss;        // [n_pairs] sum_k w_k e_k
  const int* inc_off;       // [n_cams + 1] CSR of the pair sides of each camera
  const int* inc;           // [2 n_pairs] pair << 1 | side
};
hipError_t launch_ga_init(const double* R0, const double* t0, int n_cams, double* p, double* adam, hipStream_t s);
hipError_t launch_ga_pairs(const GaParams& a, int n_pairs, int mode, hipStream_t s);
hipError_t launch_ga_chain(const GaParams& a, int n_pairs, hipStream_t s);
hipError_t launch_ga_table(const uint32_t* hist, double alpha, int lr_bin1, int lr_bin2, double lr0, double lr1,
                           double lr2, double* table, double* scal, hipStream_t s);
hipError_t launch_ga_adam(const GaParams& a, int n_cams, int step, double beta1, double beta2, double eps,
                          hipStream_t s);
hipError_t launch_ga_loss(const double* pair_loss, int n_pairs, const double* scal, double* out, hipStream_t s);
hipError_t launch_ga_out(const double* p, const double* f0, int n_cams, double* R_out, double* t_out, double* f_out,
                         hipStream_t s);
hipError_t launch_ga_weights(const uint8_t* bins, const double* table, int64_t n, float* w, hipStream_t s);
hipError_t launch_ga_zero_u32(uint32_t* x, int n, hipStream_t s);
constexpr int kAucBins = 31;  // AUC@30 error bins: [b, b+1) degrees for b < 30, then >= 30
hipError_t launch_auc30(const double* Rp, const double* tp, const double* Rg, const double* tg, int n, int both_orders,
                        uint32_t* counts, double* auc, hipStream_t s);

}  // namespace vggtx
