// Per-frame patch-embedding front end (arXiv 2509.25191, Sec. 3.2: a
// DINO-based patch embedding of every frame, intra-frame only, so frames are
// processed in chunks).  The pieces around the transformer blocks:
//   patchify        images -> patch matrix (the operand of one GEMM whose
//                   EPI_EMBED epilogue adds bias and position embedding and
//                   scatters the patch tokens into the token rows)
//   embed_special   class token (+ its position embedding) and register tokens
//   embed_finish    final LayerNorm of the patch tokens, written as aggregator
//                   input rows, with the camera / register tokens in front
// All three are memory-bound elementwise passes over the chunk.  The file also
// holds the head-input packing (pack_heads), the token-to-map layout change on
// the other side of the aggregator.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace vggtx {

static inline unsigned grid_for(int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 65536); }

// wp[r][k] = w[r][k] for k < K and 0 for K <= k < Kp.
template <typename T>
__global__ __launch_bounds__(256) void pad_cols_kernel(const T* w, T* wp, int rows, int K, int Kp) {
  const int64_t n = (int64_t)rows * Kp;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int64_t r = i / Kp;
    const int k = (int)(i - r * Kp);
    wp[i] = k < K ? w[r * K + k] : (T)0.f;
  }
}

// Patch matrix of frames [f0, f0 + n_frames) of images [S, 3, height, width]:
// row (f - f0) * n_patch + py * gw + px, column c * 196 + ky * 14 + kx holds
// pixel (c, 14 py + ky, 14 px + kx) of frame f; columns 588 .. Kp-1 are zero.
template <typename T>
__global__ __launch_bounds__(256) void patchify_kernel(const float* img, int height, int width, int64_t f0,
                                                       int n_frames, T* a, int Kp) {
  constexpr int PP = kEmbedPatch * kEmbedPatch;
  const int gw = width / kEmbedPatch, n_patch = (height / kEmbedPatch) * gw;
  const int64_t n = (int64_t)n_frames * n_patch * Kp;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int64_t row = i / Kp;
    const int k = (int)(i - row * Kp);
    float v = 0.f;
    if (k < kEmbedK) {
      const int64_t fl = row / n_patch;
      const int p = (int)(row - fl * n_patch);
      const int py = p / gw, px = p - py * gw;
      const int c = k / PP, rem = k - c * PP;
      const int ky = rem / kEmbedPatch, kx = rem - ky * kEmbedPatch;
      const int64_t plane = (f0 + fl) * 3 + c;
      v = img[(plane * height + py * kEmbedPatch + ky) * (int64_t)width + px * kEmbedPatch + kx];
    }
    a[i] = (T)v;
  }
}

// Rows f * Pd + j of the chunk's residual stream, j < kEmbedSpecial: the class
// token plus position-embedding row 0 (j = 0), then the register tokens.
template <typename T>
__global__ __launch_bounds__(256) void embed_special_kernel(const T* pos, const T* cls, const T* reg, float* x,
                                                            int n_frames, int Pd, int C) {
  const int64_t n = (int64_t)n_frames * kEmbedSpecial * C;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int64_t fj = i / C;
    const int c = (int)(i - fj * C);
    const int64_t f = fj / kEmbedSpecial;
    const int j = (int)(fj - f * kEmbedSpecial);
    const float v = j == 0 ? ldf(cls + c) + ldf(pos + c) : ldf(reg + (int64_t)(j - 1) * C + c);
    x[(f * Pd + j) * C + c] = v;
  }
}

// One wave per token row of the chunk.  Patch rows: LayerNorm (float32 mean
// and biased variance, two passes over the row in registers) into the output
// token row.  Special rows: the camera token (j = 0) or register token j - 1
// of set 0 (first frame of a scene, bit set in `first`) or set 1.
template <int NPL, typename T>
__global__ __launch_bounds__(256) void embed_finish_kernel(const float* x, int Pd, const T* g, const T* b, float eps,
                                                           const T* cam, const T* agg_reg, float* out, int64_t f0,
                                                           int n_frames, FirstMask first) {
  constexpr int C = NPL * 64;
  const int lane = threadIdx.x & 63;
  const int64_t row = blockIdx.x * 4ll + (threadIdx.x >> 6);
  if (row >= (int64_t)n_frames * Pd) return;
  const int f = (int)(row / Pd), t = (int)(row - (int64_t)f * Pd);
  float* o = out + ((f0 + f) * Pd + t) * (int64_t)C;
  if (t < kEmbedSpecial) {
    const int set = ((first.w[f >> 5] >> (f & 31)) & 1u) ? 0 : 1;
    const T* src = t == 0 ? cam + (int64_t)set * C : agg_reg + ((int64_t)set * (kEmbedSpecial - 1) + (t - 1)) * C;
#pragma unroll
    for (int j = 0; j < NPL; ++j) o[lane + 64 * j] = ldf(src + lane + 64 * j);
    return;
  }
  const float* xr = x + row * C;
  float v[NPL];
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < NPL; ++j) {
    v[j] = xr[lane + 64 * j];
    s += v[j];
  }
  const float mean = wave_sum(s) * (1.f / C);
  float q = 0.f;
#pragma unroll
  for (int j = 0; j < NPL; ++j) {
    const float d = v[j] - mean;
    q += d * d;
  }
  const float rstd = 1.f / __builtin_sqrtf(wave_sum(q) * (1.f / C) + eps);
#pragma unroll
  for (int j = 0; j < NPL; ++j) {
    const int c = lane + 64 * j;
    o[c] = (v[j] - mean) * rstd * ldf(g + c) + ldf(b + c);
  }
}

// Head inputs (the prediction heads read the kept layers' patch tokens as
// channels-first maps): for every (layer, frame) the patch rows [n_patch, C2]
// behind the special tokens are transposed to [C2, n_patch].  One workgroup
// per 256-token x 32-channel tile: every token's 32 channels are one full
// 64-byte segment (bf16), read with 16-byte loads, and every output row
// receives 256 contiguous tokens, so that only the two ends of each run are
// partial lines.  The tile is transposed in LDS (channel-major).
template <typename T>
__global__ __launch_bounds__(256) void pack_heads_kernel(const T* feats, int P, int C2, int n_patch, T* out) {
  constexpr int TT = 256, TC = 32, VEC = 16 / sizeof(T), GPR = TC / VEC;  // granules per token row
  __shared__ T tile[TC][TT + 2];
  const int t0 = blockIdx.x * TT, c0 = blockIdx.y * TC;
  const int64_t ls = blockIdx.z;  // layer * S + frame
  const T* src = feats + (ls * P + kEmbedSpecial) * (int64_t)C2 + c0;
  T* dst = out + ls * (int64_t)C2 * n_patch;
  typedef __attribute__((__vector_size__(16))) T vec_t;
  for (int g = threadIdx.x; g < TT * GPR; g += 256) {
    const int r = g / GPR, v = g % GPR;
    vec_t x = {};
    if (t0 + r < n_patch) x = *(const vec_t*)(src + (int64_t)(t0 + r) * C2 + v * VEC);
#pragma unroll
    for (int j = 0; j < VEC; ++j) tile[v * VEC + j][r] = x[j];
  }
  __syncthreads();
  const int nt = min(TT, n_patch - t0);
  for (int i = threadIdx.x; i < TC * TT; i += 256) {
    const int c = i / TT, r = i % TT;
    if (r < nt) dst[(int64_t)(c0 + c) * n_patch + t0 + r] = tile[c][r];
  }
}

hipError_t launch_pack_heads(const void* feats, bool bf16_io, int n_ls, int P, int C2, int n_patch, void* out,
                             hipStream_t s) {
  if (n_ls <= 0 || n_patch <= 0) return hipSuccess;
  // C2 is a multiple of 32 (2 x a multiple of the 64-wide head size)
  const dim3 grid((unsigned)((n_patch + 255) / 256), (unsigned)(C2 / 32), (unsigned)n_ls);
  if (bf16_io)
    hipLaunchKernelGGL(pack_heads_kernel<bf16>, grid, dim3(256), 0, s, (const bf16*)feats, P, C2, n_patch, (bf16*)out);
  else
    hipLaunchKernelGGL(pack_heads_kernel<float>, grid, dim3(256), 0, s, (const float*)feats, P, C2, n_patch,
                       (float*)out);
  return hipGetLastError();
}

hipError_t launch_pad_cols(const void* w, void* wp, int rows, int K, int Kp, bool bf16_io, hipStream_t s) {
  const unsigned grid = grid_for((int64_t)rows * Kp);
  if (bf16_io) hipLaunchKernelGGL(pad_cols_kernel<bf16>, dim3(grid), dim3(256), 0, s, (const bf16*)w, (bf16*)wp, rows, K, Kp);
  else hipLaunchKernelGGL(pad_cols_kernel<float>, dim3(grid), dim3(256), 0, s, (const float*)w, (float*)wp, rows, K, Kp);
  return hipGetLastError();
}

hipError_t launch_patchify(const float* img, int height, int width, int64_t f0, int n_frames, void* a, int Kp,
                           bool bf16_io, hipStream_t s) {
  const int64_t n = (int64_t)n_frames * (height / kEmbedPatch) * (width / kEmbedPatch) * Kp;
  if (n <= 0) return hipSuccess;
  if (bf16_io)
    hipLaunchKernelGGL(patchify_kernel<bf16>, dim3(grid_for(n)), dim3(256), 0, s, img, height, width, f0, n_frames,
                       (bf16*)a, Kp);
  else
    hipLaunchKernelGGL(patchify_kernel<float>, dim3(grid_for(n)), dim3(256), 0, s, img, height, width, f0, n_frames,
                       (float*)a, Kp);
  return hipGetLastError();
}

hipError_t launch_embed_special(const void* pos, const void* cls, const void* reg, float* x, int n_frames, int Pd,
                                int C, bool bf16_io, hipStream_t s) {
  const int64_t n = (int64_t)n_frames * kEmbedSpecial * C;
  if (n <= 0) return hipSuccess;
  if (bf16_io)
    hipLaunchKernelGGL(embed_special_kernel<bf16>, dim3(grid_for(n)), dim3(256), 0, s, (const bf16*)pos,
                       (const bf16*)cls, (const bf16*)reg, x, n_frames, Pd, C);
  else
    hipLaunchKernelGGL(embed_special_kernel<float>, dim3(grid_for(n)), dim3(256), 0, s, (const float*)pos,
                       (const float*)cls, (const float*)reg, x, n_frames, Pd, C);
  return hipGetLastError();
}

template <typename T>
static hipError_t finish_dispatch(const float* x, int Pd, const void* g, const void* b, float eps, const void* cam,
                                  const void* agg_reg, float* out, int64_t f0, int n_frames, const FirstMask& first,
                                  int C, hipStream_t s) {
  const int64_t rows = (int64_t)n_frames * Pd;
  dim3 grid((unsigned)((rows + 3) / 4)), block(256);
  const T *gg = (const T*)g, *bb = (const T*)b, *cc = (const T*)cam, *rr = (const T*)agg_reg;
  switch (C / 64) {
#define VGGTX_FIN_CASE(n)                                                                                    \
  case n:                                                                                                    \
    hipLaunchKernelGGL((embed_finish_kernel<n, T>), grid, block, 0, s, x, Pd, gg, bb, eps, cc, rr, out, f0, \
                       n_frames, first);                                                                     \
    break;
    VGGTX_FIN_CASE(2) VGGTX_FIN_CASE(4) VGGTX_FIN_CASE(6) VGGTX_FIN_CASE(8) VGGTX_FIN_CASE(10) VGGTX_FIN_CASE(12)
    VGGTX_FIN_CASE(14) VGGTX_FIN_CASE(16) VGGTX_FIN_CASE(18) VGGTX_FIN_CASE(20) VGGTX_FIN_CASE(22)
    VGGTX_FIN_CASE(24) VGGTX_FIN_CASE(26) VGGTX_FIN_CASE(28) VGGTX_FIN_CASE(30) VGGTX_FIN_CASE(32)
#undef VGGTX_FIN_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_embed_finish(const float* x, int Pd, const void* g, const void* b, float eps, const void* cam,
                               const void* agg_reg, float* out, int64_t f0, int n_frames, const FirstMask& first,
                               int C, bool bf16_io, hipStream_t s) {
  if (n_frames <= 0) return hipSuccess;
  return bf16_io ? finish_dispatch<bf16>(x, Pd, g, b, eps, cam, agg_reg, out, f0, n_frames, first, C, s)
                 : finish_dispatch<float>(x, Pd, g, b, eps, cam, agg_reg, out, f0, n_frames, first, C, s);
}

}  // namespace vggtx
