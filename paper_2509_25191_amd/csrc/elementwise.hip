// LayerNorm of the float32 residual stream (the pre-LN of both sub-blocks).
// One wave per row; mean and biased variance in float32 (two passes over the
// row held in registers), output in the GEMM operand type.
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace vggtx {

template <int NPL, typename T>
__global__ __launch_bounds__(256) void layernorm_kernel(const float* x, int64_t ldx, const T* g, const T* b, float eps,
                                                        T* h, int64_t ldh, int rows) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  constexpr int C = NPL * 64;
  const float* xr = x + (int64_t)row * ldx;
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
  const float var = wave_sum(q) * (1.f / C);
  const float rstd = 1.f / __builtin_sqrtf(var + eps);
  T* hr = h + (int64_t)row * ldh;
#pragma unroll
  for (int j = 0; j < NPL; ++j) {
    const int c = lane + 64 * j;
    hr[c] = (T)((v[j] - mean) * rstd * ldf(g + c) + ldf(b + c));
  }
}

template <typename T>
static hipError_t ln_dispatch(const float* x, int64_t ldx, const void* g, const void* b, float eps, void* h,
                              int64_t ldh, int rows, int C, hipStream_t s) {
  dim3 grid((rows + 3) / 4), block(256);
  const T* gg = (const T*)g;
  const T* bb = (const T*)b;
  T* hh = (T*)h;
  switch (C / 64) {
#define VGGTX_LN_CASE(n)                                                                         \
  case n:                                                                                        \
    return launch(layernorm_kernel<n, T>, grid, block, 0, s, x, ldx, gg, bb, eps, hh, ldh, rows);
    VGGTX_LN_CASE(2) VGGTX_LN_CASE(4) VGGTX_LN_CASE(6) VGGTX_LN_CASE(8) VGGTX_LN_CASE(10) VGGTX_LN_CASE(12)
    VGGTX_LN_CASE(14) VGGTX_LN_CASE(16) VGGTX_LN_CASE(18) VGGTX_LN_CASE(20) VGGTX_LN_CASE(22) VGGTX_LN_CASE(24)
    VGGTX_LN_CASE(26) VGGTX_LN_CASE(28) VGGTX_LN_CASE(30) VGGTX_LN_CASE(32)
#undef VGGTX_LN_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_layernorm(const float* x, int64_t ldx, const void* g, const void* b, float eps, void* h, int64_t ldh,
                            int rows, int C, bool bf16_io, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  return bf16_io ? ln_dispatch<bf16>(x, ldx, g, b, eps, h, ldh, rows, C, s)
                 : ln_dispatch<float>(x, ldx, g, b, eps, h, ldh, rows, C, s);
}

// Row statistics in the layout ln_apply_kernel consumes: for every row
// and every 128-column slice t, (mean_t, M2_t) = (mean of the slice, sum of
// squared deviations from it), two passes over the slice in float32.  One
// wave per row, two values per lane per slice.  The RESID epilogue of the
// projection GEMMs produces the same statistics for the rows it updates; this
// kernel covers residual streams that no epilogue wrote (the aggregator's
// input tokens, the front end's embedded tokens).
__global__ __launch_bounds__(256) void row_stats_kernel(const float* x, int64_t ldx, int rows, int C, float* stats) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const float* xr = x + (int64_t)row * ldx;
  const int nt = C / 128;
  for (int t = 0; t < nt; ++t) {
    const float a = xr[128 * t + 2 * lane], b = xr[128 * t + 2 * lane + 1];
    const float mean = wave_sum(a + b) * (1.f / 128.f);
    const float m2 = wave_sum((a - mean) * (a - mean) + (b - mean) * (b - mean));
    if (lane == 0) {
      stats[((int64_t)row * nt + t) * 2] = mean;
      stats[((int64_t)row * nt + t) * 2 + 1] = m2;
    }
  }
}

hipError_t launch_row_stats(const float* x, int64_t ldx, int rows, int C, float* stats, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  if (C % 128) return hipErrorInvalidValue;
  return launch(row_stats_kernel, dim3((rows + 3) / 4), dim3(256), 0, s, x, ldx, rows, C, stats);
}

// LayerNorm from precomputed row statistics: h[r] = bf16((x[r] - mean) /
// sqrt(var + eps) * g + b), with mean and the biased variance combined from
// the (mean, M2) pairs of the row's 128-column slices (Chan et al.'s pairwise
// update: every slice holds 128 values) at stats[(srow0 + r) * C/128 * 2].
// The projection GEMMs' residual epilogues write those pairs for the rows
// they update, so the statistics cost no pass of their own.  One wave per
// row, four consecutive columns per lane and step.
__global__ __launch_bounds__(256) void ln_apply_kernel(const float* x, int64_t ldx, const float* stats, int64_t srow0,
                                                       const bf16* g, const bf16* b, float eps, bf16* h, int64_t ldh,
                                                       int rows, int C) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const int nt = C / 128;
  const float* st = stats + (srow0 + row) * nt * 2;
  float mu = 0.f;
  for (int t = 0; t < nt; ++t) mu += st[2 * t];
  mu /= (float)nt;
  float m2 = 0.f;
  for (int t = 0; t < nt; ++t) {
    const float d = st[2 * t] - mu;
    m2 += st[2 * t + 1] + 128.f * d * d;
  }
  const float rs = 1.f / __builtin_sqrtf(m2 / (float)C + eps), nm = -mu * rs;
  const float* xr = x + (int64_t)row * ldx;
  bf16* hr = h + (int64_t)row * ldh;
  for (int c = 4 * lane; c < C; c += 256) {
    const f32x4 v = *(const f32x4*)(xr + c);
    const bf16x4 gg = *(const bf16x4*)(g + c), bb = *(const bf16x4*)(b + c);
    bf16x4 o;
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = f2bf(__builtin_fmaf(__builtin_fmaf(v[j], rs, nm), bf2f(gg[j]), bf2f(bb[j])));
    *(bf16x4*)(hr + c) = o;
  }
}

hipError_t launch_ln_apply(const float* x, int64_t ldx, const float* stats, int64_t srow0, const void* g, const void* b,
                           float eps, void* h, int64_t ldh, int rows, int C, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  if (C % 128) return hipErrorInvalidValue;
  return launch(ln_apply_kernel, dim3((rows + 3) / 4), dim3(256), 0, s, x, ldx, stats, srow0, (const bf16*)g,
                (const bf16*)b, eps, (bf16*)h, ldh, rows, C);
}

// Seeded synthetic bfloat16 values for the autotuner: a counter-based hash
// (SplitMix64 finaliser) of (seed, index) mapped to a uniform value in
// [-scale, scale).
__global__ void fill_hash_bf16_kernel(bf16* x, int64_t n, uint64_t seed, float scale) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    const float u = (float)(z >> 40) * (1.f / 16777216.f);  // [0, 1)
    x[i] = f2bf((2.f * u - 1.f) * scale);
  }
}

hipError_t launch_fill_hash_bf16(bf16* x, int64_t n, uint64_t seed, float scale, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  return launch(fill_hash_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, n, seed, scale);
}

// Plain copy (a kernel rather than a runtime copy so that it can be recorded
// into a graph like every other step of the forward).
__global__ __launch_bounds__(256) void copy_f32_kernel(const float* src, float* dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t n4 = ((uintptr_t)src % 16 == 0 && (uintptr_t)dst % 16 == 0) ? n / 4 : 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n4; i += stride)
    ((f32x4*)dst)[i] = ((const f32x4*)src)[i];
  for (int64_t i = 4 * n4 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

hipError_t launch_copy_f32(const float* src, float* dst, int64_t n, hipStream_t s) {
  if (src == dst || n == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n / 4 + 255) / 256 + 1, 8192);
  return launch(copy_f32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src, dst, n);
}

}  // namespace vggtx
