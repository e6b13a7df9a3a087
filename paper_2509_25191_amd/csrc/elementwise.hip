// LayerNorm of the float32 residual stream (the pre-LN of both sub-blocks).
// One wave per row; mean and biased variance in float32 (two passes over the
// row held in registers), output in the GEMM operand type.
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
    hipLaunchKernelGGL((layernorm_kernel<n, T>), grid, block, 0, s, x, ldx, gg, bb, eps, hh, ldh, rows); \
    break;
    VGGTX_LN_CASE(2) VGGTX_LN_CASE(4) VGGTX_LN_CASE(6) VGGTX_LN_CASE(8) VGGTX_LN_CASE(10) VGGTX_LN_CASE(12)
    VGGTX_LN_CASE(14) VGGTX_LN_CASE(16) VGGTX_LN_CASE(18) VGGTX_LN_CASE(20) VGGTX_LN_CASE(22) VGGTX_LN_CASE(24)
    VGGTX_LN_CASE(26) VGGTX_LN_CASE(28) VGGTX_LN_CASE(30) VGGTX_LN_CASE(32)
#undef VGGTX_LN_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_layernorm(const float* x, int64_t ldx, const void* g, const void* b, float eps, void* h, int64_t ldh,
                            int rows, int C, bool bf16_io, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  return bf16_io ? ln_dispatch<bf16>(x, ldx, g, b, eps, h, ldh, rows, C, s)
                 : ln_dispatch<float>(x, ldx, g, b, eps, h, ldh, rows, C, s);
}

hipError_t launch_copy_f32(const float* src, float* dst, int64_t n, hipStream_t s) {
  if (src == dst || n == 0) return hipSuccess;
  return hipMemcpyAsync(dst, src, n * sizeof(float), hipMemcpyDeviceToDevice, s);
}

}  // namespace vggtx
