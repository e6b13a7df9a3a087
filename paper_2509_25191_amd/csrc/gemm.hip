// Projection GEMMs of the transformer blocks with fused epilogues:
//   EPI_QKV   [q | k | v] = h W_qkv^T + b, written head-major [H, tokens, D]
//   EPI_RESID x += y W^T + b in place (attention out-projection and second MLP
//             Linear), optionally copying the new residual into an output slot
//   EPI_GELU  hidden = GELU(h W_1^T + b_1) with the erf GELU (library erff in
//             float32; Abramowitz & Stegun 7.1.26 where hidden is bfloat16)
//   EPI_EMBED patch tokens = patches W_patch^T + b + position embedding,
//             scattered into the token rows behind each frame's special tokens
// C[M, N] = A[M, K] W[N, K]^T: both operands are K-contiguous ("NT"), which is
// the natural operand order of the MFMA (8 consecutive k per lane).
#include "common.h"
#include "kernels.h"

#include <type_traits>

namespace vggtx {

__device__ __forceinline__ float gelu_erf(float u) { return 0.5f * u * (1.f + erff(u * 0.70710678118654752f)); }

// GELU with erf from Abramowitz & Stegun 7.1.26 (Hastings): for x >= 0,
// erf(x) = 1 - t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) e^(-x^2),
// t = 1 / (1 + p x), |error| <= 1.5e-7; odd extension for x < 0.  Branch free
// (the library erff takes two code paths per element); used where the result
// is stored in bfloat16, whose rounding (2^-9 relative) dwarfs that error.
__device__ __forceinline__ float gelu_erf_as(float u) {
  const float x = u * 0.70710678118654752f;
  const float ax = __builtin_fabsf(x);
  const float t = __builtin_amdgcn_rcpf(__builtin_fmaf(0.3275911f, ax, 1.f));
  float poly = __builtin_fmaf(1.061405429f, t, -1.453152027f);
  poly = __builtin_fmaf(poly, t, 1.421413741f);
  poly = __builtin_fmaf(poly, t, -0.284496736f);
  poly = __builtin_fmaf(poly, t, 0.254829592f);
  poly *= t;
  const float e = __builtin_amdgcn_exp2f(-ax * ax * 1.4426950408889634f);
  const float erf_ax = __builtin_fmaf(-poly, e, 1.f);
  const float erf_x = __builtin_copysignf(erf_ax, x);
  return 0.5f * u * (1.f + erf_x);
}

template <typename T> __device__ __forceinline__ void st4(T* p, const float v[4]);
template <> __device__ __forceinline__ void st4<float>(float* p, const float v[4]) {
  const f32x4 x = {v[0], v[1], v[2], v[3]};
  *(f32x4*)p = x;
}
template <> __device__ __forceinline__ void st4<bf16>(bf16* p, const float v[4]) {
  const bf16x4 x = {f2bf(v[0]), f2bf(v[1]), f2bf(v[2]), f2bf(v[3])};
  *(bf16x4*)p = x;
}

// Epilogue of 4 consecutive output columns of local row r (A's row r).
// T: element type of the bias and of the q/k/v or hidden outputs.
template <int EPI, typename T>
__device__ __forceinline__ void epi4(const GemmParams& p, int r, int col, float v[4]) {
  const T* bias = (const T*)p.bias;
#pragma unroll
  for (int j = 0; j < 4; ++j) v[j] += ldf(bias + col + j);
  const int64_t grow = (int64_t)p.row0 + r;
  if (EPI == EPI_QKV) {
    const int part = col / p.C, cc = col - part * p.C;
    const int hh = cc / kHeadDim, d = cc - hh * kHeadDim;
    if (part == 0) {
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] *= p.q_scale;
    }
    st4<T>((T*)p.qkv[part] + hh * p.qkv_hs[part] + (int64_t)r * kHeadDim + d, v);
  } else if (EPI == EPI_RESID) {
    float* x = p.x + grow * p.ldx + col;
    const f32x4 old = *(const f32x4*)x;
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] += old[j];  // the new residual, also returned to the caller
    st4<float>(x, v);
    if (p.out) {
      if (p.out_f32) st4<float>((float*)p.out + grow * p.ldo + col, v);
      else st4<bf16>((bf16*)p.out + grow * p.ldo + col, v);
    }
  } else if (EPI == EPI_EMBED) {
    const int64_t f = grow / p.emb_np;
    const int i = (int)(grow - f * p.emb_np);
    const T* pos = (const T*)p.pos + (int64_t)(1 + i) * p.N + col;
    float nv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) nv[j] = v[j] + ldf(pos + j);
    st4<float>(p.x + (f * p.emb_pd + kEmbedSpecial + i) * p.ldx + col, nv);
  } else if (sizeof(T) == 2) {
    float gv[4] = {gelu_erf_as(v[0]), gelu_erf_as(v[1]), gelu_erf_as(v[2]), gelu_erf_as(v[3])};
    st4<T>((T*)p.hid + (int64_t)r * p.ldh + col, gv);
  } else {
    float gv[4] = {gelu_erf(v[0]), gelu_erf(v[1]), gelu_erf(v[2]), gelu_erf(v[3])};
    st4<T>((T*)p.hid + (int64_t)r * p.ldh + col, gv);
  }
}

// Sum over the 32 lanes of a half wave (lanes l and l ^ o for o < 32).
__device__ __forceinline__ float half_wave_sum(float v) {
#pragma unroll
  for (int o = 16; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// ------------------------------------------------------------------ BF16 MFMA
// 128 x 128 output tile, BK = 64, 4 waves in a 2 x 2 grid of 64 x 64 wave
// tiles (2 x 2 MFMA 32x32x16 blocks each).  A and W tiles are staged in LDS
// with 16-byte granules XOR-swizzled by row; the accumulators go through LDS
// once more so that the epilogue reads and writes whole rows.
//
// Pipeline: the global loads run two K tiles ahead through two register
// sets (tile j in set j % 2), the stores of tile kt + 1 into the other LDS
// buffer follow the MFMAs of tile kt, and within a tile the LDS reads of
// k-step kk + 1 are issued before the MFMAs of k-step kk (scheduling
// barriers keep that order).  Control flow is uniform, so the compiler's
// load counters never have to assume a path without loads: rows past M read
// row M - 1 (their results are never stored), the loads past the last tile
// repeat it, and the final store goes to the buffer nobody reads any more.
// The barrier between tiles is a plain s_barrier after the LDS stores:
// __syncthreads() would also wait for the loads still in flight.
template <int EPI>
__global__ __launch_bounds__(256, 2) void gemm_bf16_kernel(GemmParams p) {
  constexpr int BM = 128, BN = 128, BK = 64, CLD = BN + 4;
  __shared__ __attribute__((aligned(16))) char smem[BM * CLD * 4];
  bf16* As = (bf16*)smem;
  bf16* Ws = As + 2 * BM * BK;
  float* Cs = (float*)smem;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 5, r32 = lane & 31;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int ch = tid & 7;
  const int64_t a_rs = p.a_hs ? kHeadDim : p.lda;  // A row stride
  const int64_t a_ts = p.a_hs ? p.a_hs : BK;       // A step per K tile
  const bf16* asrc[4];
  const bf16* wsrc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = (tid >> 3) + 32 * i;
    asrc[i] = (const bf16*)p.a + min(m0 + r, p.M - 1) * a_rs + ch * 8;
    wsrc[i] = (const bf16*)p.w + (int64_t)(n0 + r) * p.K + ch * 8;
  }
  bf16x8 areg[2][4], wreg[2][4];
  auto gload = [&](auto set_c, int kt) {
    constexpr int SET = decltype(set_c)::value;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      areg[SET][i] = *(const bf16x8*)(asrc[i] + kt * a_ts);
      wreg[SET][i] = *(const bf16x8*)(wsrc[i] + kt * BK);
    }
  };
  auto lstore = [&](auto set_c, int buf) {
    constexpr int SET = decltype(set_c)::value;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = (tid >> 3) + 32 * i;
      *(bf16x8*)&As[buf * BM * BK + r * BK + ((ch ^ lds_swz8(r)) * 8)] = areg[SET][i];
      *(bf16x8*)&Ws[buf * BN * BK + r * BK + ((ch ^ lds_swz8(r)) * 8)] = wreg[SET][i];
    }
  };
  auto barrier = [&]() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  };

  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x16{};

  using S0 = std::integral_constant<int, 0>;
  using S1 = std::integral_constant<int, 1>;
  const int nk = p.K / BK;
  gload(S0{}, 0);
  gload(S1{}, min(1, nk - 1));
  lstore(S0{}, 0);
  barrier();
  // step kt: tile kt + 2 -> register set SET (= kt % 2), MFMAs on LDS buffer
  // kt & 1, tile kt + 1 (set 1 - SET) -> the other buffer
  auto step = [&](int kt, auto set_c) {
    constexpr int SET = decltype(set_c)::value;
    const int buf = kt & 1;
    gload(set_c, min(kt + 2, nk - 1));
    __builtin_amdgcn_sched_barrier(0);
    bf16x8 a[2][2], b[2][2];  // operands of k-step kk in set kk & 1
    auto rd = [&](int kk, auto s_c) {
      constexpr int S = decltype(s_c)::value;
#pragma unroll
      for (int mi = 0; mi < 2; ++mi) {
        const int r = wm * 64 + mi * 32 + r32;
        a[S][mi] = *(const bf16x8*)&As[buf * BM * BK + r * BK + (((2 * kk + g) ^ lds_swz8(r)) * 8)];
      }
#pragma unroll
      for (int nj = 0; nj < 2; ++nj) {
        const int r = wn * 64 + nj * 32 + r32;
        b[S][nj] = *(const bf16x8*)&Ws[buf * BN * BK + r * BK + (((2 * kk + g) ^ lds_swz8(r)) * 8)];
      }
    };
    auto mm = [&](auto s_c) {
      constexpr int S = decltype(s_c)::value;
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int nj = 0; nj < 2; ++nj) acc[mi][nj] = mfma_bf16(a[S][mi], b[S][nj], acc[mi][nj]);
    };
    rd(0, S0{});
    rd(1, S1{});
    __builtin_amdgcn_sched_barrier(0);
    mm(S0{});
    __builtin_amdgcn_sched_barrier(0);
    rd(2, S0{});
    __builtin_amdgcn_sched_barrier(0);
    mm(S1{});
    __builtin_amdgcn_sched_barrier(0);
    rd(3, S1{});
    __builtin_amdgcn_sched_barrier(0);
    mm(S0{});
    __builtin_amdgcn_sched_barrier(0);
    mm(S1{});
    lstore(std::integral_constant<int, 1 - SET>{}, buf ^ 1);
    barrier();
  };
  int kt = 0;
  for (; kt + 2 <= nk; kt += 2) {
    step(kt, S0{});
    step(kt + 1, S1{});
  }
  if (kt < nk) step(kt, S0{});
  __syncthreads();

#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int nj = 0; nj < 2; ++nj)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int row = wm * 64 + mi * 32 + 8 * (i >> 2) + 4 * g + (i & 3);
        const int col = wn * 64 + nj * 32 + r32;
        Cs[row * CLD + col] = acc[mi][nj][i];
      }
  __syncthreads();
  // the 32 lanes of a half wave share one row (idx / 32)
  for (int idx = tid; idx < BM * (BN / 4); idx += 256) {
    const int row = idx / (BN / 4), c4 = (idx % (BN / 4)) * 4;
    const bool valid = m0 + row < p.M;
    const f32x4 cv = *(const f32x4*)&Cs[row * CLD + c4];
    float v[4] = {cv[0], cv[1], cv[2], cv[3]};
    if (valid) epi4<EPI, bf16>(p, m0 + row, n0 + c4, v);
    if (EPI == EPI_RESID && p.stats) {
      // (mean, M2) of the new residual over this tile's 128 columns, two passes
      const float mean = half_wave_sum(v[0] + v[1] + v[2] + v[3]) * (1.f / BN);
      float q = 0.f;
#pragma unroll
      for (int j = 0; j < 4; ++j) q += (v[j] - mean) * (v[j] - mean);
      q = half_wave_sum(q);
      if (valid && (tid & 31) == 0) {
        const int nt = p.N / BN;
        float* st = p.stats + (((int64_t)p.row0 + m0 + row) * nt + n0 / BN) * 2;
        st[0] = mean;
        st[1] = q;
      }
    }
  }
}

// ------------------------------------------------------------------ FP32
// Plain VALU tiled GEMM (64 x 64 tile, BK = 16, 4 x 4 outputs per thread); it
// serves the float32 reference-precision path.
template <int EPI>
__global__ __launch_bounds__(256) void gemm_f32_kernel(GemmParams p) {
  constexpr int BM = 64, BN = 64, BK = 16;
  __shared__ float As[BK][BM + 4];
  __shared__ float Ws[BK][BN + 4];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const float* A = (const float*)p.a;
  const float* W = (const float*)p.w;
  float acc[4][4] = {};
  const int lr = tid >> 2, lk = (tid & 3) * 4;
  for (int k0 = 0; k0 < p.K; k0 += BK) {
    f32x4 av = {}, wv;
    if (m0 + lr < p.M)
      av = *(const f32x4*)(p.a_hs ? A + (k0 >> 6) * p.a_hs + (int64_t)(m0 + lr) * kHeadDim + (k0 & 63) + lk
                                  : A + (int64_t)(m0 + lr) * p.lda + k0 + lk);
    wv = *(const f32x4*)(W + (int64_t)(n0 + lr) * p.K + k0 + lk);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      As[lk + j][lr] = av[j];
      Ws[lk + j][lr] = wv[j];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < BK; ++k) {
      const f32x4 a = *(const f32x4*)&As[k][ty * 4];
      const f32x4 b = *(const f32x4*)&Ws[k][tx * 4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = m0 + ty * 4 + i;
    if (row < p.M) epi4<EPI, float>(p, row, n0 + tx * 4, acc[i]);
  }
}

hipError_t launch_gemm_bf16(const GemmParams& p, Epi epi, hipStream_t s) {
  if (p.M <= 0) return hipSuccess;  // nothing to compute (the kernel reads row M - 1)
  dim3 grid(p.N / 128, (p.M + 127) / 128), block(256);
  switch (epi) {
    case EPI_QKV: return launch(gemm_bf16_kernel<EPI_QKV>, grid, block, 0, s, p);
    case EPI_RESID: return launch(gemm_bf16_kernel<EPI_RESID>, grid, block, 0, s, p);
    case EPI_GELU: return launch(gemm_bf16_kernel<EPI_GELU>, grid, block, 0, s, p);
    case EPI_EMBED: return launch(gemm_bf16_kernel<EPI_EMBED>, grid, block, 0, s, p);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gemm_f32(const GemmParams& p, Epi epi, hipStream_t s) {
  if (p.stats) return hipErrorInvalidValue;  // the float32 path computes its LayerNorm statistics itself
  dim3 grid(p.N / 64, (p.M + 63) / 64), block(256);
  switch (epi) {
    case EPI_QKV: return launch(gemm_f32_kernel<EPI_QKV>, grid, block, 0, s, p);
    case EPI_RESID: return launch(gemm_f32_kernel<EPI_RESID>, grid, block, 0, s, p);
    case EPI_GELU: return launch(gemm_f32_kernel<EPI_GELU>, grid, block, 0, s, p);
    case EPI_EMBED: return launch(gemm_f32_kernel<EPI_EMBED>, grid, block, 0, s, p);
  }
  return hipErrorInvalidValue;
}

}  // namespace vggtx
