// Device-side vocabulary shared by the vggtx HIP kernels (gfx950 / CDNA4).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vggtx {

typedef __bf16 bf16;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(8 * sizeof(int)))) int i32x8;
typedef __attribute__((__vector_size__(4 * sizeof(int)))) int i32x4;
typedef __attribute__((__vector_size__(2 * sizeof(int)))) int i32x2;

constexpr int kHeadDim = 64;       // D: the only head size the kernels are built for
constexpr int kKeyPad = 64;        // transposed V: every sequence padded to a multiple of this
constexpr int kQuantRows = 128;    // FP8 scale block: rows per block, per sequence
constexpr int kMaxSeqInline = 64;  // sequences a single attention launch can carry in its arguments
constexpr float kLog2e = 1.4426950408889634f;

// ---------------------------------------------------------------- MFMA
// Register layouts (verified on gfx950 with one-hot probes):
//   32x32xK: A lane l holds row l%32, k-slot group l/32; B lane l holds column
//   l%32, the same k-slot group; D lane l register i holds row
//   8*(i/4) + 4*(l/32) + i%4, column l%32.
//   16x16xK: A row l%16, group l/16; D register i holds row 4*(l/16) + i, column l%16.
__device__ __forceinline__ f32x16 mfma_bf16(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 mfma_f32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
// Same with E8M0 block scales: D = C + (2^(ea-127) A)(2^(eb-127) B).  Each lane's
// code scales the row (A) or column (B) and the 32-wide k-group it supplies;
// here every lane passes the same code.
__device__ __forceinline__ f32x16 mfma_fp8_scaled(i32x8 a, i32x8 b, f32x16 c, int ea, int eb) {
  return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, ea, 0, eb);
}

// FP8 E4M3 x E4M3, 16x16x128, unit block scales.
__device__ __forceinline__ f32x4 mfma_fp8_16(i32x8 a, i32x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
}

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }

// LDS swizzles (XOR on the 16-byte granule index of a tile row).  A
// ds_read_b128 is served 16 consecutive lanes at a time from 64 four-byte
// banks; with these swizzles 16 consecutive rows read at one logical granule
// hit 16 distinct 16-byte bank groups, and so do the tile stores (ds_write_b64
// of the FP8 V tile included, 32 lanes per pass).  Both depend on r mod 32
// only, so the 32-row blocks of a tile share one lane address plus an
// immediate offset.
__device__ __forceinline__ int lds_swz8(int r) { return (r ^ ((r >> 3) & 3)) & 7; }  // 128-byte rows (8 granules)
__device__ __forceinline__ int lds_swz4(int r) { return ((r >> 1) ^ (r >> 2)) & 3; }  // 64-byte rows (4 granules)

// Two float32 -> two E4M3 codes (round to nearest even) in the low 16 bits.
// The hardware conversion turns magnitudes above 464 into NaN, so inputs are
// clamped to +-448 first (saturating encode).
__device__ __forceinline__ uint32_t cvt_e4m3x2(float a, float b) {
  a = __builtin_fminf(__builtin_fmaxf(a, -448.f), 448.f);
  b = __builtin_fminf(__builtin_fmaxf(b, -448.f), 448.f);
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, 0, false) & 0xffffu;
}

__device__ __forceinline__ float bf2f(bf16 x) { return (float)x; }
__device__ __forceinline__ bf16 f2bf(float x) { return (bf16)x; }  // round to nearest even

template <typename T> __device__ __forceinline__ float ldf(const T* p) { return (float)*p; }

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = __builtin_fmaxf(v, __shfl_xor(v, o));
  return v;
}

}  // namespace vggtx
