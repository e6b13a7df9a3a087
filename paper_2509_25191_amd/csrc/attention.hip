// Streamed ("flash") attention for the frame and global blocks of the
// aggregator (arXiv 2509.25191, Sec. 3.2), plus the V transposition and the
// FP8 E4M3 quantiser that feed it.
//
// Every kernel computes, per sequence and head, O = softmax(Q K^T / sqrt(D)) V
// without storing the score matrix: keys are visited in tiles of 64, a
// running row maximum m and row sum l are kept in float32 and the partial
// output is rescaled by 2^(m_old - m_new) (logits in base 2) whenever m
// grows.
//
// Work decomposition: one workgroup (4 or 8 waves, per kernel variant) per
// (query tile, head); a wave owns 32*QB query rows.  Scores are computed
// transposed, S^T = K Q^T, so that every lane owns one query column of the
// MFMA accumulator.  That makes the softmax statistics lane-local (plus one
// exchange with lane l^32) and lets the probabilities feed the P V product
// (O^T = V^T P^T) straight from registers.
#include <stdint.h>

#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace vggtx {

struct Item {
  int q0, s0, s1, vb, bb;
};

// Map a work-item index to its query tile and sequence.
__device__ __forceinline__ Item resolve_item(const SeqTable& t, int item, int rows_per_item) {
  Item it;
  if (t.uniform) {
    const int seq = item / t.tiles_per_seq;
    const int tt = item - seq * t.tiles_per_seq;
    it.s0 = t.start[0] + seq * t.len;
    it.s1 = it.s0 + t.len;
    it.vb = t.vt_base[0] + seq * ((t.len + kKeyPad - 1) / kKeyPad * kKeyPad);
    it.bb = t.blk_base[0] + seq * ((t.len + kQuantRows - 1) / kQuantRows);
    it.q0 = it.s0 + tt * rows_per_item;
  } else {
    int seq = 0;
    while (seq < t.n_seq - 1 && item >= t.tile_end[seq]) ++seq;
    const int prev = seq ? t.tile_end[seq - 1] : 0;
    it.s0 = t.start[seq];
    it.s1 = t.end[seq];
    it.vb = t.vt_base[seq];
    it.bb = t.blk_base[seq];
    it.q0 = it.s0 + (item - prev) * rows_per_item;
  }
  return it;
}

// Work distribution.  Grid mode (p.queue null): workgroup (x, y) runs work
// item x of head y.  Queue mode: the grid has one workgroup per (item, head)
// in x, and each workgroup, when it starts, takes the next work index w from
// the counter *p.queue (zero at launch), so items start in index order
// whatever order the hardware dispatches workgroups in.  Indices run
// sequence by sequence in the table's order (longest first for list tables),
// head by head within a sequence: the longest items start first, the
// shortest ones fill the tail, and the workgroups running together share the
// K and V of one (sequence, head).
__device__ __forceinline__ void take_work(const AttnParams& p, int* slot, int& head, int& item) {
  if (!p.queue) {
    head = blockIdx.y;
    item = blockIdx.x;
    return;
  }
  if (threadIdx.x == 0) *slot = atomicAdd(p.queue, 1);
  __syncthreads();
  const int w = __builtin_amdgcn_readfirstlane(*slot);  // uniform: keeps the item arithmetic scalar
  const SeqTable& t = p.seqs;
  if (t.uniform) {
    head = w / p.n_items;
    item = w - head * p.n_items;
    return;
  }
  const int H = p.n_heads;
  int seq = 0;
  while (seq < t.n_seq - 1 && w >= H * t.tile_end[seq]) ++seq;
  const int prev = seq ? t.tile_end[seq - 1] : 0;
  const int n = t.tile_end[seq] - prev;
  const int j = w - H * prev;
  head = j / n;
  item = prev + (j - head * n);
}

// max of 2 x 16 values as four chains of three-input maxima (v_max3_f32)
__device__ __forceinline__ float max32(const f32x16& a, const f32x16& b) {
  float m[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const f32x16& x = c < 2 ? a : b;
    const int o = (c & 1) * 8;
    float r = __builtin_fmaxf(__builtin_fmaxf(x[o], x[o + 1]), x[o + 2]);
    r = __builtin_fmaxf(__builtin_fmaxf(r, x[o + 3]), x[o + 4]);
    r = __builtin_fmaxf(__builtin_fmaxf(r, x[o + 5]), x[o + 6]);
    m[c] = __builtin_fmaxf(r, x[o + 7]);
  }
  return __builtin_fmaxf(__builtin_fmaxf(__builtin_fmaxf(m[0], m[1]), m[2]), m[3]);
}

__device__ __forceinline__ float lane_swap_max(float v) {
  // v_permlane32_swap exchanges the two 32-lane halves of the wave
  auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __builtin_fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
}

// |x| >= the float whose bits are `bound`, NaN included, decided on the bits.
// This file is built without NaN semantics, under which the compiler may turn
// an integer test on a float's bits back into a float compare that a NaN
// fails (it did: a test for "inf or NaN" became |x| == inf); the empty asm
// makes the bits opaque to it.
__device__ __forceinline__ bool abs_bits_at_least(float x, uint32_t bound) {
  uint32_t u = __float_as_uint(x);
  asm("" : "+v"(u));
  return (u & 0x7fffffffu) >= bound;
}

// E4M3 conversion without a clamp: the hardware rounds to nearest even, so
// values up to 464 give 448 and larger ones give the NaN code, which the
// kernel below uses as its overflow signal.  Four floats -> four E4M3 codes
// in one dword (bytes in argument order).  The first conversion fills the
// low half (its high half is scratch), the second writes the high half in
// place.
__device__ __forceinline__ int pack_e4m3x4(float e0, float e1, float e2, float e3) {
  const int lo = __builtin_amdgcn_cvt_pk_fp8_f32(e0, e1, __float_as_int(e0), false);
  return __builtin_amdgcn_cvt_pk_fp8_f32(e2, e3, lo, true);
}

// ============================================================== BF16 kernel
//
// LDS tiles (BN = 64 keys, D = 64, 128-byte rows), double-buffered.  Tiles
// move from global memory straight into LDS (global_load_lds_dwordx4: lane l
// of one instruction fills bytes 16l..16l+15 of a 1 KB LDS block, i.e. 8 tile
// rows), so no registers stage them; the next tile's loads are issued once
// every LDS read of the current tile's fragments is, and waited for at the
// end of the tile, before the barrier.  The 16-byte granules of a row are
// XOR-swizzled with the row index (lds_swz8), which keeps the ds_read_b128 of
// the MFMA fragments conflict free.
//   Ks[r][.]  K tile, row r holding key pi(r): rows 4..7 and 8..11 of every
//             16 are swapped, so that the score MFMA leaves 8 consecutive keys
//             in accumulator registers 0..7 (and 8..15) of each lane group
//             (key of register i in lane group g: 16 (i / 8) + 8 g + i % 8);
//             the probabilities then pack into the B operand of the P V
//             product in key order.
//   Vs[d][.]  V^T tile in key order.
//
// Softmax with a lazy shift, applied inside the score MFMA.  Q is taken
// times c2 = log2(e)/sqrt(D) (rounded to bfloat16 once, when its fragments
// are loaded), so the MFMA gives logits in base 2, and each query's shift m
// enters the product as a fifth k-step: A = 1 in k-slot 0 of every key row,
// B = -m (bfloat16) in k-slot 0 of the query's column, so the accumulator
// starts at -m and the probabilities are p = 2^s with no per-score
// arithmetic before the exponential.  Full key tiles after the first take
// p against the current m (the row maximum, rounded to bfloat16, when m last
// moved) with no maximum search: softmax is shift-invariant, so m only has
// to keep p finite.  While the tile's row sum stays below 2^32 every p of the
// row is below it, and O and l (float32) stay far from overflow.  A row sum
// at or above 2^32 (an infinity or a NaN included; tested on the bits) sends
// the query block to the exact step: its scores are recomputed from the K
// tile still in LDS, m moves up to the row maximum (rounded), O and l are
// rescaled by 2^(m_old - m_new), and the probabilities are taken again.  The
// first and the partial last tile always take the exact step.  The row sum
// runs on the matrix core: a 16x16x32 MFMA with a lane-selector A operand
// over the bfloat16 probability registers of the P V product (read as its B
// operand, they are 16 columns whose four k-groups hold queries n, n+16, n,
// n+16; selector rows 4j..4j+3 take the k-groups of parity j&1, so output
// lane l receives the sum for its own query l%32), so l is summed from the
// same rounded probabilities as O.
//
// Issue order: the score MFMAs of query block qb+1 and the P V MFMAs of block
// qb-1 are issued between the exponentials of block qb.
template <int QB, int NW, int OCC>
__global__ __launch_bounds__(64 * NW, OCC) void attn_bf16_kernel(AttnParams p) {
  constexpr int BN = 64, D = kHeadDim, BM = 32 * QB * NW;
  constexpr float kLazyBound = 0x1p32f;
  __shared__ __attribute__((aligned(16))) bf16 Ks[2][BN * D];
  __shared__ __attribute__((aligned(16))) bf16 Vs[2][D * BN];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 5, r32 = lane & 31;
  __shared__ int s_work;
  int head, item;
  take_work(p, &s_work, head, item);
  const Item it = resolve_item(p.seqs, item, BM);

  const bf16* Q = (const bf16*)p.q + head * p.q_hs;
  const bf16* K = (const bf16*)p.k + head * p.k_hs;
  const bf16* Vt = (const bf16*)p.vt + head * p.vt_hs + it.vb;

  const bf16x8 zero8 = {};
  const bf16 sv = (((lane >> 2) ^ (lane >> 4)) & 1) ? (bf16)0.0f : (bf16)1.0f;  // row-sum selector
  const bf16x8 sel8 = {sv, sv, sv, sv, sv, sv, sv, sv};
  const float c2 = p.scale_log2;
  bf16x8 qf[QB][4];
  bf16x8 negm[QB];  // B operand of the shift step: -m in k-slot 0 of lane group 0
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    const int row = it.q0 + (wave * QB + qb) * 32 + r32;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      qf[qb][c] = row < it.s1 ? *(const bf16x8*)(Q + row * p.q_ts + 16 * c + 8 * g) : zero8;
#pragma unroll
      for (int j = 0; j < 8; ++j) qf[qb][c][j] = f2bf(bf2f(qf[qb][c][j]) * c2);
    }
    negm[qb] = zero8;
  }
  bf16x8 ones8 = zero8;  // A operand of the shift step: 1 in k-slot 0 of every key row
  if (g == 0) ones8[0] = (bf16)1.0f;

  // Tile t into LDS buffer buf: wave w moves the 8-row blocks w, w + NW, ...
  // of both tiles; lane l fills row 8 * block + l / 8, granule slot l % 8.
  auto dma = [&](int t, int buf) {
    const int rows_left = it.s1 - (it.s0 + t * BN);
#pragma unroll
    for (int j = 0; j < 8 / NW; ++j) {
      const int rb = 8 * (wave + NW * j);
      const int r = rb + (lane >> 3), ch = (lane & 7) ^ lds_swz8(r);
      const int q4 = (r >> 2) & 3;
      const int key = (r & ~15) | ((q4 == 1 ? 2 : (q4 == 2 ? 1 : q4)) << 2) | (r & 3);
      const int kr = key < rows_left ? key : 0;  // rows past the end: any existing key (their scores are masked)
      __builtin_amdgcn_global_load_lds((const void*)(K + (int64_t)(it.s0 + t * BN + kr) * p.k_ts + ch * 8),
                                       (__attribute__((address_space(3))) void*)&Ks[buf][rb * D], 16, 0, 0);
      __builtin_amdgcn_global_load_lds((const void*)(Vt + (int64_t)r * p.vt_ds + t * BN + ch * 8),
                                       (__attribute__((address_space(3))) void*)&Vs[buf][rb * BN], 16, 0, 0);
    }
  };

  f32x16 oacc[QB][2];
  float m_run[QB], l_run[QB];
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    oacc[qb][0] = f32x16{};
    oacc[qb][1] = f32x16{};
    m_run[qb] = 0.f;  // the shift held in negm (set by the first tile)
    l_run[qb] = 0.f;
  }
  const int ntiles = (it.s1 - it.s0 + BN - 1) / BN;

  dma(0, 0);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();

  // One key tile.  MASKED is set only for the final, partial tile of a
  // sequence, so full tiles carry no key-bound checks; FIRST only for the
  // first tile.  Both take the exact step on every query block.
  auto tile = [&](int t, auto masked, auto first) {
    constexpr bool MASKED = decltype(masked)::value, FIRST = decltype(first)::value;
    constexpr bool EXACT = MASKED || FIRST;
    const int kt = it.s0 + t * BN, buf = t & 1;

    bf16x8 kf[2][4];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int r = kb * 32 + r32;
        kf[kb][c] = *(const bf16x8*)&Ks[buf][r * D + (((2 * c + g) ^ lds_swz8(r)) * 8)];
      }
    f32x16 s[QB][2];
    bf16x8 pb[QB][2][2];
    bf16x8 vf[2][2][2];
    auto score = [&](int qb) {
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        s[qb][kb] = mfma_bf16(ones8, negm[qb], f32x16{});
#pragma unroll
        for (int c = 0; c < 4; ++c) s[qb][kb] = mfma_bf16(kf[kb][c], qf[qb][c], s[qb][kb]);
      }
    };
    auto pv = [&](int qb) {
#pragma unroll
      for (int db = 0; db < 2; ++db)
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
          for (int h = 0; h < 2; ++h) oacc[qb][db] = mfma_bf16(vf[db][kb][h], pb[qb][kb][h], oacc[qb][db]);
    };
    auto probs = [&](int qb, const f32x16& a, const f32x16& b) {
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        const f32x16& x = kb ? b : a;
#pragma unroll
        for (int i = 0; i < 16; ++i) pb[qb][kb][i >> 3][i & 7] = f2bf(fast_exp2(x[i]));
      }
    };
    auto rowsum = [&](int qb) {
      f32x4 r = {};
#pragma unroll
      for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int h = 0; h < 2; ++h) r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(sel8, pb[qb][kb][h], r, 0, 0, 0);
      return r[0];
    };
    // exact step: mask, row maximum, move m (rescaling O and l), probabilities.
    // The scores a, b are relative to the current m.
    auto exact = [&](int qb, f32x16& a, f32x16& b, auto is_first) {
      constexpr bool FIRST_ = decltype(is_first)::value;
      if (MASKED) {
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
          for (int i = 0; i < 16; ++i)
            if (kt + kb * 32 + 16 * (i >> 3) + 8 * g + (i & 7) >= it.s1) (kb ? b : a)[i] = -INFINITY;
      }
      const float mx = lane_swap_max(max32(a, b));
      // the new m, rounded to bfloat16 (the shift enters the MFMA in that type);
      // on the first tile m starts at 0 and O and l are still zero
      const float base = FIRST_ ? 0.f : m_run[qb];
      const float d = bf2f(f2bf(base + (FIRST_ ? mx : __builtin_fmaxf(mx, 0.f)))) - base;
      if (!FIRST_) {
        const float alpha = fast_exp2(-d);
        l_run[qb] *= alpha;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          oacc[qb][0][i] *= alpha;
          oacc[qb][1][i] *= alpha;
        }
      }
      m_run[qb] = base + d;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        a[i] -= d;
        b[i] -= d;
      }
      if (g == 0) negm[qb][0] = f2bf(-m_run[qb]);
      probs(qb, a, b);
    };

    score(0);
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
      __builtin_amdgcn_sched_barrier(0);
      if (qb + 1 < QB) score(qb + 1);
      if (qb >= 1) pv(qb - 1);
      if (EXACT) exact(qb, s[qb][0], s[qb][1], first);
      else probs(qb, s[qb][0], s[qb][1]);
      if (!EXACT && QB > 1) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          __builtin_amdgcn_sched_group_barrier(0x002, 10, 0);  // VALU
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
        }
      }
      if (qb == 0) {
#pragma unroll
        for (int db = 0; db < 2; ++db)
#pragma unroll
          for (int kb = 0; kb < 2; ++kb)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int d = db * 32 + r32;
              vf[db][kb][h] = *(const bf16x8*)&Vs[buf][d * BN + (((2 * (2 * kb + h) + g) ^ lds_swz8(d)) * 8)];
            }
        // every LDS read of this tile's fragments is issued: move the next tile in
        if (t + 1 < ntiles) dma(t + 1, buf ^ 1);
      }
      float ls = rowsum(qb);
      if (!EXACT && __any(abs_bits_at_least(ls, __float_as_uint(kLazyBound)))) {
        f32x16 r[2];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
          r[kb] = mfma_bf16(ones8, negm[qb], f32x16{});
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const int rr = kb * 32 + r32;
            const bf16x8 k8 = *(const volatile bf16x8*)&Ks[buf][rr * D + (((2 * c + g) ^ lds_swz8(rr)) * 8)];
            r[kb] = mfma_bf16(k8, qf[qb][c], r[kb]);
          }
        }
        exact(qb, r[0], r[1], std::false_type{});
        ls = rowsum(qb);
      }
      l_run[qb] += ls;
    }
    __builtin_amdgcn_sched_barrier(0);
    pv(QB - 1);
    __builtin_amdgcn_sched_barrier(0);
    if (t + 1 < ntiles) {
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
    }
  };
  const bool ragged = (it.s1 - it.s0) % BN != 0;
  const int nfull = ntiles - (ragged ? 1 : 0);
  if (nfull > 0) tile(0, std::false_type{}, std::true_type{});
  for (int t = 1; t < nfull; ++t) tile(t, std::false_type{}, std::false_type{});
  if (ragged) {
    if (ntiles == 1)
      tile(0, std::true_type{}, std::true_type{});
    else
      tile(ntiles - 1, std::true_type{}, std::false_type{});
  }

#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    const float inv = 1.f / l_run[qb];
    const int row = it.q0 + (wave * QB + qb) * 32 + r32;
    if (row < it.s1) {
#pragma unroll
      for (int db = 0; db < 2; ++db)
#pragma unroll
        for (int i = 0; i < 16; i += 4) {
          const int d = db * 32 + 8 * (i >> 2) + 4 * g;
          bf16* o = (bf16*)p.o + row * p.o_ts + head * p.o_hs + d;
          const bf16x4 v = {f2bf(oacc[qb][db][i] * inv), f2bf(oacc[qb][db][i + 1] * inv),
                            f2bf(oacc[qb][db][i + 2] * inv), f2bf(oacc[qb][db][i + 3] * inv)};
          *(bf16x4*)o = v;
        }
    }
  }
}

// ============================================================== BF16-score, FP8 P V kernel
//
// Global attention with the scores in bfloat16 (Q K^T exactly as in
// attn_bf16_kernel) and the P V product on OCP E4M3 operands: probabilities
// and V codes, with V's per-128-row-block power-of-two scales entering the
// scaled f8f6f4 MFMA as E8M0 operands (relative to the head's largest V
// scale, vmax, as in attn_fp8_kernel).  The E4M3 rounding of Q and K, which
// moves logits of order 10 by several percent, is avoided; P and V are the
// only operands rounded to 3 mantissa bits.
//
// K tile rows are permuted so that lane group g of the score MFMA ends up
// with the 32 consecutive keys 32 g .. 32 g + 31 of the tile (register i of
// score block kb holds key 32 g + 16 kb + i): LDS row 32 kb + r holds key
// 32 ((r >> 2) & 1) + 16 kb + 4 (r >> 3) + (r & 3).  The 32 probabilities of
// a lane then form, in key order, the lane's B operand of the 32x32x64 E4M3
// MFMA, and the V^T tile (64 d rows of 64 one-byte keys, 16-byte granules
// swizzled with lds_swz4) is read in key order.
//
// Probabilities: the score MFMA works on Q times c2 = log2(e)/sqrt(D) and
// subtracts the shift sh in an extra k-step (as in attn_bf16_kernel), so
// p = 2^(s - sh) with sh = m - (log2(448) - 2), i.e. the row maximum m is
// placed two binades below 448 when it moves (sh rounded to bfloat16); later
// full tiles skip the maximum search and convert against the current sh.  A score that rose more
// than about two binades above the placed maximum converts to the E4M3 NaN
// code (the hardware conversion returns NaN above 464); the row-sum MFMA
// (16x16x128 with the lane selector, over the same E4M3 codes as the P V
// product) turns that into a NaN sum, which is tested on its bits, and only
// then is the exact step taken (scores recomputed from the K tile in LDS,
// maximum, rescale of O and l, new m).  The first and the partial last tile
// always take the exact step.  O = vmax * sum_j p8_j (s_v(j) / vmax) V8_j /
// sum_j p8_j, a convex combination of the decoded value rows.
template <int QB, int NW, int OCC>
__global__ __launch_bounds__(64 * NW, OCC) void attn_fp8pv_kernel(AttnParams p) {
  constexpr int BN = 64, D = kHeadDim, BM = 32 * QB * NW;
  constexpr float kPlace = 8.80735492205760410745f - 2.f;  // log2(448) - 2 binades of headroom
  __shared__ __attribute__((aligned(16))) bf16 Ks[2][BN * D];
  __shared__ __attribute__((aligned(16))) uint8_t Vs[2][D * BN];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 5, r32 = lane & 31;
  __shared__ int s_work;
  int head, item;
  take_work(p, &s_work, head, item);
  const Item it = resolve_item(p.seqs, item, BM);

  const bf16* Q = (const bf16*)p.q + head * p.q_hs;
  const bf16* K = (const bf16*)p.k + head * p.k_hs;
  const uint8_t* Vt = (const uint8_t*)p.vt + head * p.vt_hs + it.vb;
  const i32x2* KI = (const i32x2*)(p.kinfo + 2 * (head * p.sc_hs + it.bb));
  const float vmax = p.vmax[head];

  const bf16x8 zero8 = {};
  const int sel4 = (((lane >> 2) ^ (lane >> 4)) & 1) ? 0 : 0x38383838;  // row-sum selector: E4M3 1.0 or 0
  const i32x8 sel8 = {sel4, sel4, sel4, sel4, sel4, sel4, sel4, sel4};
  bf16x8 qf[QB][4];
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    const int row = it.q0 + (wave * QB + qb) * 32 + r32;
#pragma unroll
    for (int c = 0; c < 4; ++c)
      qf[qb][c] = row < it.s1 ? *(const bf16x8*)(Q + row * p.q_ts + 16 * c + 8 * g) : zero8;
  }
  // shift step of the score MFMA (as in attn_bf16_kernel): Q times c2, and
  // -sh (bfloat16) in k-slot 0 against a ones column, sh = the applied shift
  bf16x8 negm[QB];
  bf16x8 ones8 = zero8;
  if (g == 0) ones8[0] = (bf16)1.0f;
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int j = 0; j < 8; ++j) qf[qb][c][j] = f2bf(bf2f(qf[qb][c][j]) * p.scale_log2);
    negm[qb] = zero8;
  }

  // Tile t into LDS buffer buf.  K: 8 blocks of 8 rows x 128 bytes; V^T: 4
  // blocks of 16 rows x 64 bytes; wave w moves K blocks w, w + NW, ... and V
  // blocks w, w + NW, ... (lane l: K row 8 b + l / 8, slot l % 8; V row
  // 16 b + l / 4, slot l % 4).
  auto dma = [&](int t, int buf) {
    const int rows_left = it.s1 - (it.s0 + t * BN);
#pragma unroll
    for (int j = 0; j < 8 / NW; ++j) {
      const int rb = 8 * (wave + NW * j);
      const int R = rb + (lane >> 3), ch = (lane & 7) ^ lds_swz8(R);
      const int r = R & 31;
      const int key = 32 * ((r >> 2) & 1) + 16 * (R >> 5) + 4 * (r >> 3) + (r & 3);
      const int kr = key < rows_left ? key : 0;  // rows past the end: any existing key (their scores are masked)
      __builtin_amdgcn_global_load_lds((const void*)(K + (int64_t)(it.s0 + t * BN + kr) * p.k_ts + ch * 8),
                                       (__attribute__((address_space(3))) void*)&Ks[buf][rb * D], 16, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < (4 + NW - 1) / NW; ++j) {
      const int vb = wave + NW * j;
      if (vb < 4) {
        const int d = 16 * vb + (lane >> 2), ch = (lane & 3) ^ lds_swz4(d);
        __builtin_amdgcn_global_load_lds((const void*)(Vt + (int64_t)d * p.vt_ds + t * BN + ch * 16),
                                         (__attribute__((address_space(3))) void*)&Vs[buf][16 * vb * BN], 16, 0, 0);
      }
    }
  };

  f32x16 oacc[QB][2];
  float m_run[QB], l_run[QB];
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    oacc[qb][0] = f32x16{};
    oacc[qb][1] = f32x16{};
    m_run[qb] = 0.f;  // the applied shift, set by the first tile
    l_run[qb] = 0.f;
  }
  const int ntiles = (it.s1 - it.s0 + BN - 1) / BN;

  dma(0, 0);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();

  auto tile = [&](int t, auto masked, auto first) {
    constexpr bool MASKED = decltype(masked)::value, FIRST = decltype(first)::value;
    constexpr bool EXACT = MASKED || FIRST;
    const int kt = it.s0 + t * BN, buf = t & 1;
    const int ev = KI[(kt - it.s0) / kQuantRows][1];  // E8M0 code of this key block's V scale / vmax

    bf16x8 kf[2][4];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int r = kb * 32 + r32;
        kf[kb][c] = *(const bf16x8*)&Ks[buf][r * D + (((2 * c + g) ^ lds_swz8(r)) * 8)];
      }
    f32x16 s[QB][2];
    i32x8 pw[QB];
    i32x8 vf[2];
    auto score = [&](int qb) {
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        s[qb][kb] = mfma_bf16(ones8, negm[qb], f32x16{});
#pragma unroll
        for (int c = 0; c < 4; ++c) s[qb][kb] = mfma_bf16(kf[kb][c], qf[qb][c], s[qb][kb]);
      }
    };
    auto pv = [&](int qb) {
      oacc[qb][0] = mfma_fp8_scaled(vf[0], pw[qb], oacc[qb][0], ev, 127);
      oacc[qb][1] = mfma_fp8_scaled(vf[1], pw[qb], oacc[qb][1], ev, 127);
    };
    // E4M3 probabilities of one query block, in key order (32 per lane); the
    // scores already hold s - sh
    auto probs = [&](int qb, const f32x16& a, const f32x16& b) {
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        const f32x16& x = kb ? b : a;
#pragma unroll
        for (int i = 0; i < 16; i += 4)
          pw[qb][(16 * kb + i) >> 2] =
              pack_e4m3x4(fast_exp2(x[i]), fast_exp2(x[i + 1]), fast_exp2(x[i + 2]), fast_exp2(x[i + 3]));
      }
    };
    auto rowsum = [&](int qb) { return mfma_fp8_16(sel8, pw[qb], f32x4{})[0]; };
    auto exact = [&](int qb, f32x16& a, f32x16& b, auto is_first) {
      if (MASKED) {
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
          for (int i = 0; i < 16; ++i)
            if (kt + 32 * g + 16 * kb + i >= it.s1) (kb ? b : a)[i] = -INFINITY;
      }
      const float mx = lane_swap_max(max32(a, b));
      // scores relative to the applied shift sh = m_run; the row maximum is
      // placed kPlace binades up when it moves (sh rounded to bfloat16, the
      // type it enters the MFMA in); on the first tile O and l are zero
      constexpr bool F_ = decltype(is_first)::value;
      const float base = F_ ? 0.f : m_run[qb];
      const float want = F_ ? mx - kPlace : __builtin_fmaxf(mx - kPlace, 0.f);
      const float d = bf2f(f2bf(base + want)) - base;
      if (!F_) {
        const float alpha = fast_exp2(-d);
        l_run[qb] *= alpha;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          oacc[qb][0][i] *= alpha;
          oacc[qb][1][i] *= alpha;
        }
      }
      m_run[qb] = base + d;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        a[i] -= d;
        b[i] -= d;
      }
      if (g == 0) negm[qb][0] = f2bf(-m_run[qb]);
      probs(qb, a, b);
    };

    score(0);
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
      __builtin_amdgcn_sched_barrier(0);
      if (qb + 1 < QB) score(qb + 1);
      if (qb >= 1) pv(qb - 1);
      if (EXACT) exact(qb, s[qb][0], s[qb][1], first);
      else probs(qb, s[qb][0], s[qb][1]);
      if (!EXACT && QB > 1) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          __builtin_amdgcn_sched_group_barrier(0x002, 8, 0);  // VALU
          __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
        }
      }
      if (qb == 0) {
#pragma unroll
        for (int db = 0; db < 2; ++db) {
          const int d = db * 32 + r32, sw = lds_swz4(d);
          const i32x4 lo = *(const i32x4*)&Vs[buf][d * BN + (((2 * g) ^ sw) * 16)];
          const i32x4 hi = *(const i32x4*)&Vs[buf][d * BN + (((2 * g + 1) ^ sw) * 16)];
          vf[db] = i32x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
        }
        // every LDS read of this tile's fragments is issued: move the next tile in
        if (t + 1 < ntiles) dma(t + 1, buf ^ 1);
      }
      float ls = rowsum(qb);
      if (!EXACT && __any(abs_bits_at_least(ls, 0x7f800000u))) {
        f32x16 r[2];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
          r[kb] = mfma_bf16(ones8, negm[qb], f32x16{});
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const int rr = kb * 32 + r32;
            const bf16x8 k8 = *(const volatile bf16x8*)&Ks[buf][rr * D + (((2 * c + g) ^ lds_swz8(rr)) * 8)];
            r[kb] = mfma_bf16(k8, qf[qb][c], r[kb]);
          }
        }
        exact(qb, r[0], r[1], std::false_type{});
        ls = rowsum(qb);
      }
      l_run[qb] += ls;
    }
    __builtin_amdgcn_sched_barrier(0);
    pv(QB - 1);
    __builtin_amdgcn_sched_barrier(0);
    if (t + 1 < ntiles) {
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
    }
  };
  const bool ragged = (it.s1 - it.s0) % BN != 0;
  const int nfull = ntiles - (ragged ? 1 : 0);
  if (nfull > 0) tile(0, std::false_type{}, std::true_type{});
  for (int t = 1; t < nfull; ++t) tile(t, std::false_type{}, std::false_type{});
  if (ragged) {
    if (ntiles == 1)
      tile(0, std::true_type{}, std::true_type{});
    else
      tile(ntiles - 1, std::true_type{}, std::false_type{});
  }

#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    const float inv = vmax / l_run[qb];
    const int row = it.q0 + (wave * QB + qb) * 32 + r32;
    if (row < it.s1) {
#pragma unroll
      for (int db = 0; db < 2; ++db)
#pragma unroll
        for (int i = 0; i < 16; i += 4) {
          const int d = db * 32 + 8 * (i >> 2) + 4 * g;
          bf16* o = (bf16*)p.o + row * p.o_ts + head * p.o_hs + d;
          const bf16x4 v = {f2bf(oacc[qb][db][i] * inv), f2bf(oacc[qb][db][i + 1] * inv),
                            f2bf(oacc[qb][db][i + 2] * inv), f2bf(oacc[qb][db][i + 3] * inv)};
          *(bf16x4*)o = v;
        }
    }
  }
}

// ============================================================== FP32 kernel
// Same structure on the float32 MFMA (32x32x2): 32 queries per wave, BN = 32
// keys per tile, K and V key-major in LDS with padded rows.
__global__ __launch_bounds__(256, 1) void attn_f32_kernel(AttnParams p) {
  constexpr int BN = 32, D = kHeadDim, BM = 128;
  __shared__ float Ks[2][BN][D + 1];
  __shared__ float Vs[2][BN][D + 4];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 5, r32 = lane & 31;
  const int head = blockIdx.y;
  const Item it = resolve_item(p.seqs, blockIdx.x, BM);
  const float* Q = (const float*)p.q + head * p.q_hs;
  const float* K = (const float*)p.k + head * p.k_hs;
  const float* V = (const float*)p.v + head * p.v_hs;

  float qf[32];
  const int qrow = it.q0 + wave * 32 + r32;
#pragma unroll
  for (int c = 0; c < 32; ++c) qf[c] = qrow < it.s1 ? Q[qrow * p.q_ts + 2 * c + g] : 0.f;

  f32x4 kreg[2], vreg[2];
  const int lr = tid >> 3, ld0 = (tid & 7) * 8;
  auto gload = [&](int kt) {
    const int key = kt + lr;
    const f32x4 z = {};
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      kreg[i] = key < it.s1 ? *(const f32x4*)(K + key * p.k_ts + ld0 + 4 * i) : z;
      vreg[i] = key < it.s1 ? *(const f32x4*)(V + key * p.v_ts + ld0 + 4 * i) : z;
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        Ks[buf][lr][ld0 + 4 * i + j] = kreg[i][j];
        Vs[buf][lr][ld0 + 4 * i + j] = vreg[i][j];
      }
  };

  f32x16 oacc[2] = {f32x16{}, f32x16{}};
  float m_run = -INFINITY, l_run = 0.f;
  const float c2 = p.scale_log2;
  const int ntiles = (it.s1 - it.s0 + BN - 1) / BN;
  gload(it.s0);
  lstore(0);
  __syncthreads();
  for (int t = 0; t < ntiles; ++t) {
    const int kt = it.s0 + t * BN, buf = t & 1;
    if (t + 1 < ntiles) gload(kt + BN);
    f32x16 s = {};
#pragma unroll
    for (int c = 0; c < 32; ++c) s = mfma_f32(Ks[buf][r32][2 * c + g], qf[c], s);
    if (kt + BN > it.s1) {
#pragma unroll
      for (int i = 0; i < 16; ++i)
        if (kt + 8 * (i >> 2) + 4 * g + (i & 3) >= it.s1) s[i] = -INFINITY;
    }
    float mx = s[0];
#pragma unroll
    for (int i = 1; i < 16; ++i) mx = __builtin_fmaxf(mx, s[i]);
    mx = __builtin_fmaxf(mx, __shfl_xor(mx, 32));
    const float m_new = __builtin_fmaxf(m_run, mx);
    const float alpha = fast_exp2((m_run - m_new) * c2);
    m_run = m_new;
    l_run *= alpha;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      oacc[0][i] *= alpha;
      oacc[1][i] *= alpha;
    }
    const float mc = m_new * c2;
    float pv[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      pv[i] = fast_exp2(__builtin_fmaf(s[i], c2, -mc));
      l_run += pv[i];
    }
#pragma unroll
    for (int db = 0; db < 2; ++db)
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        const int key = 8 * (c >> 2) + 4 * g + (c & 3);
        oacc[db] = mfma_f32(Vs[buf][key][db * 32 + r32], pv[c], oacc[db]);
      }
    if (t + 1 < ntiles) lstore(buf ^ 1);
    __syncthreads();
  }
  const float lt = l_run + __shfl_xor(l_run, 32);
  const float inv = 1.f / lt;
  if (qrow < it.s1) {
#pragma unroll
    for (int db = 0; db < 2; ++db)
#pragma unroll
      for (int i = 0; i < 16; i += 4) {
        const int d = db * 32 + 8 * (i >> 2) + 4 * g;
        float* o = (float*)p.o + qrow * p.o_ts + head * p.o_hs + d;
        const f32x4 v = {oacc[db][i] * inv, oacc[db][i + 1] * inv, oacc[db][i + 2] * inv, oacc[db][i + 3] * inv};
        *(f32x4*)o = v;
      }
  }
}


// ============================================================== FP8 kernel
// E4M3 probabilities 2^x of one 32-query x 64-key score block, packed as the
// B operand of the P V product.
__device__ __forceinline__ i32x8 probs(const f32x16& a, const f32x16& b) {
  i32x8 pw;
#pragma unroll
  for (int kb = 0; kb < 2; ++kb) {
    const f32x16& x = kb ? b : a;
#pragma unroll
    for (int i = 0; i < 16; i += 4)
      pw[(16 * kb + i) >> 2] = pack_e4m3x4(fast_exp2(x[i]), fast_exp2(x[i + 1]), fast_exp2(x[i + 2]),
                                           fast_exp2(x[i + 3]));
  }
  return pw;
}

// Global attention on OCP E4M3 operands (MFMA 32x32x64 f8f6f4 with E8M0
// block scales, one MFMA per 32x32 score block since K = D = 64).  Q, K and V
// carry one power-of-two scale per 128-row block of their sequence, and Q was
// quantised after multiplication by log2(e)/sqrt(D), so the scaled MFMA
// yields base-2 logits directly: the Q- and K-block scales enter as the
// instruction's E8M0 operands.  The accumulator input of the score MFMA is
// log2(448) - m per query row, so the MFMA result x is already the exponent:
// p = 2^x is the E4M3-ready probability and the tile needs no per-score
// multiply-add.  m is not the running maximum itself: a rescale places the
// row maximum kHeadroom binades below 448, and later tiles skip the maximum
// search altogether.  They convert 2^x against the current m; a score that
// rose more than kHeadroom (+ log2(464/448)) binades above the placed
// maximum converts to the NaN code, the row-sum MFMA turns that into a NaN
// sum, and only then are the tile's scores recomputed from the K tile still
// in LDS and the exact step taken (maximum, rescale, new m).  The first tile
// and the partial last tile always take the exact step.  Softmax is
// shift-invariant, so the result does not depend on m; the headroom costs
// kHeadroom binades of E4M3 range at the small end (probabilities below
// 2^-9, the smallest subnormal, flush to zero).
//
// The V-block scale s_v(b) / vmax enters the P V MFMA as its E8M0 operand
// for the V tile, so one PV accumulator serves every key block and
// O = vmax * sum_j p8_j (s_v(j) / vmax) V8_j / sum_j p8_j.  The row sum is
// taken from the same rounded p8 values that feed the PV product, so the
// output stays a convex combination of value rows whatever the rounding of
// P.  It runs on the 16x16x128 MFMA (half the cycles of a 32x32x64 one) and
// accumulates in that MFMA's accumulator: read as its B operand, the
// probability registers are 16 columns whose 4 lane groups (k-groups) hold
// queries n, n+16, n, n+16; the selector A (rows 4j..4j+3 take the groups
// of parity j&1, E4M3 1.0 or 0) makes output lane l, which holds rows
// 4*(l/16)+i, receive the sum for its own query l%32 in all four registers.
//
// LDS: Ks[row][d] bytes and Vs[d][key] bytes (V^T in key order), 16-byte
//      granules swizzled with lds_swz4(row) and lds_swz4(d), both filled by
//      direct-to-LDS loads.  The K rows of each 32-row block are permuted
//      (row 32 kb + r holds key 32 ((r >> 2) & 1) + 16 kb + 4 (r >> 3) + (r & 3))
//      so that the score registers of lane group g hold the 32 consecutive
//      keys 32 g .. 32 g + 31, the keys whose V^T bytes the same group reads
//      from granules 2 g and 2 g + 1 of a V^T row: P goes from the score
//      accumulator to the P V operand with no permutation.
template <int QB, int NW, int OCC>
__global__ __launch_bounds__(64 * NW, OCC) void attn_fp8_kernel(AttnParams p) {
  constexpr int BN = 64, D = kHeadDim, BM = 32 * QB * NW;
  constexpr float kLog2Max = 8.80735492205760410745f;  // log2(448)
  // a rescale places the row maximum this many binades below 448, so that
  // later tiles may raise it by up to a factor 2^kHeadroom without overflow
  constexpr float kHeadroom = 2.f;
  constexpr float kPlace = kLog2Max - kHeadroom;
  __shared__ __attribute__((aligned(16))) uint8_t Ks[2][BN * D];
  __shared__ __attribute__((aligned(16))) uint8_t Vs[2][D * BN];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 5, r32 = lane & 31;
  __shared__ int s_work;
  int head, item;
  take_work(p, &s_work, head, item);
  const Item it = resolve_item(p.seqs, item, BM);
  const uint8_t* Q = (const uint8_t*)p.q + head * p.q_hs;
  const uint8_t* K = (const uint8_t*)p.k + head * p.k_hs;
  const uint8_t* Vt = (const uint8_t*)p.vt + head * p.vt_hs + it.vb;
  const float* SQ = p.sq + head * p.sc_hs + it.bb;
  const i32x2* KI = (const i32x2*)(p.kinfo + 2 * (head * p.sc_hs + it.bb));
  const float vmax = p.vmax[head];

  const i32x8 zero8 = {};
  // row-sum selector (see above)
  const int sel4 = (((lane >> 2) ^ (lane >> 4)) & 1) ? 0 : 0x38383838;  // E4M3 1.0 codes or 0
  const i32x8 sel8 = {sel4, sel4, sel4, sel4, sel4, sel4, sel4, sel4};
  i32x8 qf[QB];
  int eq[QB];  // E8M0 code of the query block's scale
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    const int row = it.q0 + (wave * QB + qb) * 32 + r32;
    qf[qb] = row < it.s1 ? *(const i32x8*)(Q + row * p.q_ts + 32 * g) : zero8;
    // the 32 rows of a query block lie inside one 128-row scale block
    eq[qb] = (int)(__float_as_uint(SQ[(it.q0 - it.s0 + (wave * QB + qb) * 32) / kQuantRows]) >> 23);
  }

  // Tile t into LDS buffer buf: 4 blocks of 16 K rows and 4 blocks of 16 V^T
  // rows (64 B each, 1 KB per block); wave w moves blocks w, w + NW, ...
  // (blocks 0-3 K, 4-7 V^T).  K rows permuted so that each lane group's
  // score registers hold 32 consecutive keys (LDS row 32 kb + r holds key
  // 32 ((r >> 2) & 1) + 16 kb + 4 (r >> 3) + (r & 3)); V^T in key order.
  auto dma = [&](int t, int buf) {
    const int rows_left = it.s1 - (it.s0 + t * BN);
#pragma unroll
    for (int j = 0; j < (8 + NW - 1) / NW; ++j) {
      const int b = wave + NW * j;
      if (b < 4) {
        const int R = 16 * b + (lane >> 2), ch = (lane & 3) ^ lds_swz4(R);
        const int r = R & 31;
        const int key = 32 * ((r >> 2) & 1) + 16 * (R >> 5) + 4 * (r >> 3) + (r & 3);
        const int kr = key < rows_left ? key : 0;  // rows past the end: any existing key (masked)
        __builtin_amdgcn_global_load_lds((const void*)(K + (int64_t)(it.s0 + t * BN + kr) * p.k_ts + ch * 16),
                                         (__attribute__((address_space(3))) void*)&Ks[buf][16 * b * D], 16, 0, 0);
      } else if (b < 8) {
        const int d = 16 * (b - 4) + (lane >> 2), ch = (lane & 3) ^ lds_swz4(d);
        __builtin_amdgcn_global_load_lds((const void*)(Vt + (int64_t)d * p.vt_ds + t * BN + ch * 16),
                                         (__attribute__((address_space(3))) void*)&Vs[buf][16 * (b - 4) * BN], 16,
                                         0, 0);
      }
    }
  };

  f32x16 oacc[QB][2];
  f32x16 cin[QB];  // accumulator input of the score MFMA: log2(448) - m, per query
  float m_run[QB];
  f32x4 lacc[QB];  // running row sum, kept in the row-sum MFMA's accumulator (4 equal copies)
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    oacc[qb][0] = f32x16{};
    oacc[qb][1] = f32x16{};
    cin[qb] = f32x16{};
    m_run[qb] = kLog2Max;  // consistent with cin = 0; the first tile always places m
    lacc[qb] = f32x4{};
  }
  const int ntiles = (it.s1 - it.s0 + BN - 1) / BN;
  dma(0, 0);
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  // One key tile.  MASKED is set only for the final, partial tile of a
  // sequence, so full tiles carry no key-bound checks; FIRST only for the
  // first tile.  Both take the exact step on every query block, the other
  // tiles the overflow-checked one.
  auto tile = [&](int t, auto masked, auto first) {
    constexpr bool MASKED = decltype(masked)::value, FIRST = decltype(first)::value;
    constexpr bool EXACT = MASKED || FIRST;
    const int kt = it.s0 + t * BN, buf = t & 1;
    i32x8 kf[2];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) {
      const int r = kb * 32 + r32, sw = lds_swz4(r);
      const i32x4 lo = *(const i32x4*)&Ks[buf][r * D + (((2 * g) ^ sw) * 16)];
      const i32x4 hi = *(const i32x4*)&Ks[buf][r * D + (((2 * g + 1) ^ sw) * 16)];
      kf[kb] = i32x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    }
    // key-block E8M0 codes: K scale, V scale relative to vmax
    const i32x2 ki = KI[(kt - it.s0) / kQuantRows];
    f32x16 s[QB][2];
    i32x8 pw[QB];
    i32x8 vf[2];  // V fragments, read during the first query block
    auto score = [&](int qb) {
      s[qb][0] = mfma_fp8_scaled(kf[0], qf[qb], cin[qb], ki[0], eq[qb]);
      s[qb][1] = mfma_fp8_scaled(kf[1], qf[qb], cin[qb], ki[0], eq[qb]);
    };
    auto pv = [&](int qb) {
      oacc[qb][0] = mfma_fp8_scaled(vf[0], pw[qb], oacc[qb][0], ki[1], 127);
      oacc[qb][1] = mfma_fp8_scaled(vf[1], pw[qb], oacc[qb][1], ki[1], 127);
    };
    // Exact step: mask, row maximum, rescale when the maximum grew (always on
    // the first tile), then the probabilities.
    auto exact_probs = [&](int qb, f32x16& a, f32x16& b) {
      if (MASKED) {
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
          for (int i = 0; i < 16; ++i)
            if (kt + 32 * g + 16 * kb + i >= it.s1) (kb ? b : a)[i] = -INFINITY;
      }
      const float xmax = lane_swap_max(max32(a, b));
      if (FIRST || __any(xmax > kLog2Max)) {
        // the first tile places the maximum; later tiles move it only for
        // rows that would exceed 448
        const float delta = FIRST ? xmax - kPlace : (xmax > kLog2Max ? xmax - kPlace : 0.f);
        // on the first tile l and O are still zero: no rescale (2^-delta may
        // overflow there when every logit of the tile is very negative)
        const float alpha = FIRST ? 0.f : fast_exp2(-delta);
#pragma unroll
        for (int i = 0; i < 4; ++i) lacc[qb][i] *= alpha;
        m_run[qb] += delta;
        const float c = kLog2Max - m_run[qb];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          oacc[qb][0][i] *= alpha;
          oacc[qb][1][i] *= alpha;
          a[i] -= delta;
          b[i] -= delta;
          cin[qb][i] = c;
        }
      }
      return probs(a, b);
    };
    // Query blocks in turn.  While the vector ALU runs the exponentials of
    // block qb, the matrix core gets the score MFMAs of block qb+1 and the
    // P V MFMAs of block qb-1, issued between the exponentials (scheduling
    // groups), so that one wave keeps both units busy.
    score(0);
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
      __builtin_amdgcn_sched_barrier(0);
      if (qb + 1 < QB) score(qb + 1);
      if (qb >= 1) pv(qb - 1);
      pw[qb] = EXACT ? exact_probs(qb, s[qb][0], s[qb][1]) : probs(s[qb][0], s[qb][1]);
      if (!EXACT && QB > 1) {
        __builtin_amdgcn_sched_group_barrier(0x002, 12, 0);  // VALU
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
        __builtin_amdgcn_sched_group_barrier(0x002, 12, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      }
      f32x4 lsum = mfma_fp8_16(sel8, pw[qb], lacc[qb]);
      if (qb == 0) {
#pragma unroll
        for (int db = 0; db < 2; ++db) {
          const int d = db * 32 + r32, sw = lds_swz4(d);
          const i32x4 lo = *(const i32x4*)&Vs[buf][d * BN + (((2 * g) ^ sw) * 16)];
          const i32x4 hi = *(const i32x4*)&Vs[buf][d * BN + (((2 * g + 1) ^ sw) * 16)];
          vf[db] = i32x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
        }
        // every LDS read of this tile's fragments is issued: move the next tile in
        if (t + 1 < ntiles) dma(t + 1, buf ^ 1);
      }
      // full tiles after the first: probabilities against the current m; a
      // NaN code makes the row sum NaN (tested on the bits, not with a float
      // compare: this file is built without NaN semantics), and only then
      // are the scores recomputed from the K tile in LDS for the exact step
      if (!EXACT && __any(abs_bits_at_least(lsum[0], 0x7f800000u))) {
        f32x16 r[2];
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) {
          const int rr = kb * 32 + r32, sw = lds_swz4(rr);
          const i32x4 lo = *(const volatile i32x4*)&Ks[buf][rr * D + (((2 * g) ^ sw) * 16)];
          const i32x4 hi = *(const volatile i32x4*)&Ks[buf][rr * D + (((2 * g + 1) ^ sw) * 16)];
          const i32x8 k8 = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
          r[kb] = mfma_fp8_scaled(k8, qf[qb], cin[qb], ki[0], eq[qb]);
        }
        pw[qb] = exact_probs(qb, r[0], r[1]);
        lsum = mfma_fp8_16(sel8, pw[qb], lacc[qb]);
      }
      lacc[qb] = lsum;
    }
    __builtin_amdgcn_sched_barrier(0);
    pv(QB - 1);
    __builtin_amdgcn_sched_barrier(0);
    if (t + 1 < ntiles) {
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      __syncthreads();
    }
  };
  const bool ragged = (it.s1 - it.s0) % BN != 0;
  const int nfull = ntiles - (ragged ? 1 : 0);
  if (nfull > 0) tile(0, std::false_type{}, std::true_type{});
  for (int t = 1; t < nfull; ++t) tile(t, std::false_type{}, std::false_type{});
  if (ragged) {
    if (ntiles == 1)
      tile(0, std::true_type{}, std::true_type{});
    else
      tile(ntiles - 1, std::true_type{}, std::false_type{});
  }
#pragma unroll
  for (int qb = 0; qb < QB; ++qb) {
    const float inv = vmax / lacc[qb][0];
    const int qrow = it.q0 + (wave * QB + qb) * 32 + r32;
    if (qrow < it.s1) {
#pragma unroll
      for (int db = 0; db < 2; ++db)
#pragma unroll
        for (int i = 0; i < 16; i += 4) {
          const int d = db * 32 + 8 * (i >> 2) + 4 * g;
          bf16* o = (bf16*)p.o + qrow * p.o_ts + head * p.o_hs + d;
          const bf16x4 v = {f2bf(oacc[qb][db][i] * inv), f2bf(oacc[qb][db][i + 1] * inv),
                            f2bf(oacc[qb][db][i + 2] * inv), f2bf(oacc[qb][db][i + 3] * inv)};
          *(bf16x4*)o = v;
        }
    }
  }
}

// ============================================================== V transpose
// One workgroup per (64-token tile, head): v [tokens, H, D] -> vt[h][d][col]
// with every sequence starting at a multiple of 64 columns; columns past the
// end of a sequence are written as zeros.
__global__ __launch_bounds__(256) void v_transpose_bf16_kernel(const bf16* v, int64_t v_ts, int64_t v_hs, bf16* vt,
                                                               int64_t vt_hs, int64_t vt_ds, SeqTable seqs) {
  __shared__ bf16 T[64][64 + 2];
  const int tid = threadIdx.x, head = blockIdx.y;
  const Item it = resolve_item(seqs, blockIdx.x, 64);
  const bf16* V = v + head * v_hs;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int r = (tid >> 3) + 32 * i, ch = tid & 7;
    const int row = it.q0 + r;
    bf16x8 x = {};
    if (row < it.s1) x = *(const bf16x8*)(V + row * v_ts + ch * 8);
#pragma unroll
    for (int j = 0; j < 8; ++j) T[r][ch * 8 + j] = x[j];
  }
  __syncthreads();
  bf16* out = vt + head * vt_hs + it.vb + (it.q0 - it.s0);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int d = (tid >> 3) + 32 * i, ch = tid & 7;
    bf16x8 y;
#pragma unroll
    for (int j = 0; j < 8; ++j) y[j] = T[ch * 8 + j][d];
    *(bf16x8*)(out + d * vt_ds + ch * 8) = y;
  }
}

// ============================================================== FP8 quantiser
// Smallest integer e with amax <= 448 * 2^e, clamped to [-127, 127]; 0 for
// amax = 0.  With amax = M * 2^A (M in [1, 2)): 448 * 2^e = 1.75 * 2^(e + 8),
// so e = A - 8, plus one when M > 1.75 (mantissa field above 0x600000).
__device__ __forceinline__ int block_exponent(float amax) {
  if (!(amax > 0.f)) return 0;
  const uint32_t b = __float_as_uint(amax);
  const int ef = (int)(b >> 23);  // biased exponent; amax > 0, so no sign bit
  if (ef == 0) return -127;       // subnormal amax: the clamp applies
  const int e = ef - 127 - 8 + ((b & 0x7fffffu) > 0x600000u ? 1 : 0);
  return e < -127 ? -127 : (e > 127 ? 127 : e);
}

// 2^e as a float for e in [-127, 127] (2^-127 is the subnormal 0x00400000).
__device__ __forceinline__ float exp2i(int e) {
  return e >= -126 ? __uint_as_float((uint32_t)(e + 127) << 23) : __uint_as_float(0x00400000u);
}

// One workgroup per (128-row scale block, head).  x' = x * pre (float32);
// amax over the block's rows and all D columns; s = 2^e with
// e = block_exponent(amax); codes = E4M3(x' / s), the division by a power of
// two being exact.  s is stored as a float (an exact power of two, so its
// exponent field is the OCP E8M0 code of the scale).
__global__ __launch_bounds__(256) void quant_fp8_kernel(const bf16* x, int64_t x_ts, int64_t x_hs, float pre,
                                                        uint8_t* codes, int64_t c_hs, int64_t c_ds, int transposed,
                                                        int64_t out_row0, float* scales, int64_t sc_hs,
                                                        SeqTable seqs) {
  __shared__ float red[4];
  __shared__ uint8_t T[64][128 + 4];
  const int tid = threadIdx.x, head = blockIdx.y;
  const Item it = resolve_item(seqs, blockIdx.x, kQuantRows);
  const int blk = it.bb + (it.q0 - it.s0) / kQuantRows;
  const bf16* X = x + head * x_hs;
  const int r = tid >> 1, half = tid & 1;
  const int row = it.q0 + r;
  float v[32];
  const bool valid = row < it.s1;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    bf16x8 t = {};
    if (valid) t = *(const bf16x8*)(X + row * x_ts + half * 32 + 8 * c);
#pragma unroll
    for (int j = 0; j < 8; ++j) v[8 * c + j] = bf2f(t[j]) * pre;
  }
  float amax = 0.f;
#pragma unroll
  for (int j = 0; j < 32; ++j) amax = __builtin_fmaxf(amax, __builtin_fabsf(v[j]));
  amax = wave_max(amax);
  if ((tid & 63) == 0) red[tid >> 6] = amax;
  __syncthreads();
  amax = __builtin_fmaxf(__builtin_fmaxf(red[0], red[1]), __builtin_fmaxf(red[2], red[3]));
  const int ex = block_exponent(amax);
  const float inv = exp2i(-ex);
  if (tid == 0) scales[head * sc_hs + blk] = exp2i(ex);
  uint32_t w[8];
#pragma unroll
  for (int j = 0; j < 8; ++j)
    w[j] = cvt_e4m3x2(v[4 * j] * inv, v[4 * j + 1] * inv) | (cvt_e4m3x2(v[4 * j + 2] * inv, v[4 * j + 3] * inv) << 16);
  if (!transposed) {
    if (valid) {
      uint8_t* o = codes + head * c_hs + (out_row0 + row) * kHeadDim + half * 32;
      const i32x4 a = {(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
      const i32x4 b = {(int)w[4], (int)w[5], (int)w[6], (int)w[7]};
      *(i32x4*)o = a;
      *(i32x4*)(o + 16) = b;
    }
    return;
  }
  // transposed: stage [d][row] in LDS, then write padded rows of codes
#pragma unroll
  for (int j = 0; j < 32; ++j) T[half * 32 + j][r] = (uint8_t)((w[j >> 2] >> (8 * (j & 3))) & 0xff);
  __syncthreads();
  const int len = it.s1 - it.s0;
  const int padlen = (len + kKeyPad - 1) / kKeyPad * kKeyPad;
  const int c0 = it.q0 - it.s0;
  const int ncols = min(kQuantRows, padlen - c0);  // 64 or 128
  uint8_t* o = codes + head * c_hs + it.vb + c0;
  // 64 rows (d) x ncols bytes; each thread writes 16-byte pieces
  const int pieces = ncols / 16;
  for (int idx = tid; idx < 64 * pieces; idx += 256) {
    const int d = idx / pieces, pc = idx % pieces;
    uint32_t q4[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      uint32_t word = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int col = pc * 16 + 4 * k + b;
        const uint8_t cv = (c0 + col < len) ? T[d][col] : (uint8_t)0;
        word |= (uint32_t)cv << (8 * b);
      }
      q4[k] = word;
    }
    const i32x4 a = {(int)q4[0], (int)q4[1], (int)q4[2], (int)q4[3]};
    *(i32x4*)(o + d * c_ds + pc * 16) = a;
  }
}

// Per head: vmax = the largest V block scale (a power of two), then the E8M0
// codes the FP8 attention kernel hands to the matrix instructions, per key
// block b: kinfo[b] = {E8M0(s_k(b)), E8M0(s_v(b) / vmax)} (the latter clamped
// at 2^-127).  An exact power of two's float exponent field is its E8M0 code.
__global__ void scale_max_kernel(const float* sk, const float* sv, int64_t sc_hs, int n_blocks, float* vmax,
                                 int* kinfo) {
  const int head = blockIdx.x;
  float m = 0.f;
  for (int i = threadIdx.x; i < n_blocks; i += 64) m = __builtin_fmaxf(m, sv[head * sc_hs + i]);
  m = wave_max(m);
  if (threadIdx.x == 0) vmax[head] = m;
  const int em = (int)(__float_as_uint(m) >> 23);
  for (int i = threadIdx.x; i < n_blocks; i += 64) {
    const int64_t b = head * sc_hs + i;
    const int ev = (int)(__float_as_uint(sv[b]) >> 23) - em + 127;
    const i32x2 ki = {(int)(__float_as_uint(sk[b]) >> 23), ev < 0 ? 0 : ev};
    *(i32x2*)(kinfo + 2 * b) = ki;
  }
}

// ============================================================== launchers
// Kernel variants: (32-row query blocks per wave, waves per workgroup, waves
// per SIMD the register budget is sized for; the occupancy reached is set by
// the registers actually used).  Every variant of one
// precision performs the same per-row arithmetic in the same order, so they
// agree bitwise; they differ in LDS reuse, register pressure and occupancy.
struct AttnVariant {
  int qb, nw, occ;
};
static const AttnVariant kBf16Variants[] = {{1, 4, 2}, {2, 4, 2}, {1, 8, 2}};
static const AttnVariant kFp8Variants[] = {{1, 4, 2}, {2, 4, 2}, {1, 8, 2}, {2, 8, 2}};
constexpr int kNumBf16Variants = sizeof(kBf16Variants) / sizeof(kBf16Variants[0]);
constexpr int kNumFp8Variants = sizeof(kFp8Variants) / sizeof(kFp8Variants[0]);

int attn_n_variants(int prec) {
  if (prec == 1) return kNumBf16Variants;
  if (prec == 2) return kNumFp8Variants;
  return 1;
}

int attn_block_rows(int prec, int variant) {
  if (prec == 1 && variant >= 0 && variant < kNumBf16Variants)
    return 32 * kBf16Variants[variant].qb * kBf16Variants[variant].nw;
  if (prec == 2 && variant >= 0 && variant < kNumFp8Variants)
    return 32 * kFp8Variants[variant].qb * kFp8Variants[variant].nw;
  return 128;
}

__global__ void zero_i32_kernel(int* x, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = 0;
}

// Grid launch (workgroup (x, y) = item x of head y) or, with p.queue, the
// counter reset and one workgroup per (item, head) in x, each taking its work
// index from the counter (take_work).
template <typename Kernel>
static hipError_t launch_attn_kernel(Kernel kernel, const AttnParams& p, int H, int threads, hipStream_t s) {
  if (p.n_items <= 0 || H <= 0) return hipSuccess;
  if (!p.queue) return launch(kernel, dim3(p.n_items, H), dim3(threads), 0, s, p);
  const int64_t n_work = (int64_t)H * p.n_items;
  if (p.n_heads != H || n_work > INT32_MAX) return hipErrorInvalidValue;
  const hipError_t e = launch(zero_i32_kernel, dim3(1), dim3(64), 0, s, p.queue, 1);
  if (e != hipSuccess) return e;
  return launch(kernel, dim3((unsigned)n_work), dim3(threads), 0, s, p);
}

hipError_t launch_attn_bf16(const AttnParams& p, int H, int variant, hipStream_t s) {
  switch (variant) {
    case 0: return launch_attn_kernel(attn_bf16_kernel<1, 4, 2>, p, H, 256, s);
    case 1: return launch_attn_kernel(attn_bf16_kernel<2, 4, 2>, p, H, 256, s);
    case 2: return launch_attn_kernel(attn_bf16_kernel<1, 8, 2>, p, H, 512, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_attn_fp8pv(const AttnParams& p, int H, int variant, hipStream_t s) {
  switch (variant) {
    case 0: return launch_attn_kernel(attn_fp8pv_kernel<1, 4, 2>, p, H, 256, s);
    case 1: return launch_attn_kernel(attn_fp8pv_kernel<2, 4, 2>, p, H, 256, s);
    case 2: return launch_attn_kernel(attn_fp8pv_kernel<1, 8, 2>, p, H, 512, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_attn_f32(const AttnParams& p, int H, hipStream_t s) {
  if (p.queue) return hipErrorInvalidValue;  // grid mode only
  return launch(attn_f32_kernel, dim3(p.n_items, H), dim3(256), 0, s, p);
}

hipError_t launch_attn_fp8(const AttnParams& p, int H, int variant, hipStream_t s) {
  switch (variant) {
    case 0: return launch_attn_kernel(attn_fp8_kernel<1, 4, 2>, p, H, 256, s);
    case 1: return launch_attn_kernel(attn_fp8_kernel<2, 4, 2>, p, H, 256, s);
    case 2: return launch_attn_kernel(attn_fp8_kernel<1, 8, 2>, p, H, 512, s);
    case 3: return launch_attn_kernel(attn_fp8_kernel<2, 8, 2>, p, H, 512, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_v_transpose_bf16(const bf16* v, int64_t v_ts, int64_t v_hs, bf16* vt, int64_t vt_hs, int64_t vt_ds,
                                   const SeqTable& seqs, int n_tiles, int H, hipStream_t s) {
  return launch(v_transpose_bf16_kernel, dim3(n_tiles, H), dim3(256), 0, s, v, v_ts, v_hs, vt, vt_hs, vt_ds, seqs);
}

hipError_t launch_quant_fp8(const bf16* x, int64_t x_ts, int64_t x_hs, float pre, uint8_t* codes, int64_t c_hs,
                            int64_t c_ds, bool transposed, int64_t out_row0, float* scales, int64_t sc_hs,
                            const SeqTable& seqs, int n_blocks, int H, hipStream_t s) {
  return launch(quant_fp8_kernel, dim3(n_blocks, H), dim3(256), 0, s, x, x_ts, x_hs, pre, codes, c_hs, c_ds,
                transposed ? 1 : 0, out_row0, scales, sc_hs, seqs);
}

hipError_t launch_scale_max(const float* sk, const float* sv, int64_t sc_hs, int n_blocks, float* vmax, int* kinfo,
                            int H, hipStream_t s) {
  return launch(scale_max_kernel, dim3(H), dim3(64), 0, s, sk, sv, sc_hs, n_blocks, vmax, kinfo);
}

}  // namespace vggtx
