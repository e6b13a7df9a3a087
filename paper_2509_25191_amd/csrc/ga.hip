// Camera global alignment (arXiv 2509.25191, Sec. 3.3, Eqs. epi / weight / lr):
// refine every camera (rotation, translation, focal length) by Adam on the
// weighted mean epipolar distance of the pairwise correspondences, with the
// weights taken from a histogram of the initial residuals and the learning
// rate from their median.  All arithmetic is float64: the work is bound by
// streaming the correspondences (16 + 1 bytes each per iteration), and the
// vector units run float64 at half the float32 rate.
//
// Per camera n the parameters are p[n] = (q0..q3, t0..t2, phi): R = R(q/|q|),
// t, f = f0 exp(phi).  A pair (i, j) has R_ij = R_j R_i^T, t_ij = t_j - R_ij t_i
// and F = K_j^-T [t_ij]_x R_ij K_i^-1; a correspondence (x, x') has the
// residual e = |x'^T F x| / |(F x)_{0,1}|, the pixel distance of x' from the
// epipolar line of x.
//
// Kernels (one wave per pair streams that pair's correspondences):
//   ga_init_kernel   parameters from the initial cameras, Adam state zeroed
//   ga_pair_kernel   MODE_BINS: residual histogram bin of every correspondence
//                    (initial cameras) and the global bin counts;
//                    MODE_GRAD: per pair sum_k w_k e_k and its gradient with
//                    respect to F; MODE_LOSS: sum_k w_k e_k only
//   ga_chain_kernel  per pair: gradient w.r.t. the 16 parameters of the two cameras
//   ga_table_kernel  weight per bin, total weight, learning rate (median bin)
//   ga_adam_kernel   per camera: sum of its pairs' gradients / W, Adam step
//   ga_loss_kernel   sum of the pair losses / W into the loss history
//   ga_out_kernel    R, t, f of the parameters; optional per-correspondence weights
#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace vggtx {

namespace {

struct M3 {
  double a[3][3];
};

__device__ __forceinline__ M3 mul(const M3& x, const M3& y) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.a[i][j] = x.a[i][0] * y.a[0][j] + x.a[i][1] * y.a[1][j] + x.a[i][2] * y.a[2][j];
  return r;
}
__device__ __forceinline__ M3 tr(const M3& x) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.a[i][j] = x.a[j][i];
  return r;
}
__device__ __forceinline__ M3 skew3(const double t[3]) {
  M3 r = {{{0.0, -t[2], t[1]}, {t[2], 0.0, -t[0]}, {-t[1], t[0], 0.0}}};
  return r;
}
// K^-1 for focal f and principal point (cx, cy)
__device__ __forceinline__ M3 kinv(double f, double cx, double cy) {
  M3 r = {{{1.0 / f, 0.0, -cx / f}, {0.0, 1.0 / f, -cy / f}, {0.0, 0.0, 1.0}}};
  return r;
}
// numerator matrix N(q) with R(q / |q|) = N(q) / |q|^2
__device__ __forceinline__ M3 quat_num(const double q[4]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  M3 r = {{{w * w + x * x - y * y - z * z, 2 * (x * y - w * z), 2 * (x * z + w * y)},
           {2 * (x * y + w * z), w * w - x * x + y * y - z * z, 2 * (y * z - w * x)},
           {2 * (x * z - w * y), 2 * (y * z + w * x), w * w - x * x - y * y + z * z}}};
  return r;
}
__device__ __forceinline__ M3 quat_rot(const double q[4]) {
  M3 r = quat_num(q);
  const double inv = 1.0 / (q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.a[i][j] *= inv;
  return r;
}

// Camera of the pair side: R, t, f, principal point.
struct Cam {
  M3 R;
  double t[3], f, cx, cy;
};
__device__ __forceinline__ Cam load_cam(const double* p, const double* f0, const double* pp, int n) {
  Cam c;
  const double* q = p + 8 * n;
  c.R = quat_rot(q);
  c.t[0] = q[4]; c.t[1] = q[5]; c.t[2] = q[6];
  c.f = f0[n] * exp(q[7]);
  c.cx = pp[2 * n]; c.cy = pp[2 * n + 1];
  return c;
}

// Fundamental matrix of the pair and the intermediates of its chain rule.
struct PairGeom {
  M3 Rij, E, Ki, Kj, F;
  double tij[3];
};
__device__ __forceinline__ PairGeom pair_geom(const Cam& ci, const Cam& cj) {
  PairGeom g;
  g.Rij = mul(cj.R, tr(ci.R));
#pragma unroll
  for (int r = 0; r < 3; ++r)
    g.tij[r] = cj.t[r] - (g.Rij.a[r][0] * ci.t[0] + g.Rij.a[r][1] * ci.t[1] + g.Rij.a[r][2] * ci.t[2]);
  g.E = mul(skew3(g.tij), g.Rij);
  g.Ki = kinv(ci.f, ci.cx, ci.cy);
  g.Kj = kinv(cj.f, cj.cx, cj.cy);
  g.F = mul(mul(tr(g.Kj), g.E), g.Ki);
  return g;
}

// Residual of one correspondence; with GRAD also de/dF = g x^T (g returned).
__device__ __forceinline__ double residual(const M3& F, const f32x4 c, double g[3], bool grad) {
  const double x[3] = {(double)c[0], (double)c[1], 1.0};
  const double xp[3] = {(double)c[2], (double)c[3], 1.0};
  double l[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) l[r] = F.a[r][0] * x[0] + F.a[r][1] * x[1] + F.a[r][2];
  const double s = xp[0] * l[0] + xp[1] * l[1] + l[2];
  // 1/sqrt(n2): hardware estimate refined by two Newton steps
  // (y <- y (3 - n2 y^2) / 2, each step doubling the correct bits)
  const double n2 = l[0] * l[0] + l[1] * l[1];
  double rn = __builtin_amdgcn_rsq(n2);
  rn = rn * __builtin_fma(-0.5 * n2 * rn, rn, 1.5);
  rn = rn * __builtin_fma(-0.5 * n2 * rn, rn, 1.5);
  const double e = fabs(s) * rn;
  if (grad) {
    const double sg = s > 0.0 ? rn : (s < 0.0 ? -rn : 0.0);
    const double er2 = e * rn * rn;
    g[0] = sg * xp[0] - er2 * l[0];
    g[1] = sg * xp[1] - er2 * l[1];
    g[2] = sg;
  }
  return e;
}

__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  return s;
}

}  // namespace

__global__ __launch_bounds__(256) void ga_init_kernel(const double* R0, const double* t0, int n_cams, double* p,
                                                      double* adam) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= n_cams) return;
  const double* m = R0 + 9 * n;
  // quaternion (w >= 0) from the largest of the four diagonal combinations
  const double tr0 = m[0] + m[4] + m[8];
  const double cand[4] = {tr0, m[0] - m[4] - m[8], m[4] - m[0] - m[8], m[8] - m[0] - m[4]};
  int k = 0;
  for (int i = 1; i < 4; ++i)
    if (cand[i] > cand[k]) k = i;
  const double s = sqrt(fmax(cand[k] + 1.0, 0.0)) * 2.0;
  double q[4];
  if (k == 0) {
    q[0] = s / 4; q[1] = (m[7] - m[5]) / s; q[2] = (m[2] - m[6]) / s; q[3] = (m[3] - m[1]) / s;
  } else if (k == 1) {
    q[0] = (m[7] - m[5]) / s; q[1] = s / 4; q[2] = (m[1] + m[3]) / s; q[3] = (m[2] + m[6]) / s;
  } else if (k == 2) {
    q[0] = (m[2] - m[6]) / s; q[1] = (m[1] + m[3]) / s; q[2] = s / 4; q[3] = (m[5] + m[7]) / s;
  } else {
    q[0] = (m[3] - m[1]) / s; q[1] = (m[2] + m[6]) / s; q[2] = (m[5] + m[7]) / s; q[3] = s / 4;
  }
  const double sg = q[0] >= 0.0 ? 1.0 : -1.0;
  double* o = p + 8 * n;
  for (int i = 0; i < 4; ++i) o[i] = sg * q[i];
  for (int i = 0; i < 3; ++i) o[4 + i] = t0[3 * n + i];
  o[7] = 0.0;
  for (int i = 0; i < 16; ++i) adam[16 * n + i] = 0.0;
}

// One wave per pair (four pairs per workgroup): the lanes stride over the
// pair's correspondences, then a fixed butterfly sums the wave's partial sums,
// so no workgroup barrier is needed outside the histogram pass.
template <int MODE>
__global__ __launch_bounds__(256) void ga_pair_kernel(GaParams a, int n_pairs) {
  __shared__ uint32_t hist[kGaBins + 1];
  const int lane = threadIdx.x & 63;
  const int m = blockIdx.x * 4 + (threadIdx.x >> 6);
  const bool live = m < n_pairs;
  const f32x4* corr = (const f32x4*)a.corr;
  if (MODE == GA_MODE_BINS) {
    for (int b = threadIdx.x; b <= kGaBins; b += 256) hist[b] = 0u;
    __syncthreads();
    if (live) {
      const Cam ci = load_cam(a.p, a.f0, a.pp, a.pairs[2 * m]);
      const Cam cj = load_cam(a.p, a.f0, a.pp, a.pairs[2 * m + 1]);
      const M3 F = pair_geom(ci, cj).F;
      for (int64_t k = a.offsets[m] + lane; k < a.offsets[m + 1]; k += 64) {
        double g[3];
        const double e = residual(F, corr[k], g, false);
        const int b = e < (double)kGaBins / kGaBinsPerPixel ? (int)floor(e * kGaBinsPerPixel) : kGaBins;
        a.bins[k] = (uint8_t)b;
        atomicAdd(&hist[b], 1u);
      }
    }
    __syncthreads();
    for (int b = threadIdx.x; b <= kGaBins; b += 256)
      if (hist[b]) atomicAdd(&a.hist[b], hist[b]);
    return;
  }
  if (!live) return;
  M3 F;
  {
    const Cam ci = load_cam(a.p, a.f0, a.pp, a.pairs[2 * m]);
    const Cam cj = load_cam(a.p, a.f0, a.pp, a.pairs[2 * m + 1]);
    F = pair_geom(ci, cj).F;
  }
  // weighted residual sum and, for MODE_GRAD, sum_k w_k (de_k/dF)
  double acc[10] = {};
  for (int64_t k = a.offsets[m] + lane; k < a.offsets[m + 1]; k += 64) {
    const double w = a.table[a.bins[k]];
    const f32x4 c = corr[k];
    double g[3];
    const double e = residual(F, c, g, MODE == GA_MODE_GRAD);
    acc[9] += w * e;
    if (MODE == GA_MODE_GRAD) {
      const double x0 = (double)c[0], x1 = (double)c[1];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const double wg = w * g[r];
        acc[3 * r] += wg * x0;
        acc[3 * r + 1] += wg * x1;
        acc[3 * r + 2] += wg;
      }
    }
  }
  constexpr int NR = MODE == GA_MODE_GRAD ? 10 : 1;
  const int r0 = MODE == GA_MODE_GRAD ? 0 : 9;
#pragma unroll
  for (int r = r0; r < r0 + NR; ++r)
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc[r] += __shfl_xor(acc[r], o);
  if (lane != 0) return;
  a.pair_loss[m] = acc[9];
  if (MODE == GA_MODE_GRAD) {
    double* gf = a.pair_gf + 9 * (int64_t)m;
#pragma unroll
    for (int r = 0; r < 9; ++r) gf[r] = acc[r];
  }
}

// One thread per pair: chain rule from dL/dF to the 16 parameters of the two
// cameras.  F = Kj^-T E Ki^-1, E = [t_ij]_x R_ij, R_ij = R_j R_i^T,
// t_ij = t_j - R_ij t_i, R = N(q) / |q|^2, f = f0 exp(phi).
__global__ __launch_bounds__(256) void ga_chain_kernel(GaParams a, int n_pairs) {
  const int m = blockIdx.x * 256 + threadIdx.x;
  if (m >= n_pairs) return;
  const int i = a.pairs[2 * m], j = a.pairs[2 * m + 1];
  const Cam ci = load_cam(a.p, a.f0, a.pp, i);
  const Cam cj = load_cam(a.p, a.f0, a.pp, j);
  const PairGeom pg = pair_geom(ci, cj);
  M3 GF;
  const double* gf = a.pair_gf + 9 * (int64_t)m;
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) GF.a[r][c] = gf[3 * r + c];
  const M3 GE = mul(mul(pg.Kj, GF), tr(pg.Ki));
  const M3 GKi = mul(tr(mul(tr(pg.Kj), pg.E)), GF);
  const M3 GKjT = mul(GF, tr(mul(pg.E, pg.Ki)));
  const double fi2 = ci.f * ci.f, fj2 = cj.f * cj.f;
  // d(Ki^-1)/df_i and d(Kj^-T)/df_j contracted with the gradients, times df/dphi = f
  const double gphi_i = (-(GKi.a[0][0] + GKi.a[1][1]) / fi2 + (GKi.a[0][2] * ci.cx + GKi.a[1][2] * ci.cy) / fi2) * ci.f;
  const double gphi_j =
      (-(GKjT.a[0][0] + GKjT.a[1][1]) / fj2 + (GKjT.a[2][0] * cj.cx + GKjT.a[2][1] * cj.cy) / fj2) * cj.f;
  const M3 Mt = mul(GE, tr(pg.Rij));
  const double gt[3] = {Mt.a[2][1] - Mt.a[1][2], Mt.a[0][2] - Mt.a[2][0], Mt.a[1][0] - Mt.a[0][1]};
  M3 GR = mul(tr(skew3(pg.tij)), GE);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) GR.a[r][c] -= gt[r] * ci.t[c];
  const M3 gRj = mul(GR, ci.R);
  const M3 gRi = mul(tr(GR), cj.R);
  double* out = a.pair_grad + 16 * (int64_t)m;
  // dR/dq for each camera, contracted with its rotation gradient
  for (int side = 0; side < 2; ++side) {
    const double* q = (side == 0 ? a.p + 8 * i : a.p + 8 * j);
    const M3& gRs = side == 0 ? gRi : gRj;
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    const double n2 = w * w + x * x + y * y + z * z;
    const M3 N = quat_num(q);
    const M3 dN[4] = {
        {{{2 * w, -2 * z, 2 * y}, {2 * z, 2 * w, -2 * x}, {-2 * y, 2 * x, 2 * w}}},
        {{{2 * x, 2 * y, 2 * z}, {2 * y, -2 * x, -2 * w}, {2 * z, 2 * w, -2 * x}}},
        {{{-2 * y, 2 * x, 2 * w}, {2 * x, 2 * y, 2 * z}, {-2 * w, 2 * z, -2 * y}}},
        {{{-2 * z, -2 * w, 2 * x}, {2 * w, -2 * z, 2 * y}, {2 * x, 2 * y, 2 * z}}},
    };
    for (int qa = 0; qa < 4; ++qa) {
      double s = 0.0;
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) s += (dN[qa].a[r][c] * n2 - N.a[r][c] * 2.0 * q[qa]) * gRs.a[r][c];
      out[8 * side + qa] = s / (n2 * n2);
    }
  }
  // translations: dL/dt_j = gt, dL/dt_i = -R_ij^T gt
  for (int r = 0; r < 3; ++r) {
    out[8 + 4 + r] = gt[r];
    out[4 + r] = -(pg.Rij.a[0][r] * gt[0] + pg.Rij.a[1][r] * gt[1] + pg.Rij.a[2][r] * gt[2]);
  }
  out[7] = gphi_i;
  out[15] = gphi_j;
}

// One workgroup: weight table, total weight and learning rate from the bin counts.
__global__ __launch_bounds__(256) void ga_table_kernel(const uint32_t* hist, double alpha, int lr_bin1, int lr_bin2,
                                                       double lr0, double lr1, double lr2, double* table,
                                                       double* scal) {
  __shared__ double red[4];
  __shared__ double dens[kGaBins + 1];
  __shared__ uint64_t cum[kGaBins + 1];
  double K = 0.0;
  for (int b = 0; b <= kGaBins; ++b) K += (double)hist[b];  // every thread, same order
  const double h = 1.0 / kGaBinsPerPixel;
  for (int b = threadIdx.x; b <= kGaBins; b += 256) dens[b] = b < kGaBins && K > 0.0 ? (double)hist[b] / (K * h) : 0.0;
  __syncthreads();
  double part = 0.0;
  for (int b = threadIdx.x; b <= kGaBins; b += 256) part += (double)hist[b] * dens[b];
  const double avg = block_sum(part, red) / (K > 0.0 ? K : 1.0);
  for (int b = threadIdx.x; b <= kGaBins; b += 256) table[b] = avg > 0.0 ? pow(dens[b] / avg, alpha) : 1.0;
  __syncthreads();
  double wp = 0.0;
  for (int b = threadIdx.x; b <= kGaBins; b += 256) wp += (double)hist[b] * table[b];
  const double W = block_sum(wp, red);
  if (threadIdx.x == 0) {
    uint64_t c = 0;
    for (int b = 0; b <= kGaBins; ++b) {
      c += hist[b];
      cum[b] = c;
    }
    const uint64_t rank = (c + 1) / 2;
    int mb = 0;
    while (mb < kGaBins && cum[mb] < rank) ++mb;
    scal[0] = mb < lr_bin1 ? lr0 : (mb < lr_bin2 ? lr1 : lr2);
    scal[1] = W;
    scal[2] = (double)mb;
  }
}

// One wave per camera: its pair sides are summed lane-strided (fixed order per
// lane, then a fixed butterfly), scaled by 1/W, then one Adam step.
__global__ __launch_bounds__(256) void ga_adam_kernel(GaParams a, int n_cams, int step, double beta1, double beta2,
                                                      double eps) {
  const int n = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (n >= n_cams) return;
  double g[8] = {};
  for (int e = a.inc_off[n] + lane; e < a.inc_off[n + 1]; e += 64) {
    const int side = a.inc[e] & 1;
    const double* src = a.pair_grad + 16 * (int64_t)(a.inc[e] >> 1) + 8 * side;
#pragma unroll
    for (int r = 0; r < 8; ++r) g[r] += src[r];
  }
#pragma unroll
  for (int r = 0; r < 8; ++r)
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) g[r] += __shfl_xor(g[r], o);
  if (lane >= 8) return;
  const double W = a.scal[1], lr = a.scal[0];
  const double invW = W > 0.0 ? 1.0 / W : 0.0;
  const double c1 = 1.0 - pow(beta1, (double)step), c2 = 1.0 - pow(beta2, (double)step);
  double gr = 0.0;
#pragma unroll
  for (int r = 0; r < 8; ++r)
    if (lane == r) gr = g[r] * invW;
  double* p = a.p + 8 * n;
  double* mo = a.adam + 16 * n;
  mo[lane] = beta1 * mo[lane] + (1.0 - beta1) * gr;
  mo[8 + lane] = beta2 * mo[8 + lane] + (1.0 - beta2) * gr * gr;
  p[lane] -= lr * (mo[lane] / c1) / (sqrt(mo[8 + lane] / c2) + eps);
}

// One workgroup: loss = sum of the pair sums / W (fixed order per thread, then a tree).
__global__ __launch_bounds__(1024) void ga_loss_kernel(const double* pair_loss, int n_pairs, const double* scal,
                                                       double* out) {
  __shared__ double red[16];
  double s = 0.0;
  for (int m = threadIdx.x; m < n_pairs; m += 1024) s += pair_loss[m];
  const double t = block_sum(s, red);
  if (threadIdx.x == 0) *out = scal[1] > 0.0 ? t / scal[1] : 0.0;
}

__global__ __launch_bounds__(256) void ga_out_kernel(const double* p, const double* f0, int n_cams, double* R_out,
                                                     double* t_out, double* f_out) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= n_cams) return;
  const double* q = p + 8 * n;
  const M3 R = quat_rot(q);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) R_out[9 * n + 3 * r + c] = R.a[r][c];
  for (int r = 0; r < 3; ++r) t_out[3 * n + r] = q[4 + r];
  f_out[n] = f0[n] * exp(q[7]);
}

__global__ __launch_bounds__(256) void ga_weights_kernel(const uint8_t* bins, const double* table, int64_t n,
                                                         float* w) {
  for (int64_t k = blockIdx.x * 256ll + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256) w[k] = (float)table[bins[k]];
}

__global__ __launch_bounds__(256) void ga_zero_u32_kernel(uint32_t* x, int n) {
  for (int k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) x[k] = 0u;
}

// ------------------------------------------------------------------ AUC@30
// One thread per ordered pair (i, j), i != j (both_orders) or i < j: relative
// poses E_i^-1 E_j = (R_i^T R_j, R_i^T (t_j - t_i)) of the prediction and the
// ground truth, error = max(rotation angle of dR_pred^T dR_gt, angle between
// dt_pred and dt_gt) in degrees, counted in bins [b, b+1) for b < 30 and one
// bin for 30 or more (integer counts, so the result is exact and order-free).
__global__ __launch_bounds__(256) void auc30_kernel(const double* Rp, const double* tp, const double* Rg,
                                                    const double* tg, int n, int both_orders, uint32_t* counts) {
  __shared__ uint32_t hist[kAucBins];
  for (int b = threadIdx.x; b < kAucBins; b += 256) hist[b] = 0u;
  __syncthreads();
  const int64_t idx = blockIdx.x * 256ll + threadIdx.x;
  const int64_t nn = (int64_t)n * n;
  if (idx < nn) {
    const int i = (int)(idx / n), j = (int)(idx - (int64_t)i * n);
    if (i != j && (both_orders || i < j)) {
      double err[2];
      double dR[2][3][3], dt[2][3];
      for (int s = 0; s < 2; ++s) {
        const double* R = s == 0 ? Rp : Rg;
        const double* t = s == 0 ? tp : tg;
        const double* Ri = R + 9 * (int64_t)i;
        const double* Rj = R + 9 * (int64_t)j;
        for (int r = 0; r < 3; ++r) {
          for (int c = 0; c < 3; ++c) dR[s][r][c] = Ri[r] * Rj[c] + Ri[3 + r] * Rj[3 + c] + Ri[6 + r] * Rj[6 + c];
          dt[s][r] = Ri[r] * (t[3 * j] - t[3 * i]) + Ri[3 + r] * (t[3 * j + 1] - t[3 * i + 1]) +
                     Ri[6 + r] * (t[3 * j + 2] - t[3 * i + 2]);
        }
      }
      // trace(dR_pred^T dR_gt) = sum of the elementwise products
      double tr = 0.0;
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) tr += dR[0][r][c] * dR[1][r][c];
      const double kDeg = 57.295779513082320876798;  // 180 / pi
      err[0] = acos(fmin(1.0, fmax(-1.0, (tr - 1.0) / 2.0))) * kDeg;
      const double na = sqrt(dt[0][0] * dt[0][0] + dt[0][1] * dt[0][1] + dt[0][2] * dt[0][2]);
      const double nb = sqrt(dt[1][0] * dt[1][0] + dt[1][1] * dt[1][1] + dt[1][2] * dt[1][2]);
      err[1] = 0.0;
      if (na > 0.0 && nb > 0.0) {
        const double c = (dt[0][0] * dt[1][0] + dt[0][1] * dt[1][1] + dt[0][2] * dt[1][2]) / (na * nb);
        err[1] = acos(fmin(1.0, fmax(-1.0, c))) * kDeg;
      }
      const double e = fmax(err[0], err[1]);
      const int b = e < (double)(kAucBins - 1) ? (int)floor(e) : kAucBins - 1;
      atomicAdd(&hist[b], 1u);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kAucBins; b += 256)
    if (hist[b]) atomicAdd(&counts[b], hist[b]);
}

// AUC@30 = mean over tau = 1..30 of the fraction of errors below tau.
__global__ void auc30_finish_kernel(const uint32_t* counts, double* auc) {
  if (threadIdx.x != 0) return;
  double total = 0.0;
  for (int b = 0; b < kAucBins; ++b) total += (double)counts[b];
  double below = 0.0, s = 0.0;
  for (int tau = 1; tau < kAucBins; ++tau) {
    below += (double)counts[tau - 1];
    s += total > 0.0 ? below / total : 0.0;
  }
  *auc = s / (kAucBins - 1);
}

// ------------------------------------------------------------------ launchers
hipError_t launch_auc30(const double* Rp, const double* tp, const double* Rg, const double* tg, int n, int both_orders,
                        uint32_t* counts, double* auc, hipStream_t s) {
  hipLaunchKernelGGL(ga_zero_u32_kernel, dim3(1), dim3(256), 0, s, counts, kAucBins);
  const int64_t nn = (int64_t)n * n;
  if (nn > 0)
    hipLaunchKernelGGL(auc30_kernel, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, Rp, tp, Rg, tg, n,
                       both_orders, counts);
  if (auc) hipLaunchKernelGGL(auc30_finish_kernel, dim3(1), dim3(64), 0, s, counts, auc);
  return hipGetLastError();
}
static unsigned cdiv_u(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

hipError_t launch_ga_init(const double* R0, const double* t0, int n_cams, double* p, double* adam, hipStream_t s) {
  hipLaunchKernelGGL(ga_init_kernel, dim3(cdiv_u(n_cams, 256)), dim3(256), 0, s, R0, t0, n_cams, p, adam);
  return hipGetLastError();
}

hipError_t launch_ga_pairs(const GaParams& a, int n_pairs, int mode, hipStream_t s) {
  if (n_pairs <= 0) return hipSuccess;
  const dim3 grid(cdiv_u(n_pairs, 4));
  switch (mode) {
    case GA_MODE_BINS: hipLaunchKernelGGL(ga_pair_kernel<GA_MODE_BINS>, grid, dim3(256), 0, s, a, n_pairs); break;
    case GA_MODE_GRAD: hipLaunchKernelGGL(ga_pair_kernel<GA_MODE_GRAD>, grid, dim3(256), 0, s, a, n_pairs); break;
    default: hipLaunchKernelGGL(ga_pair_kernel<GA_MODE_LOSS>, grid, dim3(256), 0, s, a, n_pairs); break;
  }
  return hipGetLastError();
}

hipError_t launch_ga_table(const uint32_t* hist, double alpha, int lr_bin1, int lr_bin2, double lr0, double lr1,
                           double lr2, double* table, double* scal, hipStream_t s) {
  hipLaunchKernelGGL(ga_table_kernel, dim3(1), dim3(256), 0, s, hist, alpha, lr_bin1, lr_bin2, lr0, lr1, lr2, table,
                     scal);
  return hipGetLastError();
}

hipError_t launch_ga_adam(const GaParams& a, int n_cams, int step, double beta1, double beta2, double eps,
                          hipStream_t s) {
  hipLaunchKernelGGL(ga_adam_kernel, dim3(cdiv_u(n_cams, 4)), dim3(256), 0, s, a, n_cams, step, beta1, beta2, eps);
  return hipGetLastError();
}

hipError_t launch_ga_chain(const GaParams& a, int n_pairs, hipStream_t s) {
  if (n_pairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(ga_chain_kernel, dim3(cdiv_u(n_pairs, 256)), dim3(256), 0, s, a, n_pairs);
  return hipGetLastError();
}

hipError_t launch_ga_loss(const double* pair_loss, int n_pairs, const double* scal, double* out, hipStream_t s) {
  hipLaunchKernelGGL(ga_loss_kernel, dim3(1), dim3(1024), 0, s, pair_loss, n_pairs, scal, out);
  return hipGetLastError();
}

hipError_t launch_ga_out(const double* p, const double* f0, int n_cams, double* R_out, double* t_out, double* f_out,
                         hipStream_t s) {
  hipLaunchKernelGGL(ga_out_kernel, dim3(cdiv_u(n_cams, 256)), dim3(256), 0, s, p, f0, n_cams, R_out, t_out, f_out);
  return hipGetLastError();
}

hipError_t launch_ga_weights(const uint8_t* bins, const double* table, int64_t n, float* w, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>(cdiv_u(n, 256), 65536);
  hipLaunchKernelGGL(ga_weights_kernel, dim3(grid), dim3(256), 0, s, bins, table, n, w);
  return hipGetLastError();
}

hipError_t launch_ga_zero_u32(uint32_t* x, int n, hipStream_t s) {
  hipLaunchKernelGGL(ga_zero_u32_kernel, dim3(cdiv_u(n, 256)), dim3(256), 0, s, x, n);
  return hipGetLastError();
}

}  // namespace vggtx
