// Hand-written adjoint kernels of the Radar-STDA network (gfx950), NHWC, FP32 or BF16 storage.
#pragma once
#include <type_traits>

#include "net_kernels.h"

namespace stda {

// --------------------------------------------------------------------- ECA adjoint
// gap-like partials of sum_hw G * Y per (clip, tile, channel).
template <class T, int C>
struct k_eca_bwd_part_args {
  const T* Gd;
  const T* Y;
  float* part;
  int hw;
  int tiles;
};
template <class T, int C>
__global__ __launch_bounds__(256) void k_eca_bwd_part(SegL<k_eca_bwd_part_args<T, C>> L) {
  const SegB sb = seg_block(L);
  if (sb.x >= sb.gx) return;
  const int bx = sb.x, gx = sb.gx;  // workgroup index and count within the segment
  (void)gx;
  const k_eca_bwd_part_args<T, C>& a_ = L.a[sb.s];
  const T* __restrict__ const Gd = a_.Gd;
  const T* __restrict__ const Y = a_.Y;
  float* __restrict__ const part = a_.part;
  const int hw = a_.hw;
  const int tiles = a_.tiles;
  constexpr int G = C / 4;
  __shared__ float sm[4 * STDA_BLOCK];
  __shared__ float red[C];
  const int b = bx / tiles, tx = bx - b * tiles;  // clip, tile of the clip
  const int64_t items = (int64_t)hw * G, base = (int64_t)b * hw * C;
  int64_t i = (int64_t)tx * STDA_BLOCK + threadIdx.x;
  const int c0 = (int)(i % G) * 4;
  float acc[1][4];
  zero4(acc[0]);
  for (; i < items; i += (int64_t)tiles * STDA_BLOCK) {
    const int64_t off = base + (i / G) * C + c0;
    float g[4], y[4];
    ld4(Gd + off, g);
    ld4(Y + off, y);
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[0][j] += g[j] * y[j];
  }
  block_chan_reduce<G, 1>(acc, sm, red);
  for (int q = threadIdx.x; q < C; q += STDA_BLOCK) part[((int64_t)b * tiles + tx) * C + q] = red[q];
}

// ECA adjoint of one clip: da = sum_hw G Y; ds = da a (1 - a); dg[c] = w0 ds[c+1] + w1 ds[c]
// + w2 ds[c-1]; e = dg / hw (added to every pixel of the channel).  Also the clip's
// contribution to the three ECA weight gradients.
template <int C>
__device__ __forceinline__ void eca_adjoint_clip(const float* __restrict__ part, int tiles, int hw,
                                                 const float* __restrict__ a, const float* __restrict__ g,
                                                 const float* __restrict__ weca, float* ds_s, float* e_s,
                                                 float* dw3 /* nullable */) {
  for (int c = threadIdx.x; c < C; c += STDA_BLOCK) {
    double s = 0.0;
    for (int t = 0; t < tiles; ++t) s += (double)part[t * C + c];
    const float da = (float)s;
    ds_s[c] = da * a[c] * (1.f - a[c]);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += STDA_BLOCK) {
    const float dsp = c < C - 1 ? ds_s[c + 1] : 0.f, dsm = c > 0 ? ds_s[c - 1] : 0.f;
    e_s[c] = (weca[0] * dsp + weca[1] * ds_s[c] + weca[2] * dsm) / (float)hw;
  }
  if (dw3 && threadIdx.x < 3) {
    const int k = threadIdx.x;  // s[c] uses g[c - 1 + k] with weight k
    double s = 0.0;
    for (int c = 0; c < C; ++c) {
      const int cc = c - 1 + k;
      if (cc >= 0 && cc < C) s += (double)ds_s[c] * (double)g[cc];
    }
    dw3[k] = (float)s;
  }
  __syncthreads();
}

// Stage-2 adjoint, statistics pass.  dY = a G + e; BN output recomputed from T to get the
// ReLU mask; dM = mask * dY.  Partials part[blk][2][C]: sum dM, sum dM * that.  Tile 0 of
// each clip writes e (coef_e[clip][C]) and the ECA weight partial (ecaw[clip][3]).
template <class T, int C>
struct k_s2_bwd_stats_args {
  const T* Gd;
  const T* Tm;
  const uint8_t* mask;
  const float* epart;
  const float* a_sv;
  const float* g_sv;
  const float* weca;
  const float* stats;
  const float* gamma;
  const float* beta;
  float* coef_e;
  float* ecaw;
  float* part;
  int hw;
  int etiles;
  int tiles;
};
template <class T, int C>
__global__ __launch_bounds__(256) void k_s2_bwd_stats(SegL<k_s2_bwd_stats_args<T, C>> L) {
  const SegB sb = seg_block(L);
  if (sb.x >= sb.gx) return;
  const int bx = sb.x, gx = sb.gx;  // workgroup index and count within the segment
  (void)gx;
  const k_s2_bwd_stats_args<T, C>& a_ = L.a[sb.s];
  const T* __restrict__ const Gd = a_.Gd;
  const T* __restrict__ const Tm = a_.Tm;
  const uint8_t* __restrict__ const mask = a_.mask;
  const float* __restrict__ const epart = a_.epart;
  const float* __restrict__ const a_sv = a_.a_sv;
  const float* __restrict__ const g_sv = a_.g_sv;
  const float* __restrict__ const weca = a_.weca;
  const float* __restrict__ const stats = a_.stats;
  const float* __restrict__ const gamma = a_.gamma;
  const float* __restrict__ const beta = a_.beta;
  float* __restrict__ const coef_e = a_.coef_e;
  float* __restrict__ const ecaw = a_.ecaw;
  float* __restrict__ const part = a_.part;
  const int hw = a_.hw;
  const int etiles = a_.etiles;
  const int tiles = a_.tiles;
  constexpr int G = C / 4;
  __shared__ float ds_s[C], e_s[C];
  __shared__ float sm[2 * 4 * STDA_BLOCK];
  __shared__ float red[2 * C];
  const int b = bx / tiles, tx = bx - b * tiles;  // clip, tile of the clip
  eca_adjoint_clip<C>(epart + (int64_t)b * etiles * C, etiles, hw, a_sv + b * C, g_sv + b * C, weca, ds_s, e_s,
                      tx == 0 ? ecaw + b * 3 : nullptr);
  if (tx == 0)
    for (int c = threadIdx.x; c < C; c += STDA_BLOCK) coef_e[b * C + c] = e_s[c];
  const int64_t items = (int64_t)hw * G, base = (int64_t)b * hw * C;
  int64_t i = (int64_t)tx * STDA_BLOCK + threadIdx.x;
  const int c0 = (int)(i % G) * 4;
  float a4v[4], e4[4], mu[4], is[4], ga[4], be[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    a4v[j] = a_sv[b * C + c0 + j];
    e4[j] = e_s[c0 + j];
    mu[j] = stats[c0 + j];
    is[j] = stats[C + c0 + j];
    ga[j] = gamma[c0 + j];
    be[j] = beta[c0 + j];
  }
  float acc[2][4];
  zero4(acc[0]);
  zero4(acc[1]);
  for (; i < items; i += (int64_t)tiles * STDA_BLOCK) {
    const int64_t off = base + (i / G) * C + c0;
    float g[4], t[4];
    ld4(Gd + off, g);
    ld4(Tm + off, t);
    const unsigned bits = mask[off >> 2];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float th = (t[j] - mu[j]) * is[j];
      const float dm = ((bits >> j) & 1u) ? a4v[j] * g[j] + e4[j] : 0.f;
      acc[0][j] += dm;
      acc[1][j] += dm * th;
    }
  }
  block_chan_reduce<G, 2>(acc, sm, red);
  const int64_t blk = (int64_t)b * tiles + tx;
  for (int q = threadIdx.x; q < 2 * C; q += STDA_BLOCK) part[blk * 2 * C + q] = red[q];
}

// BN adjoint coefficients from column sums sums[s][C]: beta gradient = sums[0], gamma
// gradient of layer k = sums[1 + k]; coef[s][C] = sums[s] / n.
struct BnBwdOut {
  float* dgamma[3];
  float* dbeta[3];
};
struct BnBwdSegs {
  int n;                        // segments
  const float* part[kMaxSegs];  // the segment's partials part[blk][NS][C]
  int rows[kMaxSegs];           // its partial rows
  double count[kMaxSegs];       // elements per channel the segment's BN layers normalise
  float* coef[kMaxSegs];        // its coefficients coef[NS][C]
};
// Cross-block FP64 reduction of BN adjoint partials fused with the finalize: per segment the
// column sums give that segment's coefficients (its layers have their own statistics); the
// gamma and beta gradients are the sums over all segments, taken in FP64 and rounded once.
// Block = one (sum q, channel c) column, blockIdx.x = q C + c; its 256 threads take every 256th
// row, added in a fixed tree order.  Column q = 0 (the beta gradient, shared by the NS - 1 layers)
// writes dbeta, q >= 1 writes dgamma[q - 1].
__global__ __launch_bounds__(256) void k_bn_bwd_reduce(BnBwdSegs sg, int NS, int C, BnBwdOut out, int accumulate) {
  __shared__ double sm[STDA_BLOCK];
  const int q = blockIdx.x / C, c = blockIdx.x % C;
  double tot = 0.0;
  for (int sgi = 0; sgi < sg.n; ++sgi) {
    const float* __restrict__ part = sg.part[sgi];
    double a = 0.0;
#pragma unroll 4
    for (int r = threadIdx.x; r < sg.rows[sgi]; r += STDA_BLOCK) a += (double)part[(int64_t)r * NS * C + q * C + c];
    sm[threadIdx.x] = a;
    __syncthreads();
#pragma unroll
    for (int half = STDA_BLOCK / 2; half > 0; half >>= 1) {
      if ((int)threadIdx.x < half) sm[threadIdx.x] += sm[threadIdx.x + half];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      tot += sm[0];
      sg.coef[sgi][q * C + c] = (float)(sm[0] / sg.count[sgi]);
    }
    __syncthreads();  // sm is reused by the next segment
  }
  if (threadIdx.x == 0) {
    if (q == 0) {
      for (int k = 0; k < NS - 1; ++k) out.dbeta[k][c] = accumulate ? (float)((double)out.dbeta[k][c] + tot) : (float)tot;
    } else {
      out.dgamma[q - 1][c] = accumulate ? (float)((double)out.dgamma[q - 1][c] + tot) : (float)tot;
    }
  }
}

// Stage-2 adjoint, apply pass: dT = gamma * invstd * (dM - k0 - that * k1); writes dT and dY.
template <class T, int C>
struct k_s2_bwd_apply_args {
  const T* Gd;
  const T* Tm;
  const uint8_t* mask;
  const float* a_sv;
  const float* coef_e;
  const float* coef;
  const float* stats;
  const float* gamma;
  const float* beta;
  T* dT;
  T* dY;
  int hw;
  int tiles;
};
template <class T, int C>
__global__ __launch_bounds__(256) void k_s2_bwd_apply(SegL<k_s2_bwd_apply_args<T, C>> L) {
  const SegB sb = seg_block(L);
  if (sb.x >= sb.gx) return;
  const int bx = sb.x, gx = sb.gx;  // workgroup index and count within the segment
  (void)gx;
  const k_s2_bwd_apply_args<T, C>& a_ = L.a[sb.s];
  const T* __restrict__ const Gd = a_.Gd;
  const T* __restrict__ const Tm = a_.Tm;
  const uint8_t* __restrict__ const mask = a_.mask;
  const float* __restrict__ const a_sv = a_.a_sv;
  const float* __restrict__ const coef_e = a_.coef_e;
  const float* __restrict__ const coef = a_.coef;
  const float* __restrict__ const stats = a_.stats;
  const float* __restrict__ const gamma = a_.gamma;
  const float* __restrict__ const beta = a_.beta;
  T* __restrict__ const dT = a_.dT;
  T* __restrict__ const dY = a_.dY;
  const int hw = a_.hw;
  const int tiles = a_.tiles;
  constexpr int G = C / 4;
  const int b = bx / tiles, tx = bx - b * tiles;  // clip, tile of the clip
  const int64_t items = (int64_t)hw * G, base = (int64_t)b * hw * C;
  int64_t i = (int64_t)tx * STDA_BLOCK + threadIdx.x;
  const int c0 = (int)(i % G) * 4;
  float a4v[4], e4[4], mu[4], is[4], ga[4], be[4], k0[4], k1[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    a4v[j] = a_sv[b * C + c0 + j];
    e4[j] = coef_e[b * C + c0 + j];
    mu[j] = stats[c0 + j];
    is[j] = stats[C + c0 + j];
    ga[j] = gamma[c0 + j];
    be[j] = beta[c0 + j];
    k0[j] = coef[c0 + j];
    k1[j] = coef[C + c0 + j];
  }
  for (; i < items; i += (int64_t)tiles * STDA_BLOCK) {
    const int64_t off = base + (i / G) * C + c0;
    float g[4], t[4], dy[4], dt[4];
    ld4(Gd + off, g);
    ld4(Tm + off, t);
    const unsigned bits = mask[off >> 2];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float th = (t[j] - mu[j]) * is[j];
      dy[j] = a4v[j] * g[j] + e4[j];
      const float dm = ((bits >> j) & 1u) ? dy[j] : 0.f;
      dt[j] = ga[j] * is[j] * (dm - k0[j] - th * k1[j]);
    }
    st4(dT + off, dt);
    st4(dY + off, dy);
  }
}

// --------------------------------------------------------------------- input-module adjoint
// dx[c](y, x) = sum_o sum_{ky,kx} dTp[o](y - ky + 1, x - kx + 1) w[o][c][ky][kx]; planar FP32.
template <class T>
struct k_stem_dx_args {
  const T* dTp;
  const float* w;
  float* dx;
  int B;
  int H;
  int W;
};
template <class T>
__global__ __launch_bounds__(256) void k_stem_dx(SegL<k_stem_dx_args<T>> L) {
  const SegB sb = seg_block(L);
  if (sb.x >= sb.gx) return;
  const int bx = sb.x, gx = sb.gx;  // workgroup index and count within the segment
  (void)gx;
  const k_stem_dx_args<T>& a_ = L.a[sb.s];
  const T* __restrict__ const dTp = a_.dTp;
  const float* __restrict__ const w = a_.w;
  float* __restrict__ const dx = a_.dx;
  const int B = a_.B;
  const int H = a_.H;
  const int W = a_.W;
  const int64_t P = (int64_t)B * H * W;
  for (int64_t p = (int64_t)bx * STDA_BLOCK + threadIdx.x; p < P; p += (int64_t)gx * STDA_BLOCK) {
    int b, y, x;
    pix3(p, H, W, b, y, x);
    float acc[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int yy = y - t / 3 + 1, xx = x - t % 3 + 1;
      if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
      const T* row = dTp + (((int64_t)b * H + yy) * W + xx) * 16;
#pragma unroll
      for (int o = 0; o < 16; o += 4) {
        float v[4];
        ld4(row + o, v);
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[c] += w[(o + j) * 27 + c * 9 + t] * v[j];
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) dx[(((int64_t)b * 3 + c) * H + y) * W + x] = acc[c];
  }
}

// --------------------------------------------------------------------- SGD
__global__ __launch_bounds__(256) void k_sgd(float* __restrict__ w, const float* __restrict__ g, int64_t n, float lr,
                                             float wd, uint16_t* __restrict__ wb) {
  for (int64_t i = (int64_t)blockIdx.x * STDA_BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * STDA_BLOCK) {
    const float v = w[i] - lr * (g[i] + wd * w[i]);
    w[i] = v;
    if (wb) wb[i] = from_f<bf16>(v).v;
  }
}

}  // namespace stda
