// Hand-written adjoint kernels of the Radar-STDA network (gfx950), NHWC, FP32 or BF16 storage.
#pragma once
#include <type_traits>

#include "net_kernels.h"

namespace stda {

// --------------------------------------------------------------------- output module adjoint
// dd[c](y, x) = sum_{ky,kx} dz(y - ky + 1, x - kx + 1) w[c][ky][kx]   (16 channels, NHWC), and
// the output-module weight gradient from the same dz neighbourhood:
// dW[c][ky][kx] = sum_p dz(p) d[c](p + (ky - 1, kx - 1)) = sum_q d[c](q) dz(q - (ky - 1, kx - 1)).
// part[blk][10][16]: rows 0..8 the taps, row 9 channel 0 the bias gradient (sum of dz).
template <class T>
__global__ __launch_bounds__(256) void k_head_bwd(const float* __restrict__ dz, const float* __restrict__ w,
                                                  const T* __restrict__ d, T* __restrict__ dd,
                                                  float* __restrict__ part, int B, int H, int W) {
  constexpr int C = 16, G = 4;
  __shared__ float sm[4 * 10 * C];
  __shared__ float red[10 * C];
  const int64_t items = (int64_t)B * H * W * G;
  int64_t i = (int64_t)blockIdx.x * STDA_BLOCK + threadIdx.x;
  const int c0 = (int)(i % G) * 4;
  float wt[9][4];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) wt[t][j] = w[(c0 + j) * 9 + t];
  float acc[10][4];
#pragma unroll
  for (int t = 0; t < 10; ++t) zero4(acc[t]);
  for (; i < items; i += (int64_t)gridDim.x * STDA_BLOCK) {
    const int64_t p = i / G;
    int b, y, x;
    pix3(p, H, W, b, y, x);
    float dv[4], o[4];
    ld4(d + p * C + c0, dv);
    zero4(o);
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int yy = y - t / 3 + 1, xx = x - t % 3 + 1;
      if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
      const float g = dz[((int64_t)b * H + yy) * W + xx];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        o[j] += wt[t][j] * g;
        acc[t][j] += dv[j] * g;
      }
    }
    if (c0 == 0) acc[9][0] += dz[p];
    st4(dd + p * C + c0, o);
  }
  block_chan_reduce_shfl<G, 10>(acc, sm, red);
  for (int q = threadIdx.x; q < 10 * C; q += STDA_BLOCK) part[(int64_t)blockIdx.x * 10 * C + q] = red[q];
}

// ------------------------------------------------------------------ weight gradients (SIMT)
// part[blk][k][n] = sum over the block's pixels p of A(p)[k] * B(p)[n].  Pixels are taken in
// chunks of PCH: both operands of a chunk are staged in LDS, then every thread accumulates
// its fixed set of (k, n) outputs.  Loaders fill 4 consecutive k (or n) per call.
template <class L, int PCH>
__global__ __launch_bounds__(256) void k_wgrad(L ld, float* __restrict__ part) {
  constexpr int K = L::K, N = L::N, NOUT = (K * N + STDA_BLOCK - 1) / STDA_BLOCK;
  __shared__ float As[PCH * K];
  __shared__ float Bs[PCH * N];
  float acc[NOUT];
  int ko[NOUT], no[NOUT];
#pragma unroll
  for (int i = 0; i < NOUT; ++i) {
    acc[i] = 0.f;
    const int o = threadIdx.x + i * STDA_BLOCK;
    ko[i] = o < K * N ? o / N : 0;
    no[i] = o < K * N ? o % N : 0;
  }
  const int64_t P = ld.npix();
  const int64_t nchunks = (P + PCH - 1) / PCH;
  for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    const int64_t p0 = ch * PCH;
    for (int e = threadIdx.x; e < PCH * K / 4; e += STDA_BLOCK) {
      const int pp = e / (K / 4), k4 = (e % (K / 4)) * 4;
      float v[4];
      if (p0 + pp < P) ld.a4(p0 + pp, k4, v); else zero4(v);
#pragma unroll
      for (int j = 0; j < 4; ++j) As[pp * K + k4 + j] = v[j];
    }
    for (int e = threadIdx.x; e < PCH * N / 4; e += STDA_BLOCK) {
      const int pp = e / (N / 4), n4 = (e % (N / 4)) * 4;
      float v[4];
      if (p0 + pp < P) ld.b4(p0 + pp, n4, v); else zero4(v);
#pragma unroll
      for (int j = 0; j < 4; ++j) Bs[pp * N + n4 + j] = v[j];
    }
    __syncthreads();
    for (int pp = 0; pp < PCH; ++pp)
#pragma unroll
      for (int i = 0; i < NOUT; ++i) acc[i] += As[pp * K + ko[i]] * Bs[pp * N + no[i]];
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < NOUT; ++i) {
    const int o = threadIdx.x + i * STDA_BLOCK;
    if (o < K * N) part[(int64_t)blockIdx.x * K * N + o] = acc[i];
  }
}

// Conv3x3-s2-p1 weight gradient: p over output pixels (ho x wo); A = im2col of the input
// (k = tap*CIN + c), B = output gradient (n = o).
template <class T, int CIN, int COUT>
struct WgEncS2 {
  static constexpr int K = 9 * CIN, N = COUT;
  static constexpr bool kBF16Operands = std::is_same<T, bf16>::value;
  const T* X;
  const T* D;
  int B, ho, wo;
  __device__ int64_t npix() const { return (int64_t)B * ho * wo; }
  __device__ void a4(int64_t p, int k, float v[4]) const {
    int b, y, x;
    pix3(p, ho, wo, b, y, x);
    const int tap = k / CIN, c = k % CIN;
    const int iy = 2 * y - 1 + tap / 3, ix = 2 * x - 1 + tap % 3;
    if (iy < 0 || iy >= 2 * ho || ix < 0 || ix >= 2 * wo) { zero4(v); return; }
    ld4(X + (((int64_t)b * 2 * ho + iy) * 2 * wo + ix) * CIN + c, v);
  }
  __device__ void b4(int64_t p, int n, float v[4]) const { ld4(D + p * COUT + n, v); }
};

// DeConv4x4-s2-p1 weight gradient: p over input pixels (hi x wi); A = input (k = c),
// B = gathered output gradient (n = tap*COUT + o) at (2i - 1 + ky, 2j - 1 + kx).
template <class T, int CIN, int COUT>
struct WgDecS2 {
  static constexpr int K = CIN, N = 16 * COUT;
  static constexpr bool kBF16Operands = std::is_same<T, bf16>::value;
  const T* X;
  const T* D;
  int B, hi, wi;
  __device__ int64_t npix() const { return (int64_t)B * hi * wi; }
  __device__ void a4(int64_t p, int k, float v[4]) const { ld4(X + p * CIN + k, v); }
  __device__ void b4(int64_t p, int n, float v[4]) const {
    int b, i, j;
    pix3(p, hi, wi, b, i, j);
    const int tap = n / COUT, o = n % COUT;
    const int yy = 2 * i - 1 + tap / 4, xx = 2 * j - 1 + tap % 4;
    if (yy < 0 || yy >= 2 * hi || xx < 0 || xx >= 2 * wi) { zero4(v); return; }
    ld4(D + (((int64_t)b * 2 * hi + yy) * 2 * wi + xx) * COUT + o, v);
  }
};

// Pointwise weight gradient: A = input row (k = c), B = output gradient row (n = o).
template <class T, int C>
struct WgPw {
  static constexpr int K = C, N = C;
  static constexpr bool kBF16Operands = std::is_same<T, bf16>::value;
  const T* X;
  const T* D;
  int64_t P;
  __device__ int64_t npix() const { return P; }
  __device__ void a4(int64_t p, int k, float v[4]) const { ld4(X + p * C + k, v); }
  __device__ void b4(int64_t p, int n, float v[4]) const { ld4(D + p * C + n, v); }
};

// Input-module weight gradient: A = planar 3-channel im2col (k = c*9 + tap, k = 27 zero),
// B = pre-BN output gradient (16 channels).
template <class T>
struct WgStem {
  static constexpr int K = 28, N = 16;
  static constexpr bool kBF16Operands = false;  // the boundary input is FP32
  const float* x;
  const T* D;
  int B, H, W;
  __device__ int64_t npix() const { return (int64_t)B * H * W; }
  __device__ void a4(int64_t p, int k, float v[4]) const {
    int b, y, xx;
    pix3(p, H, W, b, y, xx);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kk = k + j;
      v[j] = 0.f;
      if (kk >= 27) continue;
      const int c = kk / 9, t = kk % 9;
      const int iy = y + t / 3 - 1, ix = xx + t % 3 - 1;
      if (iy >= 0 && iy < H && ix >= 0 && ix < W) v[j] = x[(((int64_t)b * 3 + c) * H + iy) * W + ix];
    }
  }
  __device__ void b4(int64_t p, int n, float v[4]) const { ld4(D + p * 16 + n, v); }
};

// Output-module weight gradient: A = 16-channel im2col (k = tap*16 + c) plus a ones column
// (k = 144) for the bias, padded to 148; B = dz in column 0 of 4.
template <class T>
struct WgHead {
  static constexpr int K = 148, N = 4;
  static constexpr bool kBF16Operands = false;  // dz is FP32
  const T* d;
  const float* dz;
  int B, H, W;
  __device__ int64_t npix() const { return (int64_t)B * H * W; }
  __device__ void a4(int64_t p, int k, float v[4]) const {
    if (k >= 144) {
      v[0] = k == 144 ? 1.f : 0.f;
      v[1] = v[2] = v[3] = 0.f;
      return;
    }
    int b, y, x;
    pix3(p, H, W, b, y, x);
    const int t = k / 16, c = k % 16;
    const int iy = y + t / 3 - 1, ix = x + t % 3 - 1;
    if (iy < 0 || iy >= H || ix < 0 || ix >= W) { zero4(v); return; }
    ld4(d + (((int64_t)b * H + iy) * W + ix) * 16 + c, v);
  }
  __device__ void b4(int64_t p, int n, float v[4]) const {
    v[0] = n == 0 ? dz[p] : 0.f;
    v[1] = v[2] = v[3] = 0.f;
  }
};

// Depthwise weight gradient: part[blk][t][c] = sum_p X[c](p + off_t) dD[c](p), written at
// the weight's own tap index (flipped for the transposed form).
template <class T, int C, bool DEC>
__global__ __launch_bounds__(256) void k_dw_wgrad(const T* __restrict__ X, const T* __restrict__ dD,
                                                  float* __restrict__ part, int B, int h, int w) {
  constexpr int G = C / 4;
  __shared__ float sm[9 * 4 * STDA_BLOCK];
  __shared__ float red[9 * C];
  const int64_t items = (int64_t)B * h * w * G;
  int64_t i = (int64_t)blockIdx.x * STDA_BLOCK + threadIdx.x;
  const int c0 = (int)(i % G) * 4;
  float acc[9][4];
#pragma unroll
  for (int t = 0; t < 9; ++t) zero4(acc[t]);
  for (; i < items; i += (int64_t)gridDim.x * STDA_BLOCK) {
    const int64_t p = i / G;
    int b, y, x;
    pix3(p, h, w, b, y, x);
    float g[4];
    ld4(dD + p * C + c0, g);
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int yy = y + t / 3 - 1, xx = x + t % 3 - 1;
      if (yy < 0 || yy >= h || xx < 0 || xx >= w) continue;
      float v[4];
      ld4(X + (((int64_t)b * h + yy) * w + xx) * C + c0, v);
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[t][j] += v[j] * g[j];
    }
  }
  block_chan_reduce<G, 9>(acc, sm, red);
  for (int q = threadIdx.x; q < 9 * C; q += STDA_BLOCK) {
    const int t = q / C, c = q % C;
    const int tw = DEC ? 8 - t : t;
    part[(int64_t)blockIdx.x * 9 * C + tw * C + c] = red[q];
  }
}

// --------------------------------------------------------------------- ECA adjoint
// gap-like partials of sum_hw G * Y per (clip, tile, channel).
template <class T, int C>
__global__ __launch_bounds__(256) void k_eca_bwd_part(const T* __restrict__ Gd, const T* __restrict__ Y,
                                                      float* __restrict__ part, int hw) {
  constexpr int G = C / 4;
  __shared__ float sm[4 * STDA_BLOCK];
  __shared__ float red[C];
  const int b = blockIdx.y, tiles = gridDim.x;
  const int64_t items = (int64_t)hw * G, base = (int64_t)b * hw * C;
  int64_t i = (int64_t)blockIdx.x * STDA_BLOCK + threadIdx.x;
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
  for (int q = threadIdx.x; q < C; q += STDA_BLOCK) part[((int64_t)b * tiles + blockIdx.x) * C + q] = red[q];
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
__global__ __launch_bounds__(256) void k_s2_bwd_stats(const T* __restrict__ Gd, const T* __restrict__ Tm,
                                                      const uint8_t* __restrict__ mask,
                                                      const float* __restrict__ epart, const float* __restrict__ a_sv,
                                                      const float* __restrict__ g_sv, const float* __restrict__ weca,
                                                      const float* __restrict__ stats, const float* __restrict__ gamma,
                                                      const float* __restrict__ beta, float* __restrict__ coef_e,
                                                      float* __restrict__ ecaw, float* __restrict__ part, int hw,
                                                      int etiles) {
  constexpr int G = C / 4;
  __shared__ float ds_s[C], e_s[C];
  __shared__ float sm[2 * 4 * STDA_BLOCK];
  __shared__ float red[2 * C];
  const int b = blockIdx.y, tiles = gridDim.x;
  eca_adjoint_clip<C>(epart + (int64_t)b * etiles * C, etiles, hw, a_sv + b * C, g_sv + b * C, weca, ds_s, e_s,
                      blockIdx.x == 0 ? ecaw + b * 3 : nullptr);
  if (blockIdx.x == 0)
    for (int c = threadIdx.x; c < C; c += STDA_BLOCK) coef_e[b * C + c] = e_s[c];
  const int64_t items = (int64_t)hw * G, base = (int64_t)b * hw * C;
  int64_t i = (int64_t)blockIdx.x * STDA_BLOCK + threadIdx.x;
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
  const int64_t blk = (int64_t)b * tiles + blockIdx.x;
  for (int q = threadIdx.x; q < 2 * C; q += STDA_BLOCK) part[blk * 2 * C + q] = red[q];
}

// BN adjoint coefficients from column sums sums[s][C]: beta gradient = sums[0], gamma
// gradient of layer k = sums[1 + k]; coef[s][C] = sums[s] / n.
struct BnBwdOut {
  float* dgamma[3];
  float* dbeta[3];
};
__global__ void k_bn_bwd_finalize(const double* __restrict__ sums, int NS, int C, double n, BnBwdOut out,
                                  float* __restrict__ coef, int accumulate) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  for (int k = 0; k < NS - 1; ++k) {
    const double db = sums[c], dg = sums[(1 + k) * C + c];
    out.dbeta[k][c] = accumulate ? (float)((double)out.dbeta[k][c] + db) : (float)db;
    out.dgamma[k][c] = accumulate ? (float)((double)out.dgamma[k][c] + dg) : (float)dg;
  }
  for (int s = 0; s < NS; ++s) coef[s * C + c] = (float)(sums[s * C + c] / n);
}

// Cross-block FP64 reduction of BN adjoint partials part[blk][NS][C] fused with
// k_bn_bwd_finalize's epilogue.  Block = 4 channels (4 NS columns) x 64 / NS row groups.
__global__ __launch_bounds__(256) void k_bn_bwd_reduce(const float* __restrict__ part, int nrows, int NS, int C,
                                                       double n, BnBwdOut out, float* __restrict__ coef,
                                                       int accumulate) {
  __shared__ double sm[256];
  const int cols = 4 * NS, groups = 256 / cols;
  const int col = threadIdx.x % cols, rg = threadIdx.x / cols;
  const int c0 = blockIdx.x * 4;
  const int s = col / 4, c = c0 + col % 4;
  double acc = 0.0;
  if (rg < groups) {
#pragma unroll 4
    for (int r = rg; r < nrows; r += groups) acc += (double)part[(int64_t)r * NS * C + s * C + c];
  }
  sm[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < cols) {
    double tot = 0.0;
    for (int k = 0; k < groups; ++k) tot += sm[k * cols + threadIdx.x];
    sm[threadIdx.x] = tot;  // each slot is read only by the thread that owns it
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int cc = c0 + threadIdx.x;
    const double db = sm[threadIdx.x];
    for (int k = 0; k < NS - 1; ++k) {
      const double dg = sm[(1 + k) * 4 + threadIdx.x];
      out.dbeta[k][cc] = accumulate ? (float)((double)out.dbeta[k][cc] + db) : (float)db;
      out.dgamma[k][cc] = accumulate ? (float)((double)out.dgamma[k][cc] + dg) : (float)dg;
    }
    for (int q = 0; q < NS; ++q) coef[q * C + cc] = (float)(sm[q * 4 + threadIdx.x] / n);
  }
}

// Stage-2 adjoint, apply pass: dT = gamma * invstd * (dM - k0 - that * k1); writes dT and dY.
template <class T, int C>
__global__ __launch_bounds__(256) void k_s2_bwd_apply(const T* __restrict__ Gd, const T* __restrict__ Tm,
                                                      const uint8_t* __restrict__ mask,
                                                      const float* __restrict__ a_sv, const float* __restrict__ coef_e,
                                                      const float* __restrict__ coef, const float* __restrict__ stats,
                                                      const float* __restrict__ gamma, const float* __restrict__ beta,
                                                      T* __restrict__ dT, T* __restrict__ dY, int hw) {
  constexpr int G = C / 4;
  const int b = blockIdx.y, tiles = gridDim.x;
  const int64_t items = (int64_t)hw * G, base = (int64_t)b * hw * C;
  int64_t i = (int64_t)blockIdx.x * STDA_BLOCK + threadIdx.x;
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

// --------------------------------------------------------------------- stage-1 adjoint
// Statistics pass: du = dX1 * [X1 > 0]; branch outputs recomputed from X.
// part[blk][4][C]: sum du, sum du*phat, sum du*dhat, sum du*xhat.
template <class T, int C, bool DEC>
__global__ __launch_bounds__(256) void k_s1_bwd_stats(const T* __restrict__ X, const T* __restrict__ X1,
                                                      const T* __restrict__ dX1, float* __restrict__ part,
                                                      S1Params prm, int B, int h, int w) {
  constexpr int G = C / 4;
  __shared__ float wp[C * C];
  __shared__ float wd[9 * C];
  __shared__ float sm[4 * 4 * STDA_BLOCK];
  __shared__ float red[4 * C];
  stage1_load_weights<C, DEC>(prm.wpw, prm.wdw, wp, wd);
  const int64_t items = (int64_t)B * h * w * G;
  int64_t i = (int64_t)blockIdx.x * STDA_BLOCK + threadIdx.x;
  const int c0 = (int)(i % G) * 4;
  float mu[3][4], is[3][4];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      mu[k][j] = prm.stats[k][c0 + j];
      is[k][j] = prm.stats[k][C + c0 + j];
    }
  float acc[4][4];
#pragma unroll
  for (int s = 0; s < 4; ++s) zero4(acc[s]);
  for (; i < items; i += (int64_t)gridDim.x * STDA_BLOCK) {
    const int64_t p = i / G;
    int b, y, x;
    pix3(p, h, w, b, y, x);
    float pv[4], dv[4], xv[4], x1[4], g[4];
    stage1_branches<T, C>(X, p, b, y, x, h, w, c0, wp, wd, pv, dv, xv);
    ld4(X1 + p * C + c0, x1);
    ld4(dX1 + p * C + c0, g);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float du = x1[j] > 0.f ? g[j] : 0.f;
      acc[0][j] += du;
      acc[1][j] += du * (pv[j] - mu[0][j]) * is[0][j];
      acc[2][j] += du * (dv[j] - mu[1][j]) * is[1][j];
      acc[3][j] += du * (xv[j] - mu[2][j]) * is[2][j];
    }
  }
  block_chan_reduce<G, 4>(acc, sm, red);
  for (int q = threadIdx.x; q < 4 * C; q += STDA_BLOCK) part[(int64_t)blockIdx.x * 4 * C + q] = red[q];
}

// Apply pass: the three BN adjoints.  Writes dP, dD and dX0 = dX_identity + dXres.
template <class T, int C, bool DEC>
__global__ __launch_bounds__(256) void k_s1_bwd_apply(const T* __restrict__ X, const T* __restrict__ X1,
                                                      const T* __restrict__ dX1, const T* __restrict__ dXr,
                                                      const float* __restrict__ coef, S1Params prm,
                                                      T* __restrict__ dP, T* __restrict__ dD, T* __restrict__ dX0,
                                                      int B, int h, int w) {
  constexpr int G = C / 4;
  __shared__ float wp[C * C];
  __shared__ float wd[9 * C];
  stage1_load_weights<C, DEC>(prm.wpw, prm.wdw, wp, wd);
  const int64_t items = (int64_t)B * h * w * G;
  int64_t i = (int64_t)blockIdx.x * STDA_BLOCK + threadIdx.x;
  const int c0 = (int)(i % G) * 4;
  float mu[3][4], is[3][4], ga[3][4], k[4][4];
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      mu[q][j] = prm.stats[q][c0 + j];
      is[q][j] = prm.stats[q][C + c0 + j];
      ga[q][j] = prm.gamma[q][c0 + j];
    }
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int j = 0; j < 4; ++j) k[s][j] = coef[s * C + c0 + j];
  for (; i < items; i += (int64_t)gridDim.x * STDA_BLOCK) {
    const int64_t p = i / G;
    int b, y, x;
    pix3(p, h, w, b, y, x);
    float pv[4], dv[4], xv[4], x1[4], g[4], r[4];
    stage1_branches<T, C>(X, p, b, y, x, h, w, c0, wp, wd, pv, dv, xv);
    ld4(X1 + p * C + c0, x1);
    ld4(dX1 + p * C + c0, g);
    ld4(dXr + p * C + c0, r);
    float op[4], od[4], ox[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float du = x1[j] > 0.f ? g[j] : 0.f;
      const float ph = (pv[j] - mu[0][j]) * is[0][j];
      const float dh = (dv[j] - mu[1][j]) * is[1][j];
      const float xh = (xv[j] - mu[2][j]) * is[2][j];
      op[j] = ga[0][j] * is[0][j] * (du - k[0][j] - ph * k[1][j]);
      od[j] = ga[1][j] * is[1][j] * (du - k[0][j] - dh * k[2][j]);
      ox[j] = ga[2][j] * is[2][j] * (du - k[0][j] - xh * k[3][j]) + r[j];
    }
    st4(dP + p * C + c0, op);
    st4(dD + p * C + c0, od);
    st4(dX0 + p * C + c0, ox);
  }
}

// Input gradient of stage 1: dX = dX0 + pointwise^T(dP) + depthwise^T(dD) (+ skip gradient).
template <class T, int C, bool DEC, bool SKIP>
__global__ __launch_bounds__(256) void k_s1_bwd_dx(const T* __restrict__ dP, const T* __restrict__ dD,
                                                   const T* __restrict__ dX0, const T* __restrict__ skip,
                                                   S1Params prm, T* __restrict__ dX, int B, int h, int w) {
  constexpr int G = C / 4;
  __shared__ float wp[C * C];
  __shared__ float wpT[C * C];
  __shared__ float wd[9 * C];
  stage1_load_weights<C, DEC>(prm.wpw, prm.wdw, wp, wd);
  for (int q = threadIdx.x; q < C * C; q += STDA_BLOCK) wpT[(q % C) * C + q / C] = wp[q];  // wpT[o][c]
  __syncthreads();
  const int64_t items = (int64_t)B * h * w * G;
  int64_t i = (int64_t)blockIdx.x * STDA_BLOCK + threadIdx.x;
  const int c0 = (int)(i % G) * 4;
  for (; i < items; i += (int64_t)gridDim.x * STDA_BLOCK) {
    const int64_t p = i / G;
    int b, y, x;
    pix3(p, h, w, b, y, x);
    float acc[4];
    ld4(dX0 + p * C + c0, acc);
    if (SKIP) {
      float s[4];
      ld4(skip + p * C + c0, s);
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] += s[j];
    }
    const T* row = dP + p * C;
#pragma unroll 4
    for (int o = 0; o < C; o += 4) {
      float v[4];
      ld4(row + o, v);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float4 wq = *reinterpret_cast<const float4*>(wpT + (o + j) * C + c0);
        acc[0] += wq.x * v[j];
        acc[1] += wq.y * v[j];
        acc[2] += wq.z * v[j];
        acc[3] += wq.w * v[j];
      }
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int yy = y - (t / 3 - 1), xx = x - (t % 3 - 1);
      if (yy < 0 || yy >= h || xx < 0 || xx >= w) continue;
      float v[4];
      ld4(dD + (((int64_t)b * h + yy) * w + xx) * C + c0, v);
      const float4 wq = *reinterpret_cast<const float4*>(wd + t * C + c0);
      acc[0] += wq.x * v[0];
      acc[1] += wq.y * v[1];
      acc[2] += wq.z * v[2];
      acc[3] += wq.w * v[3];
    }
    st4(dX + p * C + c0, acc);
  }
}

// --------------------------------------------------------------------- input-module adjoint
// The pre-BN output is recomputed from the planar input (4 channels per thread).
// Statistics: dM = dS * [S > 0] (S = stored module output); part[blk][2][16]: sum dM, sum dM*that.
template <class T>
__global__ __launch_bounds__(256) void k_stem_bwd_stats(const T* __restrict__ dS, const T* __restrict__ S,
                                                        const float* __restrict__ x, const float* __restrict__ w,
                                                        const float* __restrict__ stats, float* __restrict__ part,
                                                        int B, int H, int W) {
  constexpr int C = 16, G = 4;
  __shared__ float sm[2 * 4 * STDA_BLOCK];
  __shared__ float red[2 * C];
  const int64_t items = (int64_t)B * H * W * G;
  int64_t i = (int64_t)blockIdx.x * STDA_BLOCK + threadIdx.x;
  const int c0 = (int)(i % G) * 4;
  float mu[4], is[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    mu[j] = stats[c0 + j];
    is[j] = stats[C + c0 + j];
  }
  float acc[2][4];
  zero4(acc[0]);
  zero4(acc[1]);
  for (; i < items; i += (int64_t)gridDim.x * STDA_BLOCK) {
    const int64_t p = i / G;
    int b, y, xx;
    pix3(p, H, W, b, y, xx);
    float g[4], s[4], t[4];
    ld4(dS + p * C + c0, g);
    ld4(S + p * C + c0, s);
    stem_conv<4>(x, w, b, y, xx, H, W, c0, t);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float dm = s[j] > 0.f ? g[j] : 0.f;
      acc[0][j] += dm;
      acc[1][j] += dm * (t[j] - mu[j]) * is[j];
    }
  }
  block_chan_reduce<G, 2>(acc, sm, red);
  for (int q = threadIdx.x; q < 2 * C; q += STDA_BLOCK) part[(int64_t)blockIdx.x * 2 * C + q] = red[q];
}

// Apply: dTp = gamma * invstd * (dM - k0 - that * k1), fused with the input-module weight
// gradient dW[o][c][tap] = sum_p dTp[o](p) x[c](p + off_tap): part[blk][27][16] (row = c*9 + tap).
// dTp itself is written only when the input gradient is wanted (dTp != nullptr).
template <class T>
__global__ __launch_bounds__(256) void k_stem_bwd_apply(const T* __restrict__ dS, const T* __restrict__ S,
                                                        const float* __restrict__ x, const float* __restrict__ w,
                                                        const float* __restrict__ stats, const float* __restrict__ gamma,
                                                        const float* __restrict__ coef, T* __restrict__ dTp,
                                                        float* __restrict__ part, int B, int H, int W) {
  constexpr int C = 16, G = 4;
  __shared__ float sm[4 * 27 * C];
  __shared__ float red[27 * C];
  const int64_t items = (int64_t)B * H * W * G;
  int64_t i = (int64_t)blockIdx.x * STDA_BLOCK + threadIdx.x;
  const int c0 = (int)(i % G) * 4;
  float mu[4], is[4], ga[4], k0[4], k1[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    mu[j] = stats[c0 + j];
    is[j] = stats[C + c0 + j];
    ga[j] = gamma[c0 + j];
    k0[j] = coef[c0 + j];
    k1[j] = coef[C + c0 + j];
  }
  float acc[27][4];
#pragma unroll
  for (int k = 0; k < 27; ++k) zero4(acc[k]);
  for (; i < items; i += (int64_t)gridDim.x * STDA_BLOCK) {
    const int64_t p = i / G;
    int b, y, xx;
    pix3(p, H, W, b, y, xx);
    float g[4], s[4], t[4], o[4];
    ld4(dS + p * C + c0, g);
    ld4(S + p * C + c0, s);
    float xv[27];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int tp = 0; tp < 9; ++tp) {
        const int iy = y + tp / 3 - 1, ix = xx + tp % 3 - 1;
        xv[c * 9 + tp] = (iy >= 0 && iy < H && ix >= 0 && ix < W) ? x[(((int64_t)b * 3 + c) * H + iy) * W + ix] : 0.f;
      }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float a = 0.f;
#pragma unroll
      for (int k = 0; k < 27; ++k) a += w[(c0 + j) * 27 + k] * xv[k];
      t[j] = a;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float dm = s[j] > 0.f ? g[j] : 0.f;
      o[j] = ga[j] * is[j] * (dm - k0[j] - (t[j] - mu[j]) * is[j] * k1[j]);
    }
#pragma unroll
    for (int k = 0; k < 27; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[k][j] += o[j] * xv[k];
    if (dTp) st4(dTp + p * C + c0, o);
  }
  block_chan_reduce_shfl<G, 27>(acc, sm, red);
  for (int q = threadIdx.x; q < 27 * C; q += STDA_BLOCK) part[(int64_t)blockIdx.x * 27 * C + q] = red[q];
}

// dx[c](y, x) = sum_o sum_{ky,kx} dTp[o](y - ky + 1, x - kx + 1) w[o][c][ky][kx]; planar FP32.
template <class T>
__global__ __launch_bounds__(256) void k_stem_dx(const T* __restrict__ dTp, const float* __restrict__ w,
                                                 float* __restrict__ dx, int B, int H, int W) {
  const int64_t P = (int64_t)B * H * W;
  for (int64_t p = (int64_t)blockIdx.x * STDA_BLOCK + threadIdx.x; p < P; p += (int64_t)gridDim.x * STDA_BLOCK) {
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
