// Radar-STDA network kernels (gfx950), NHWC activations, FP32 or BF16 storage, FP32 math.
//
// Thread mapping of the per-pixel kernels: one thread per (pixel, group of 4 channels), the
// channel group fastest, so consecutive threads read consecutive 16-byte (FP32) / 8-byte (BF16)
// pieces of NHWC rows.  Per-channel sums (BN statistics, GAP, wgrad of the depthwise branch)
// are reduced inside the block in a fixed order and written as per-block partials; separate
// column-sum kernels reduce the partials across blocks in FP64.  Nothing uses float atomics,
// so every result is bitwise reproducible run to run.
#pragma once
#include "common.h"

namespace stda {

constexpr float BN_EPS = 1e-5f;

__device__ __forceinline__ void pix3(int64_t p, int h, int w, int& b, int& y, int& x) {
  const int64_t hw = (int64_t)h * w;
  b = (int)(p / hw);
  const int r = (int)(p - (int64_t)b * hw);
  y = r / w;
  x = r - y * w;
}

// Sums, per channel, the NS x 4 values each thread holds for its channel group into
// red[s * C + c] (LDS); sm is scratch of NS * 4 * STDA_BLOCK floats.
template <int G, int NS>
__device__ __forceinline__ void block_chan_reduce(const float (&v)[NS][4], float* sm, float* red) {
  const int t = threadIdx.x;
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int j = 0; j < 4; ++j) sm[(s * 4 + j) * STDA_BLOCK + t] = v[s][j];
  __syncthreads();
  constexpr int C = 4 * G;
  for (int i = t; i < NS * C; i += STDA_BLOCK) {
    const int s = i / C, c = i % C;
    const float* row = sm + (s * 4 + (c & 3)) * STDA_BLOCK;
    float acc = 0.f;
    for (int p = c >> 2; p < STDA_BLOCK; p += G) acc += row[p];
    red[i] = acc;
  }
  __syncthreads();
}

// Same result layout as block_chan_reduce, for many statistics: lanes of a wave that share a
// channel group (lane % G) are combined with shuffles, then the 4 waves through LDS, in a fixed
// order.  sm holds 4 * NS * 4 * G floats.
template <int G, int NS>
__device__ __forceinline__ void block_chan_reduce_shfl(float (&v)[NS][4], float* sm, float* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float a = v[s][j];
#pragma unroll
      for (int off = G; off < 64; off <<= 1) a += __shfl_xor(a, off);
      v[s][j] = a;
    }
  constexpr int C = 4 * G;
  if (lane < G)
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int j = 0; j < 4; ++j) sm[(wave * NS + s) * C + 4 * lane + j] = v[s][j];
  __syncthreads();
  for (int i = threadIdx.x; i < NS * C; i += STDA_BLOCK)
    red[i] = sm[i] + sm[NS * C + i] + sm[2 * NS * C + i] + sm[3 * NS * C + i];
  __syncthreads();
}

// ------------------------------------------------------------------ batch-norm statistics
// A channel's statistics are kept as (count, mean, m2 = sum of squared deviations from the mean):
// Welford's update adds one value, Chan, Golub and LeVeque's pairwise formula merges two partial
// results.  No sum of squares about zero is formed, whose difference E[x^2] - E[x]^2 would lose
// (mean / std)^2 of its precision.
// Adds the k-th value v (rk = 1 / k, the hardware reciprocal: its rounding only perturbs the weight
// of v in the running mean, which m2's update uses consistently) to (mean, m2).
__device__ __forceinline__ void wf_add(float& mean, float& m2, float v, float rk) {
  const float d = v - mean;
  mean = fmaf(d, rk, mean);
  m2 = fmaf(d, v - mean, m2);
}
// Merges (nb, mb, qb) into (ma, qa) of count na (the caller updates the count to na + nb).
__device__ __forceinline__ void chan_merge(float na, float& ma, float& qa, float nb, float mb, float qb) {
  if (nb > 0.f) {
    const float f = nb / (na + nb), d = mb - ma;
    ma = fmaf(d, f, ma);
    qa = qa + qb + d * d * na * f;
  }
}

// Block merge of per-thread statistics, channel-group layout of block_chan_reduce_shfl: thread
// holds count n (the same for all its channels) and (m, q)[s][j] for channels 4 (lane % G) + j
// of NS statistics sets.  Lanes of one channel group merge with shuffles, then the 4 waves
// through LDS in a fixed order.  Result: red[s C + c] = mean, red[NS C + s C + c] = m2, and
// red[2 NS C] = the block's count.  sm holds 4 (2 NS C + 1) floats.
template <int G, int NS>
__device__ __forceinline__ void block_chan_stats(float n, float (&m)[NS][4], float (&q)[NS][4], float* sm, float* red) {
  constexpr int C = 4 * G, ROW = 2 * NS * C + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = G; off < 64; off <<= 1) {
    const float nb = __shfl_xor(n, off);
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float mb = __shfl_xor(m[s][j], off), qb = __shfl_xor(q[s][j], off);
        chan_merge(n, m[s][j], q[s][j], nb, mb, qb);
      }
    n += nb;
  }
  if (lane < G) {
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        sm[wave * ROW + s * C + 4 * lane + j] = m[s][j];
        sm[wave * ROW + NS * C + s * C + 4 * lane + j] = q[s][j];
      }
    if (lane == 0) sm[wave * ROW + 2 * NS * C] = n;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NS * C; i += STDA_BLOCK) {
    float na = sm[2 * NS * C], ma = sm[i], qa = sm[NS * C + i];
#pragma unroll
    for (int w = 1; w < 4; ++w) {
      const float nb = sm[w * ROW + 2 * NS * C];
      chan_merge(na, ma, qa, nb, sm[w * ROW + i], sm[w * ROW + NS * C + i]);
      na += nb;
    }
    red[i] = ma;
    red[NS * C + i] = qa;
    if (i == 0) red[2 * NS * C] = na;
  }
  __syncthreads();
}

// Sum over the block of NV values per thread (all threads hold the same quantities).
template <int NV>
__device__ __forceinline__ void block_vec_reduce(const float (&v)[NV], float* sm, float* red) {
  const int t = threadIdx.x;
#pragma unroll
  for (int i = 0; i < NV; ++i) sm[i * STDA_BLOCK + t] = v[i];
  __syncthreads();
  for (int i = t; i < NV; i += STDA_BLOCK) {
    float acc = 0.f;
    for (int p = 0; p < STDA_BLOCK; ++p) acc += sm[i * STDA_BLOCK + p];
    red[i] = acc;
  }
  __syncthreads();
}

// ------------------------------------------------------------------ cross-block FP64 sums
// out[col] = sum over rows of part[row * ncols + col], in FP64, fixed order.
// Block: 16 columns x 16 row groups.  Epilogue kinds map the column to its destination.
struct ColMap {
  int kind;   // 0: double out[col]; 1..: scatter float into a weight gradient
  int a, b;   // kind-specific sizes
};
enum : int { MAP_DOUBLE = 0, MAP_ENC_S2 = 1, MAP_DEC_S2 = 2, MAP_PW_CONV = 3, MAP_IDENT = 4,
             MAP_DW = 5, MAP_STEM = 6, MAP_HEAD = 7, MAP_PW_DIAG = 8 };

__device__ __forceinline__ int64_t colmap_dst(const ColMap m, int col) {
  switch (m.kind) {
    case MAP_ENC_S2: {  // col = (tap*Cin + c)*Cout + o -> w[o][c][tap]; a = Cin, b = Cout
      const int o = col % m.b, r = col / m.b, c = r % m.a, tap = r / m.a;
      return ((int64_t)o * m.a + c) * 9 + tap;
    }
    case MAP_DEC_S2: {  // col = c*(16*Cout) + tap*Cout + o -> w[c][o][tap]; b = Cout
      const int o = col % m.b, r = col / m.b, tap = r % 16, c = r / 16;
      return ((int64_t)c * m.b + o) * 16 + tap;
    }
    case MAP_PW_CONV: {  // col = c*C + o -> w[o][c]; a = C
      const int o = col % m.a, c = col / m.a;
      return (int64_t)o * m.a + c;
    }
    case MAP_PW_DIAG: {  // col = c*C + o -> w[c] if c == o, else unused; a = C
      const int o = col % m.a, c = col / m.a;
      return c == o ? c : -1;
    }
    case MAP_DW: {  // col = tap*C + c -> w[c][tap]; a = C
      const int c = col % m.a, tap = col / m.a;
      return (int64_t)c * 9 + tap;
    }
    case MAP_STEM: {  // col = k*16 + o, k = c*9 + tap -> w[o][c][tap]
      const int o = col % 16, k = col / 16;
      return (int64_t)o * 27 + k;
    }
    case MAP_HEAD: {  // col = tap*16 + c -> w[c][tap]; tap row 9: channel 0 = bias, others unused
      const int tap = col / 16, c = col % 16;
      if (tap == 9) return c == 0 ? 144 : -1;  // the bias follows the 144 weights
      return (int64_t)c * 9 + tap;
    }
    default:
      return col;
  }
}

// acc += part[r * stride + off] for r = r0, r0 + step, ... < nrows, in that order; 16 loads are
// issued before their adds so that their latencies overlap.
__device__ __forceinline__ double strided_sum(const float* __restrict__ part, int r0, int step, int nrows, int64_t stride,
                                              int64_t off) {
  double acc = 0.0;
  int r = r0;
  for (; r + 15 * step < nrows; r += 16 * step) {
    float v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = part[(int64_t)(r + k * step) * stride + off];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += (double)v[k];
  }
  for (; r < nrows; r += step) acc += (double)part[(int64_t)r * stride + off];
  return acc;
}

// Column sums of part[nrows][ncols] in FP64 (fixed order): a block of NT threads takes CW
// consecutive columns and NT / CW row groups; wide partial arrays use CW = 64 (a wave reads 256
// contiguous bytes of a row), with NT = 1024 where there are few such blocks, so that a thread sums
// one sixteenth of the rows in few dependent batches; narrow ones CW = 16 (more row groups in
// flight per column).
template <int CW, int NT>
__device__ __forceinline__ void colsum_block(const float* __restrict__ part, int nrows, int ncols,
                                             double* __restrict__ dout, float* __restrict__ fout, ColMap map,
                                             int accumulate, int blk) {
  constexpr int RG = NT / CW;
  __shared__ double sm[RG][CW];
  const int cl = threadIdx.x % CW, rg = threadIdx.x / CW;
  const int col = blk * CW + cl;
  const double acc = col < ncols ? strided_sum(part, rg, RG, nrows, ncols, col) : 0.0;
  sm[rg][cl] = acc;
  __syncthreads();
  if (rg == 0 && col < ncols) {
    double s = 0.0;
    for (int i = 0; i < RG; ++i) s += sm[i][cl];
    if (map.kind == MAP_DOUBLE) {
      dout[col] = accumulate ? dout[col] + s : s;
    } else {
      const int64_t d = colmap_dst(map, col);
      if (d >= 0) fout[d] = accumulate ? (float)((double)fout[d] + s) : (float)s;
    }
  }
}
template <int CW, int NT = 256>
__global__ __launch_bounds__(NT) void k_colsum(const float* __restrict__ part, int nrows, int ncols,
                                               double* __restrict__ dout, float* __restrict__ fout,
                                               ColMap map, int accumulate) {
  colsum_block<CW, NT>(part, nrows, ncols, dout, fout, map, accumulate, blockIdx.x);
}
// Two independent column sums into weight gradients in one launch: blocks [0, a.nblk) take job a,
// the rest job b (CW = 16, 256 threads; the same per-column order as k_colsum<16>).
struct ColJob {
  const float* part;
  float* fout;
  ColMap map;
  int nrows, ncols, nblk;
};
__global__ __launch_bounds__(256) void k_colsum2(ColJob a, ColJob b, int accumulate) {
  if ((int)blockIdx.x < a.nblk)
    colsum_block<16, 256>(a.part, a.nrows, a.ncols, nullptr, a.fout, a.map, accumulate, blockIdx.x);
  else
    colsum_block<16, 256>(b.part, b.nrows, b.ncols, nullptr, b.fout, b.map, accumulate, blockIdx.x - a.nblk);
}

// Batch statistics of BN layers from per-block partials, for every segment of a launch.
struct BnSegs {
  int n;                        // segments, merged in this order
  const float* part[kMaxSegs];  // the segment's partials (layout below)
  int rows[kMaxSegs];           // its partial rows (workgroups of the statistics launch)
  float* stats[kMaxSegs];       // its statistics buffer (running-buffer layout)
};
struct BnLayers {
  int64_t off[3];  // offsets of the NB layers in the statistics / running layout
};
// Cross-block FP64 merge of batch-norm statistics partials fused with their finalize, segment
// by segment.  A segment's part[blk][NB][C][2] = (mean, m2) of the block's values per BN layer
// and channel, followed by the blocks' counts cnt[blk] (floats) at part + rows NB C 2.  In FP64,
// one pass in a fixed order, about the first block's mean m0 (d_b = mean_b - m0): n = sum n_b,
// s = sum n_b d_b, q = sum (m2_b + n_b d_b^2); mean = m0 + s / n, var = (q - s^2 / n) / n.  The
// block means lie within a few standard deviations of each other, so nothing cancels beyond
// FP64's reach.  Writes the segment's stats = [mean C][invstd C] per layer; if `running` is not
// null, applies one running-statistics update (momentum 0.1, unbiased variance) per segment, in
// segment order.  Block = one channel of one layer; its 256 threads take every 256th row and
// their (n, s, q) are added in a fixed tree order.
__device__ __forceinline__ void tree3(double (*sm)[3]) {
#pragma unroll
  for (int half = STDA_BLOCK / 2; half > 0; half >>= 1) {
    if ((int)threadIdx.x < half)
#pragma unroll
      for (int k = 0; k < 3; ++k) sm[threadIdx.x][k] += sm[threadIdx.x + half][k];
    __syncthreads();
  }
}
__global__ __launch_bounds__(256) void k_bn_stats_reduce(BnSegs sg, int NB, int C, BnLayers L,
                                                         float* __restrict__ running) {
  __shared__ double sm[STDA_BLOCK][3];
  const int i = blockIdx.x / C, c = blockIdx.x % C;
  const int64_t ncols = (int64_t)NB * C * 2;
  const int64_t col = (int64_t)(i * C + c) * 2;
  for (int sgi = 0; sgi < sg.n; ++sgi) {
    const float* __restrict__ part = sg.part[sgi];
    const int nrows = sg.rows[sgi];
    const float* __restrict__ cnt = part + (int64_t)nrows * ncols;
    const double m0 = (double)part[col];
    double n = 0.0, s = 0.0, q = 0.0;
#pragma unroll 4
    for (int r = threadIdx.x; r < nrows; r += STDA_BLOCK) {
      const double nb = (double)cnt[r];
      const double d = (double)part[(int64_t)r * ncols + col] - m0;
      n += nb;
      s += nb * d;
      q += (double)part[(int64_t)r * ncols + col + 1] + nb * d * d;
    }
    sm[threadIdx.x][0] = n;
    sm[threadIdx.x][1] = s;
    sm[threadIdx.x][2] = q;
    __syncthreads();
    tree3(sm);
    if (threadIdx.x == 0) {
      const double nt = sm[0][0], st = sm[0][1], qt = sm[0][2];
      const double mu = nt > 0.0 ? m0 + st / nt : 0.0;
      double var = nt > 0.0 ? (qt - st * st / nt) / nt : 0.0;
      if (var < 0.0) var = 0.0;
      float* so = sg.stats[sgi] + L.off[i];
      so[c] = (float)mu;
      so[C + c] = (float)(1.0 / sqrt(var + (double)BN_EPS));
      if (running) {
        float* rn = running + L.off[i];
        const double unb = nt > 1.0 ? var * nt / (nt - 1.0) : var;
        rn[c] = (float)(0.9 * (double)rn[c] + 0.1 * mu);
        rn[C + c] = (float)(0.9 * (double)rn[C + c] + 0.1 * unb);
      }
    }
    __syncthreads();  // sm is reused by the next segment
  }
}

// EVAL statistics: mean and 1/sqrt(var + eps) of every BN layer from the running buffer
// (both buffers: per layer C means, then C variances / inverse standard deviations), into the
// statistics buffer of every segment.
struct BnTable {
  int n;
  int off[24];
  int C[24];
  int nseg;
  float* stats[kMaxSegs];
};
__global__ void k_eval_stats(const float* __restrict__ running, BnTable tab) {
  for (int sgi = 0; sgi < tab.nseg; ++sgi) {
    float* __restrict__ stats = tab.stats[sgi];
    for (int l = 0; l < tab.n; ++l) {
      const int C = tab.C[l], off = tab.off[l];
      for (int c = threadIdx.x; c < C; c += blockDim.x) {
        stats[off + c] = running[off + c];
        stats[off + C + c] = 1.0f / sqrtf(running[off + C + c] + BN_EPS);
      }
    }
  }
}

// --------------------------------------------------------------------- stage 1
// Branches of stage 1 (mobile encoder / decoder block, first equation group): pointwise
// (C x C), depthwise 3x3 and identity.  Weights staged in LDS:
//   wp[c][o]   pointwise, out[o] = sum_c wp[c][o] x[c]
//   wd[t][o]   depthwise, t = (dy+1)*3 + (dx+1) neighbour offset, out[o] += wd[t][o] x[o](y+dy, x+dx)
template <int C, bool DEC>
__device__ __forceinline__ void stage1_load_weights(const float* __restrict__ wpw, const float* __restrict__ wdw,
                                                    float* wp, float* wd) {
  for (int i = threadIdx.x; i < C * C; i += STDA_BLOCK) {
    const int c = i / C, o = i % C;
    wp[i] = DEC ? wpw[c * C + o] : wpw[o * C + c];
  }
  for (int i = threadIdx.x; i < 9 * C; i += STDA_BLOCK) {
    const int t = i / C, o = i % C;
    const int dy = t / 3 - 1, dx = t % 3 - 1;
    // conv: weight tap (dy+1, dx+1); transposed (stride 1, pad 1): flipped tap (1-dy, 1-dx)
    wd[i] = DEC ? wdw[o * 9 + (1 - dy) * 3 + (1 - dx)] : wdw[o * 9 + (dy + 1) * 3 + (dx + 1)];
  }
  __syncthreads();
}

// Parameters of the stage-1 kernels (weights, batch statistics and affine of the three BNs).
struct S1Params {
  const float* wpw;
  const float* wdw;
  const float* stats[3];  // pw, dw, id
  const float* gamma[3];
  const float* beta[3];
};

// ---------------------------------------------------------- dense stride-2 layers: tap rules
// out[p][n] = sum over taps and input channels of src[...][k] * wl[tap][k][n]:
//   OP_ENC_FWD   Conv3x3-s2-p1, src grid 2h x 2w -> dst h x w, taps: sy = 2y - 1 + ky
//   OP_DEC_DGRAD adjoint of DeConv4x4-s2-p1 (a Conv4x4-s2-p1), same tap rule with k = 4
//   OP_DEC_FWD   DeConv4x4-s2-p1, src h x w -> dst 2h x 2w, ky = ky0, ky0 + 2, ky0 = (y+1)&1,
//                sy = (y + 1 - ky) / 2
//   OP_ENC_DGRAD adjoint of Conv3x3-s2-p1 (the same up-sampling rule with k = 3)
// wl is laid out [ky*k + kx][K][N] (prepared per call from the PyTorch weights).
enum : int { OP_ENC_FWD = 0, OP_DEC_FWD = 1, OP_ENC_DGRAD = 2, OP_DEC_DGRAD = 3 };

template <int OP> struct OpGeo {
  static constexpr int KS = (OP == OP_ENC_FWD || OP == OP_ENC_DGRAD) ? 3 : 4;
  static constexpr bool DOWN = (OP == OP_ENC_FWD || OP == OP_DEC_DGRAD);
};

// --------------------------------------------------------------- stage 2 apply + GAP
// Y = ReLU(BN(T)) + R; per-(clip, tile) channel sums of Y for the ECA global average pool.
// Workgroups: clip-major (clip, tile) pairs of the segment, `tiles` per clip; gap[clip][tile][C].
// The ReLU decision of every element is taken here, once, in FP32, and (TRAIN) stored as a
// 4-bit mask per (pixel, channel group) byte for the adjoint.
template <class T, int C>
struct k_s2_apply_args {
  const T* Tm;
  const T* R;
  T* Y;
  uint8_t* mask;
  float* gap;
  const float* stats;
  const float* gamma;
  const float* beta;
  int hw;
  int tiles;
};
template <class T, int C>
__global__ __launch_bounds__(256) void k_s2_apply(SegL<k_s2_apply_args<T, C>> L) {
  const SegB sb = seg_block(L);
  if (sb.x >= sb.gx) return;
  const int bx = sb.x, gx = sb.gx;  // workgroup index and count within the segment
  (void)gx;
  const k_s2_apply_args<T, C>& a_ = L.a[sb.s];
  const T* __restrict__ const Tm = a_.Tm;
  const T* __restrict__ const R = a_.R;
  T* __restrict__ const Y = a_.Y;
  uint8_t* __restrict__ const mask = a_.mask;
  float* __restrict__ const gap = a_.gap;
  const float* __restrict__ const stats = a_.stats;
  const float* __restrict__ const gamma = a_.gamma;
  const float* __restrict__ const beta = a_.beta;
  const int hw = a_.hw;
  const int tiles = a_.tiles;
  constexpr int G = C / 4;
  __shared__ float sm[4 * STDA_BLOCK];
  __shared__ float red[C];
  const int b = bx / tiles, tx = bx - b * tiles;  // clip, tile of the clip
  const int64_t items = (int64_t)hw * G;
  const int64_t base = (int64_t)b * hw * C;
  int64_t i = (int64_t)tx * STDA_BLOCK + threadIdx.x;
  const int c0 = (int)(i % G) * 4;
  float sc[4], sh[4];
  bn_affine4(stats, gamma, beta, C, c0, sc, sh);
  float acc[1][4];
  zero4(acc[0]);
  for (; i < items; i += (int64_t)tiles * STDA_BLOCK) {
    const int64_t off = base + (i / G) * C + c0;
    float t[4], r[4];
    ld4(Tm + off, t);
    ld4(R + off, r);
    float o[4];
    unsigned bits = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float v = t[j] * sc[j] + sh[j];
      bits |= (v > 0.f ? 1u : 0u) << j;
      o[j] = fmaxf(v, 0.f) + r[j];
    }
    st4(Y + off, o);
    if (mask) mask[off >> 2] = (uint8_t)bits;
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[0][j] += stored<T>(o[j]);  // the value as stored
  }
  block_chan_reduce<G, 1>(acc, sm, red);
  for (int q = threadIdx.x; q < C; q += STDA_BLOCK) gap[((int64_t)b * tiles + tx) * C + q] = red[q];
}

// ECA scale of one clip from its GAP partials (Sec. IV-C, Eq. (eca_process_equation)):
// g = mean over (h, w); s[c] = w0 g[c-1] + w1 g[c] + w2 g[c+1] (zero padded); a = sigmoid(s).
template <int C>
__device__ __forceinline__ void eca_scale_clip(const float* __restrict__ gap, int tiles, int hw,
                                               const float* __restrict__ weca, float* g_s, float* a_s) {
  for (int c = threadIdx.x; c < C; c += STDA_BLOCK) {
    double s = 0.0;
    for (int t = 0; t < tiles; ++t) s += (double)gap[t * C + c];
    g_s[c] = (float)(s / (double)hw);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < C; c += STDA_BLOCK) {
    const float gm = c > 0 ? g_s[c - 1] : 0.f, gp = c < C - 1 ? g_s[c + 1] : 0.f;
    const float s = weca[0] * gm + weca[1] * g_s[c] + weca[2] * gp;
    a_s[c] = 1.f / (1.f + expf(-s));
  }
  __syncthreads();
}

// Next block input Xn = a[clip][c] * Y (+ skip).  Tile 0 of each clip also saves g and a.
template <class T, int C, bool SKIP>
struct k_eca_next_args {
  const T* Y;
  const T* skip;
  T* Xn;
  const float* gap;
  const float* weca;
  float* g_out;
  float* a_out;
  int hw;
  int gap_tiles;
  int tiles;
};
template <class T, int C, bool SKIP>
__global__ __launch_bounds__(256) void k_eca_next(SegL<k_eca_next_args<T, C, SKIP>> L) {
  const SegB sb = seg_block(L);
  if (sb.x >= sb.gx) return;
  const int bx = sb.x, gx = sb.gx;  // workgroup index and count within the segment
  (void)gx;
  const k_eca_next_args<T, C, SKIP>& a_ = L.a[sb.s];
  const T* __restrict__ const Y = a_.Y;
  const T* __restrict__ const skip = a_.skip;
  T* __restrict__ const Xn = a_.Xn;
  const float* __restrict__ const gap = a_.gap;
  const float* __restrict__ const weca = a_.weca;
  float* __restrict__ const g_out = a_.g_out;
  float* __restrict__ const a_out = a_.a_out;
  const int hw = a_.hw;
  const int gap_tiles = a_.gap_tiles;
  const int tiles = a_.tiles;
  constexpr int G = C / 4;
  __shared__ float g_s[C], a_s[C];
  const int b = bx / tiles, tx = bx - b * tiles;  // clip, tile of the clip
  eca_scale_clip<C>(gap + (int64_t)b * gap_tiles * C, gap_tiles, hw, weca, g_s, a_s);
  if (tx == 0)
    for (int c = threadIdx.x; c < C; c += STDA_BLOCK) {
      g_out[b * C + c] = g_s[c];
      a_out[b * C + c] = a_s[c];
    }
  const int64_t items = (int64_t)hw * G;
  const int64_t base = (int64_t)b * hw * C;
  int64_t i = (int64_t)tx * STDA_BLOCK + threadIdx.x;
  const int c0 = (int)(i % G) * 4;
  for (; i < items; i += (int64_t)tiles * STDA_BLOCK) {
    const int64_t off = base + (i / G) * C + c0;
    float y[4], o[4];
    ld4(Y + off, y);
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = a_s[c0 + j] * y[j];
    if (SKIP) {
      float s[4];
      ld4(skip + off, s);
#pragma unroll
      for (int j = 0; j < 4; ++j) o[j] += s[j];
    }
    st4(Xn + off, o);
  }
}

// --------------------------------------------------------------------- loss
// d = z - y (in FP64); dz = 2 d / n; per-block FP64 partial of d^2 / n.
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ z, const float* __restrict__ y,
                                             float* __restrict__ dz, double* __restrict__ part, int64_t n) {
  __shared__ double sm[STDA_BLOCK];
  double acc = 0.0;
  const double inv = 1.0 / (double)n;
  for (int64_t i = (int64_t)blockIdx.x * STDA_BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * STDA_BLOCK) {
    const double d = (double)z[i] - (double)y[i];  // exact difference of two FP32 values
    dz[i] = (float)(2.0 * d * inv);
    acc += d * d * inv;
  }
  sm[threadIdx.x] = acc;
  __syncthreads();
  for (int s = STDA_BLOCK / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__global__ void k_sum_f64(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double sm[STDA_BLOCK];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += STDA_BLOCK) acc += part[i];
  sm[threadIdx.x] = acc;
  __syncthreads();
  for (int s = STDA_BLOCK / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sm[0];
}

// SINR (Sec. V-B) of one map per block: 10 log10(mean_O m^2 / mean_N m^2), FP64 sums.
__global__ __launch_bounds__(256) void k_sinr(const float* __restrict__ maps, const uint8_t* __restrict__ om,
                                              const uint8_t* __restrict__ nm, int64_t hw, double* __restrict__ out) {
  __shared__ double s[4][STDA_BLOCK];
  const int64_t base = (int64_t)blockIdx.x * hw;
  double so = 0.0, no = 0.0, sn = 0.0, nn = 0.0;
  for (int64_t i = threadIdx.x; i < hw; i += STDA_BLOCK) {
    const double v = (double)maps[base + i];
    if (om[base + i]) { so += v * v; no += 1.0; }
    if (nm[base + i]) { sn += v * v; nn += 1.0; }
  }
  s[0][threadIdx.x] = so;
  s[1][threadIdx.x] = no;
  s[2][threadIdx.x] = sn;
  s[3][threadIdx.x] = nn;
  __syncthreads();
  for (int k = STDA_BLOCK / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k)
      for (int q = 0; q < 4; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = 10.0 * log10((s[0][0] / s[1][0]) / (s[2][0] / s[3][0]));
}

}  // namespace stda
