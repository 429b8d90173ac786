// Output module (Conv3x3 p1, 16 -> 1, plus bias) and its adjoint on LDS tiles (gfx950).
//
// Forward: a block stages the 16-channel input of a TH x TW pixel tile plus a 1-pixel halo
// (zeros off the map) and each thread forms one output pixel from the staged neighbourhood.
// Adjoint: a block stages dz of the tile plus halo; thread items are (pixel, group of 4
// channels) and compute dd[c](p) = sum_t dz(p - off_t) w[c][t] and accumulate the weight
// gradient sum_p d[c](p) dz(p - off_t) (tap t = (ky, kx), off_t = (ky - 1, kx - 1)) and the bias
// gradient sum_p dz(p); part[blk][10][16] holds the taps (rows 0..8) and the bias (row 9,
// channel 0).  The grid loops over the tiles of all clips.
// SIG: logistic output z = 1 / (1 + exp(-(conv + b))); the forward also writes z to zs (when
// not null) and the adjoint stages dz * z (1 - z) from that copy in place of dz.
#pragma once
#include "stage1_tile.h"

namespace stda {

constexpr int kHeadTH = 8, kHeadTW = 32;

template <class T, bool SIG>
struct k_head_fwd_tile_args {
  const T* d;
  const float* w;
  const float* bias;
  float* z;
  float* zs;
  int B;
  int H;
  int W;
};
template <class T, bool SIG>
__global__ __launch_bounds__(256) void k_head_fwd_tile(SegL<k_head_fwd_tile_args<T, SIG>> L) {
  const SegB sb = seg_block(L);
  if (sb.x >= sb.gx) return;
  const int bx = sb.x, gx = sb.gx;  // workgroup index and count within the segment
  (void)gx;
  const k_head_fwd_tile_args<T, SIG>& a_ = L.a[sb.s];
  const T* __restrict__ const d = a_.d;
  const float* __restrict__ const w = a_.w;
  const float* __restrict__ const bias = a_.bias;
  float* __restrict__ const z = a_.z;
  float* __restrict__ const zs = a_.zs;
  const int B = a_.B;
  const int H = a_.H;
  const int W = a_.W;
  constexpr int TH = kHeadTH, TW = kHeadTW, C = 16, RW = TW + 2, XN = (TH + 2) * RW;
  __shared__ float xt[S1Lds<C, XN>::SIZE];
  __shared__ float wt[9 * C];  // [tap][c]
  // BF16 (DMAB): the next tile's input is fetched in storage form by buffer loads into an LDS
  // staging buffer as soon as this tile's is converted, in flight during this tile's outputs
  constexpr bool DMAB = sizeof(T) == 2;
  constexpr int SPPI = 64 * 16 / (C * (int)sizeof(T));                // pixels per staging load
  constexpr int XSL = (XN + 4 * SPPI - 1) / (4 * SPPI) * (4 * SPPI);  // staged pixels (whole loads in every wave)
  __shared__ uint32_t xst[DMAB ? XSL * C * sizeof(T) / 4 : 1];
  for (int q = threadIdx.x; q < 9 * C; q += STDA_BLOCK) wt[q] = w[(q % C) * 9 + q / C];
  const float b0 = bias[0];
  const int ntiles = B * ((H + TH - 1) / TH) * ((W + TW - 1) / TW);
  if constexpr (DMAB)
    if (bx < ntiles) {
      int b, y0, x0;
      tile_coords(bx, H, W, TH, TW, b, y0, x0);
      load_tile_dma_raw<T, C, TH, TW, 1, XSL>(d, b, y0, x0, H, W, xst);
    }
  for (int tile = bx; tile < ntiles; tile += gx) {
    int b, y0, x0;
    tile_coords(tile, H, W, TH, TW, b, y0, x0);
    if constexpr (DMAB) {
      wait_vmem();      // this wave's part of the staged tile is in LDS
      __syncthreads();  // every wave's, and the previous tile's outputs have read xt
      stage1_put_raw<T, C, XN, XN>(xst, xt);
      __syncthreads();
      int nb, ny0, nx0;  // the next tile (after the last tile this tile again, never read)
      tile_coords(tile + gx < ntiles ? tile + gx : tile, H, W, TH, TW, nb, ny0, nx0);
      load_tile_dma_raw<T, C, TH, TW, 1, XSL>(d, nb, ny0, nx0, H, W, xst);
    } else {
      __syncthreads();
      load_tile<T, C, TH, TW, 1>(d, b, y0, x0, H, W, xt);
      __syncthreads();
    }
    const int r = threadIdx.x / TW, cc = threadIdx.x % TW;  // one pixel per thread
    const int y = y0 + r, x = x0 + cc;
    if (y < H && x < W) {
      float acc = b0;
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const int px = (r + t / 3) * RW + cc + t % 3;
#pragma unroll
        for (int c = 0; c < C; c += 4) {
          const float4 v = *reinterpret_cast<const float4*>(xt + s1c<C, XN>(px, c >> 2));
          acc += wt[t * C + c] * v.x + wt[t * C + c + 1] * v.y + wt[t * C + c + 2] * v.z + wt[t * C + c + 3] * v.w;
        }
      }
      const int64_t o = ((int64_t)b * H + y) * W + x;
      if constexpr (SIG) {
        acc = 1.f / (1.f + expf(-acc));
        if (zs) zs[o] = acc;
      }
      z[o] = acc;
    }
  }
  if constexpr (DMAB) wait_vmem();  // the last (unused) fetch has landed
}

template <class T, bool SIG>
struct k_head_bwd_tile_args {
  const float* dz;
  const float* zs;
  const float* w;
  const T* d;
  T* dd;
  float* part;
  int B;
  int H;
  int W;
};
template <class T, bool SIG>
__global__ __launch_bounds__(256) void k_head_bwd_tile(SegL<k_head_bwd_tile_args<T, SIG>> L) {
  const SegB sb = seg_block(L);
  if (sb.x >= sb.gx) return;
  const int bx = sb.x, gx = sb.gx;  // workgroup index and count within the segment
  (void)gx;
  const k_head_bwd_tile_args<T, SIG>& a_ = L.a[sb.s];
  const float* __restrict__ const dz = a_.dz;
  const float* __restrict__ const zs = a_.zs;
  const float* __restrict__ const w = a_.w;
  const T* __restrict__ const d = a_.d;
  T* __restrict__ const dd = a_.dd;
  float* __restrict__ const part = a_.part;
  const int B = a_.B;
  const int H = a_.H;
  const int W = a_.W;
  constexpr int TH = kHeadTH, TW = kHeadTW, C = 16, G = 4, RW = TW + 2;
  static_assert(TH * TW == STDA_BLOCK, "one pixel per thread and channel group pass");
  __shared__ float zt[(TH + 2) * RW];
  __shared__ float sm[4 * 10 * C];
  __shared__ float red[10 * C];
  const int c0 = (threadIdx.x % G) * 4;
  float wr[9][4];
#pragma unroll
  for (int t = 0; t < 9; ++t)
#pragma unroll
    for (int j = 0; j < 4; ++j) wr[t][j] = w[(c0 + j) * 9 + t];
  float acc[10][4];
#pragma unroll
  for (int t = 0; t < 10; ++t) zero4(acc[t]);
  const int ntiles = B * ((H + TH - 1) / TH) * ((W + TW - 1) / TW);
  for (int tile = bx; tile < ntiles; tile += gx) {
    int b, y0, x0;
    tile_coords(tile, H, W, TH, TW, b, y0, x0);
    // the thread's G items' d, loaded before dz is staged so that their latencies overlap it and
    // each other (held in storage form until used)
    typename Raw4<T>::type dr[G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int px = (threadIdx.x + k * STDA_BLOCK) / G, y = y0 + px / TW, x = x0 + px % TW;
      if (y < H && x < W)
        raw_ld4(d + (((int64_t)b * H + y) * W + x) * C + c0, dr[k]);
      else
        raw_zero4(dr[k]);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < (TH + 2) * RW; q += STDA_BLOCK) {
      const int y = y0 - 1 + q / RW, x = x0 - 1 + q % RW;
      float g = 0.f;
      if (y >= 0 && y < H && x >= 0 && x < W) {
        const int64_t o = ((int64_t)b * H + y) * W + x;
        g = dz[o];
        if constexpr (SIG) g *= zs[o] * (1.f - zs[o]);
      }
      zt[q] = g;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int e = threadIdx.x + k * STDA_BLOCK;
      const int px = e / G, r = px / TW, cc = px % TW;
      const int y = y0 + r, x = x0 + cc;
      if (y >= H || x >= W) continue;
      const int64_t off = (((int64_t)b * H + y) * W + x) * C + c0;
      float dv[4], o[4];
      raw_cvt4(dr[k], dv);
      zero4(o);
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        // dz at p - off_t = (y - ky + 1, x - kx + 1): tile position (r + 2 - ky, cc + 2 - kx)
        const float g = zt[(r + 2 - t / 3) * RW + cc + 2 - t % 3];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          o[j] += wr[t][j] * g;
          acc[t][j] += dv[j] * g;
        }
      }
      if (c0 == 0) acc[9][0] += zt[(r + 1) * RW + cc + 1];
      st4(dd + off, o);
    }
  }
  block_chan_reduce_shfl<G, 10>(acc, sm, red);
  for (int q = threadIdx.x; q < 10 * C; q += STDA_BLOCK) part[(int64_t)bx * 10 * C + q] = red[q];
}

}  // namespace stda
