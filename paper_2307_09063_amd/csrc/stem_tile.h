// Input module (Conv3x3 p1, 3 -> 16 on the channel concatenation of frames t, t-1, t-2, then BN
// and ReLU) on LDS tiles (gfx950).
//
// A block stages the three planar input maps of a TH x TW pixel tile plus a 1-pixel halo in LDS;
// the convolution is an M x 16 x 28 GEMM (M = tile pixels, k = c*9 + tap, k = 27 zero) on the
// matrix cores, reading the im2col operand straight from the staged planes.  The pre-BN output
// is never stored: every pass recomputes it.
//   MODE 0  TRAIN statistics: part[blk][16][2] = (sum, sum of squares) of the conv output
//   MODE 1  s0 = ReLU(BN(conv)) with the given statistics
//   MODE 2  adjoint statistics: dM = dS [S > 0]; part[blk][2][16] = sum dM, sum dM * that
//   MODE 3  adjoint apply: dTp = gamma invstd (dM - k0 - that k1); weight gradient
//           dW[o][k] = sum_p dTp[o](p) im2col(p, k) -> part[blk][27][16]; dTp written if wanted
#pragma once
#include "stage1_tile.h"

namespace stda {

struct StemArgs {
  const float* x;      // [B][3][H][W]
  const float* w;      // [16][27]
  const float* stats;  // [mean 16][invstd 16]
  const float* gamma;
  const float* beta;
  const float* coef;   // MODE 3: [k0 16][k1 16]
  float* part;
};

template <class T, int MODE>
__global__ __launch_bounds__(256) void k_stem_tile(StemArgs a, const T* __restrict__ dS, const T* __restrict__ S,
                                                   T* __restrict__ out, int B, int H, int W) {
  constexpr int TH = 8, TW = 32, M = TH * TW, C = 16, G = 4, PS = C + 4, XR = TH + 2, XC = TW + 2;
  __shared__ float xs[3 * XR * XC];
  __shared__ float wk[C * 28];
  __shared__ float tt[M * PS];   // conv output of the tile (then dTp in MODE 3)
  __shared__ float sm[4 * 2 * C];
  __shared__ float red[2 * C];
  for (int q = threadIdx.x; q < C * 28; q += STDA_BLOCK) {
    const int o = q / 28, kk = q % 28;
    wk[q] = kk < 27 ? a.w[o * 27 + kk] : 0.f;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, lg = lane >> 4;
  const int c0 = (threadIdx.x % G) * 4;
  float mu[4], is[4], sc[4], sh[4], k0[4], k1[4], ga[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (MODE >= 1) {
      mu[j] = a.stats[c0 + j];
      is[j] = a.stats[C + c0 + j];
      ga[j] = a.gamma[c0 + j];
    }
    if (MODE == 1) {
      sc[j] = ga[j] * is[j];
      sh[j] = a.beta[c0 + j] - mu[j] * sc[j];
    }
    if (MODE == 3) {
      k0[j] = a.coef[c0 + j];
      k1[j] = a.coef[C + c0 + j];
    }
  }
  float acc[2][4];
  zero4(acc[0]);
  zero4(acc[1]);
  floatx4_t wacc = {0.f, 0.f, 0.f, 0.f};  // MODE 3: waves 0, 1 own the 16 x 16 weight-gradient tiles
  auto im2col = [&](int p, int kk) -> float {
    if (kk >= 27) return 0.f;
    const int c = kk / 9, t = kk % 9;
    return xs[(c * XR + p / TW + t / 3) * XC + p % TW + t % 3];
  };
  const int ntiles = B * ((H + TH - 1) / TH) * ((W + TW - 1) / TW);
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    int b, y0, x0;
    tile_coords(tile, H, W, TH, TW, b, y0, x0);
    // adjoint modes: this thread's dS and S, loaded before the staging and the GEMM so that
    // their latency overlaps them
    constexpr int KI = (M * G + STDA_BLOCK - 1) / STDA_BLOCK;
    float pg[KI][4], ps[KI][4];
    if constexpr (MODE >= 2) {
#pragma unroll
      for (int k = 0; k < KI; ++k) {
        const int e = threadIdx.x + k * STDA_BLOCK;
        const int px = e / G, y = y0 + px / TW, x = x0 + px % TW;
        if (e < M * G && y < H && x < W) {
          const int64_t off = (((int64_t)b * H + y) * W + x) * C + c0;
          ld4(dS + off, pg[k]);
          ld4(S + off, ps[k]);
        } else {
          zero4(pg[k]);
          zero4(ps[k]);
        }
      }
    }
    __syncthreads();
    {
      // the three planes of the tile plus halo; all loads issued before the LDS writes
      constexpr int NX = 3 * XR * XC, KX = (NX + STDA_BLOCK - 1) / STDA_BLOCK;
      float xv[KX];
#pragma unroll
      for (int k = 0; k < KX; ++k) {
        const int q = threadIdx.x + k * STDA_BLOCK;
        const int c = q / (XR * XC), r = (q / XC) % XR, cc = q % XC;
        const int y = y0 - 1 + r, x = x0 - 1 + cc;
        xv[k] = (q < NX && y >= 0 && y < H && x >= 0 && x < W) ? a.x[(((int64_t)b * 3 + c) * H + y) * W + x] : 0.f;
      }
#pragma unroll
      for (int k = 0; k < KX; ++k) {
        const int q = threadIdx.x + k * STDA_BLOCK;
        if (q < NX) xs[q] = xv[k];
      }
    }
    __syncthreads();
    lds_gemm<M, C, 28>(im2col, [&](int kk, int n) { return wk[n * 28 + kk]; }, tt, PS);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KI; ++k) {
      const int e = threadIdx.x + k * STDA_BLOCK;
      if (e >= M * G) break;
      const int px = e / G, y = y0 + px / TW, x = x0 + px % TW;
      const bool in = y < H && x < W;
      const float4 tq = *reinterpret_cast<const float4*>(tt + px * PS + c0);
      const float t[4] = {tq.x, tq.y, tq.z, tq.w};
      const int64_t off = (((int64_t)b * H + y) * W + x) * C + c0;
      if (MODE == 0) {
        if (!in) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[0][j] += t[j];
          acc[1][j] += t[j] * t[j];
        }
      } else if (MODE == 1) {
        if (!in) continue;
        float o[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) o[j] = fmaxf(t[j] * sc[j] + sh[j], 0.f);
        st4(out + off, o);
      } else {
        const float* g = pg[k];
        const float* s = ps[k];
        float o[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float dm = s[j] > 0.f ? g[j] : 0.f;
          const float th = (t[j] - mu[j]) * is[j];
          if (MODE == 2) {
            acc[0][j] += dm;
            acc[1][j] += dm * th;
          } else {
            o[j] = in ? ga[j] * is[j] * (dm - k0[j] - th * k1[j]) : 0.f;
          }
        }
        if (MODE == 3) {  // each (pixel, group) slot of tt is read and rewritten by one thread only
          *reinterpret_cast<float4*>(tt + px * PS + c0) = make_float4(o[0], o[1], o[2], o[3]);
          if (out && in) st4(out + off, o);
        }
      }
    }
    if (MODE == 3) {
      __syncthreads();
      // dW[o][k] += sum_p dTp[p][o] im2col(p, k): tile (o 0..15) x (k 0..15 | 16..31)
      if (wave < 2) {
        const int n0 = 16 * wave;
#pragma unroll 4
        for (int p = 0; p < M; p += 4)
          wacc = __builtin_amdgcn_mfma_f32_16x16x4f32(tt[(p + lg) * PS + li], im2col(p + lg, n0 + li), wacc, 0, 0, 0);
      }
    }
  }
  if (MODE == 0 || MODE == 2) {
    block_chan_reduce_shfl<G, 2>(acc, sm, red);
    for (int q = threadIdx.x; q < 2 * C; q += STDA_BLOCK) {
      // MODE 0: [16][2] (sum, sumsq per channel); MODE 2: [2][16]
      const int s = q / C, c = q % C;
      a.part[(int64_t)blockIdx.x * 2 * C + (MODE == 0 ? c * 2 + s : q)] = red[q];
    }
  }
  if (MODE == 3 && wave < 2) {
    // lane holds D[4 lg + r][li] = dW[o = 4 lg + r][k = 16 wave + li]
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = 4 * lg + r, kk = 16 * wave + li;
      if (kk < 27) a.part[(int64_t)blockIdx.x * 27 * C + kk * C + o] = wacc[r];
    }
  }
}

}  // namespace stda
