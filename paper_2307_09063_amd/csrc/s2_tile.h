// Dense stride-2 layers of the mobile blocks (stage 2: Conv3x3-s2 in the encoder, DeConv4x4-s2 in
// the decoder, and the input gradients of both) as an LDS-tiled implicit GEMM on the matrix cores.
//
//   out[p][n] = sum over the taps t valid for p and channels k of  src(p, t)[k] * W[t][k][n]
//
// with the tap rules of OpGeo.  A workgroup owns a TH x TW tile of output pixels (all four
// sub-pixel phases of it for the up-sampling operators) and NB of the N output channels; it
//   1. copies its NB-column slice of the weights, already in MFMA fragment order, into LDS once;
//   2. per tile, copies the source rectangle the tile reads (tile plus halo, zeros off the map)
//      into LDS with 16-byte loads, channels innermost, rows padded against bank conflicts;
//   3. runs the GEMM: wave w takes row tiles w*R .. w*R+R-1 (16 output pixels each) of every
//      phase, all NB/16 column tiles, A fragments and B fragments both read from LDS;
//   4. writes the FP32 accumulators, rounded to the storage type, into an LDS staging tile that
//      aliases the source rectangle, and stores it with 16-byte writes, contiguous along a row;
//   5. optionally accumulates BN partial sums (sum, sum of squares) of the FP32 results.
// Tiles are handed out XCD by XCD: consecutive workgroup indices alternate over the 8 XCDs, so
// workgroup b walks the tiles of the contiguous range owned by XCD b % 8, which keeps the halo
// rows shared by neighbouring tiles inside one L2.
#pragma once
#include "dense_mfma.h"

namespace stda {

template <class T> struct S2Pad;
template <> struct S2Pad<float> { static constexpr int v = 4; };  // 16 bytes per padded row end
template <> struct S2Pad<bf16> { static constexpr int v = 8; };

template <class T, int OP, int K, int N, int NB, int TH, int TW>
struct S2Cfg {
  static constexpr int KS = OpGeo<OP>::KS;
  static constexpr bool DOWN = OpGeo<OP>::DOWN;
  static constexpr int ES = sizeof(T);
  static constexpr int SH = DOWN ? 2 * TH + KS - 2 : TH / 2 + (KS == 4 ? 2 : 1);  // source rows
  static constexpr int SW = DOWN ? 2 * TW + KS - 2 : TW / 2 + (KS == 4 ? 2 : 1);  // source columns
  static constexpr int SOFF = DOWN ? 1 : (KS == 4 ? 1 : 0);  // source origin: 2 y0 - 1 or y0 / 2 - SOFF
  static constexpr int KP = K + S2Pad<T>::v;                  // LDS row pitch of the source (elements)
  static constexpr int OP_ = NB + S2Pad<T>::v;                // LDS row pitch of the output staging
  static constexpr int PH = DOWN ? 1 : 4;                     // sub-pixel phases per tile
  static constexpr int PW = DOWN ? TW : TW / 2;               // width of one phase's pixel grid
  static constexpr int MT = (DOWN ? TH * TW : TH * TW / 4) / 16;  // 16-row tiles per phase
  static constexpr int R = MT / 4;                            // row tiles per wave per phase
  static constexpr int KC = K / 16, NT = N / 16, NTB = NB / 16;
  static constexpr int TAPS = KS * KS;
  static constexpr int SRC_ELEMS = SH * SW * KP;
  static constexpr int OUT_ELEMS = TH * TW * OP_;
  static constexpr int TILE_ELEMS = SRC_ELEMS > OUT_ELEMS ? SRC_ELEMS : OUT_ELEMS;
  static constexpr int W_ELEMS = TAPS * K * NB;
  static constexpr int LDS_BYTES = (TILE_ELEMS + W_ELEMS) * ES;
  static_assert(K % 16 == 0 && N % NB == 0 && NB % 16 == 0, "channel counts");
  static_assert(MT % 4 == 0 && R >= 1, "each wave needs whole row tiles of every phase");
  static_assert(DOWN || (TH % 2 == 0 && TW % 2 == 0), "up-sampling tiles cover whole phase pairs");
  static_assert(LDS_BYTES <= 160 * 1024, "LDS of one workgroup");
};

// Tile t of the spatial tiling -> clip and tile origin.
__device__ __forceinline__ void s2_tile_origin(int64_t t, int nty, int ntx, int TH, int TW, int& b, int& y0, int& x0) {
  const int64_t per = (int64_t)nty * ntx;
  b = (int)(t / per);
  const int r = (int)(t - (int64_t)b * per);
  y0 = (r / ntx) * TH;
  x0 = (r % ntx) * TW;
}

template <class T, int OP, int K, int N, int NB, int TH, int TW, bool STATS>
__global__ __launch_bounds__(256) void k_s2_tile(const T* __restrict__ src, const T* __restrict__ wfrag,
                                                 T* __restrict__ dst, float* __restrict__ part, int B, int hd,
                                                 int wd) {
  typedef S2Cfg<T, OP, K, N, NB, TH, TW> C;
  typedef typename FragT<T>::type F;
  constexpr int KS = C::KS, KP = C::KP, SW = C::SW, SH = C::SH, R = C::R, NTB = C::NTB, KC = C::KC;
  constexpr int PH = C::PH, PW = C::PW;
  constexpr int VE = 16 / C::ES;  // elements per 16-byte vector
  __shared__ __attribute__((aligned(16))) T lds[C::TILE_ELEMS + C::W_ELEMS];
  T* const tile_lds = lds;
  T* const w_lds = lds + C::TILE_ELEMS;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, m = lane & 15, g = lane >> 4;
  const int cb = blockIdx.y;  // column block
  const int hs = C::DOWN ? 2 * hd : hd / 2, ws = C::DOWN ? 2 * wd : wd / 2;

  // 1. weights of this column block: frag[(tap, s, nt)][lane] -> w_lds[(tap, s, ntb)][lane]
  {
    const F* wf = reinterpret_cast<const F*>(wfrag);
    F* wl = reinterpret_cast<F*>(w_lds);
    constexpr int UNITS = C::TAPS * KC * NTB * 64;
    for (int u = threadIdx.x; u < UNITS; u += STDA_BLOCK) {
      const int ln = u & 63, q = u >> 6;
      const int ntb = q % NTB, ts = q / NTB;  // ts = tap * KC + s
      wl[u] = wf[((int64_t)ts * C::NT + cb * NTB + ntb) * 64 + ln];
    }
  }

  float st1[NTB], st2[NTB];
#pragma unroll
  for (int j = 0; j < NTB; ++j) st1[j] = st2[j] = 0.f;

  const int nty = (hd + TH - 1) / TH, ntx = (wd + TW - 1) / TW;
  const int64_t ntiles = (int64_t)B * nty * ntx;
  // XCD-contiguous tile ranges (falls back to a plain stride when the grid is not a multiple of 8)
  int64_t t_begin, t_end, t_step;
  if ((gridDim.x & 7) == 0) {
    const int xcd = blockIdx.x & 7, l = blockIdx.x >> 3, per = gridDim.x >> 3;
    const int64_t chunk = (ntiles + 7) / 8;
    t_begin = xcd * chunk + l;
    t_end = (xcd + 1) * chunk < ntiles ? (xcd + 1) * chunk : ntiles;
    t_step = per;
  } else {
    t_begin = blockIdx.x;
    t_end = ntiles;
    t_step = gridDim.x;
  }

  for (int64_t t = t_begin; t < t_end; t += t_step) {
    int b, y0, x0;
    s2_tile_origin(t, nty, ntx, TH, TW, b, y0, x0);
    const int sy0 = C::DOWN ? 2 * y0 - 1 : y0 / 2 - C::SOFF;
    const int sx0 = C::DOWN ? 2 * x0 - 1 : x0 / 2 - C::SOFF;
    __syncthreads();  // previous tile's staging reads are done (and the weights are in LDS)
    // 2. source rectangle -> LDS
    {
      constexpr int CH = K / VE;  // 16-byte chunks per pixel
      constexpr int TOTAL = SH * SW * CH;
      constexpr int PER = (TOTAL + STDA_BLOCK - 1) / STDA_BLOCK;
      uint4 v[PER];
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = threadIdx.x + i * STDA_BLOCK;
        v[i] = make_uint4(0u, 0u, 0u, 0u);
        if (e < TOTAL) {
          const int c = e % CH, px = e / CH;
          const int sy = sy0 + px / SW, sx = sx0 + px % SW;
          if (sy >= 0 && sy < hs && sx >= 0 && sx < ws)
            v[i] = *reinterpret_cast<const uint4*>(src + (((int64_t)b * hs + sy) * ws + sx) * K + c * VE);
        }
      }
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int e = threadIdx.x + i * STDA_BLOCK;
        if (e < TOTAL) {
          const int c = e % CH, px = e / CH;
          *reinterpret_cast<uint4*>(tile_lds + px * KP + c * VE) = v[i];
        }
      }
    }
    __syncthreads();
    // 3. GEMM: every phase, R row tiles per wave, NTB column tiles
    floatx4 acc[PH][R][NTB];
#pragma unroll
    for (int ph = 0; ph < PH; ++ph) {
      const int py = C::DOWN ? 0 : ph >> 1, px = C::DOWN ? 0 : ph & 1;
      int ry[R], rx[R];  // this lane's GEMM row: phase-grid (or tile) coordinates
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int p = 16 * (wave * R + r) + m;
        ry[r] = p / PW;
        rx[r] = p % PW;
#pragma unroll
        for (int j = 0; j < NTB; ++j) acc[ph][r][j] = floatx4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int a = 0; a < (C::DOWN ? KS : 2); ++a) {
        const int ky = C::DOWN ? a : ((py + 1) & 1) + 2 * a;
        if (ky >= KS) continue;
        const int oy = C::DOWN ? ky : (py + 1 - ky) / 2 + C::SOFF;
#pragma unroll
        for (int cc = 0; cc < (C::DOWN ? KS : 2); ++cc) {
          const int kx = C::DOWN ? cc : ((px + 1) & 1) + 2 * cc;
          if (kx >= KS) continue;
          const int ox = C::DOWN ? kx : (px + 1 - kx) / 2 + C::SOFF;
          const int tap = ky * KS + kx;
          int base[R];
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const int ly = C::DOWN ? 2 * ry[r] + oy : ry[r] + oy;
            const int lx = C::DOWN ? 2 * rx[r] + ox : rx[r] + ox;
            base[r] = (ly * SW + lx) * KP + 4 * g;
          }
          const F* wl = reinterpret_cast<const F*>(w_lds) + (tap * KC * NTB) * 64 + lane;
#pragma unroll
          for (int s = 0; s < KC; ++s) {
            F av[R];
#pragma unroll
            for (int r = 0; r < R; ++r) av[r] = *reinterpret_cast<const F*>(tile_lds + base[r] + 16 * s);
#pragma unroll
            for (int j = 0; j < NTB; ++j) {
              const F bv = wl[(s * NTB + j) * 64];
#pragma unroll
              for (int r = 0; r < R; ++r) acc[ph][r][j] = mfma_chunk(av[r], bv, acc[ph][r][j]);
            }
          }
        }
      }
    }
    __syncthreads();  // all waves are done reading the source rectangle
    // 4. accumulators -> LDS staging [pixel of the tile][NB]; lane holds rows 4g + i, column 16 j + m
#pragma unroll
    for (int ph = 0; ph < PH; ++ph) {
      const int py = C::DOWN ? 0 : ph >> 1, px = C::DOWN ? 0 : ph & 1;
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int p = 16 * (wave * R + r) + 4 * g + i;
          const int ty = C::DOWN ? p / PW : 2 * (p / PW) + py;
          const int tx = C::DOWN ? p % PW : 2 * (p % PW) + px;
          const bool valid = y0 + ty < hd && x0 + tx < wd;
#pragma unroll
          for (int j = 0; j < NTB; ++j) {
            const float v = acc[ph][r][j][i];
            tile_lds[(ty * TW + tx) * C::OP_ + 16 * j + m] = from_f<T>(v);
            if (STATS && valid) {
              st1[j] += v;
              st2[j] += v * v;
            }
          }
        }
    }
    __syncthreads();
    // 5. staging -> global, 16-byte vectors, contiguous along each tile row
    {
      constexpr int CH = NB / VE;
      constexpr int TOTAL = TH * TW * CH;
      for (int e = threadIdx.x; e < TOTAL; e += STDA_BLOCK) {
        const int c = e % CH, p = e / CH;
        const int ty = p / TW, tx = p % TW;
        const int y = y0 + ty, x = x0 + tx;
        if (y < hd && x < wd)
          *reinterpret_cast<uint4*>(dst + (((int64_t)b * hd + y) * wd + x) * N + cb * NB + c * VE) =
              *reinterpret_cast<const uint4*>(tile_lds + p * C::OP_ + c * VE);
      }
    }
  }
  if (STATS) {
    // part[blockIdx.x][n][2] (n = cb * NB + column): reduce over the 4 lane groups, then the 4
    // waves, in a fixed order
    __syncthreads();
    float* sm = reinterpret_cast<float*>(lds);  // 4 x 2 x NB floats, the tile is no longer needed
#pragma unroll
    for (int j = 0; j < NTB; ++j) {
      float a1 = st1[j], a2 = st2[j];
      a1 += __shfl_xor(a1, 16);
      a2 += __shfl_xor(a2, 16);
      a1 += __shfl_xor(a1, 32);
      a2 += __shfl_xor(a2, 32);
      if (g == 0) {
        sm[(wave * 2 + 0) * NB + 16 * j + m] = a1;
        sm[(wave * 2 + 1) * NB + 16 * j + m] = a2;
      }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 2 * NB; q += STDA_BLOCK) {
      const int c = q >> 1, s = q & 1;
      part[((int64_t)blockIdx.x * N + cb * NB + c) * 2 + s] =
          sm[(0 * 2 + s) * NB + c] + sm[(1 * 2 + s) * NB + c] + sm[(2 * 2 + s) * NB + c] + sm[(3 * 2 + s) * NB + c];
    }
  }
}

}  // namespace stda
