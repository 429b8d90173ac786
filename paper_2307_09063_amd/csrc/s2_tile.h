// Dense stride-2 layers of the mobile blocks (stage 2: Conv3x3-s2 in the encoder, DeConv4x4-s2 in
// the decoder, and the input gradients of both) as an LDS-tiled implicit GEMM on the matrix cores.
//
//   out[p][n] = sum over the taps t valid for p and channels k of  src(p, t)[k] * W[t][k][n]
//
// with the tap rules of OpGeo.  A workgroup owns a TH x TW tile of output pixels (all four
// sub-pixel phases of it for the up-sampling operators) and NB of the N output channels; it
//   1. copies its NB-column slice of the weights, already in MFMA fragment order, into LDS once;
//   2. per tile, copies the source rectangle the tile reads (tile plus halo, zeros off the map)
//      into LDS with 16-byte loads, channels innermost, rows padded against bank conflicts; the
//      next tile's rectangle is loaded into registers while this tile's GEMM runs;
//   3. runs the GEMM (4 or 8 waves per workgroup; 8 where the LDS allows one workgroup per CU, so
//      that two waves share each SIMD): wave w takes row tiles w*R .. w*R+R-1 (16 output pixels each) of every
//      phase, all NB/16 column tiles, A fragments and B fragments both read from LDS (BF16 with 32 or
//      more input channels: two 16-channel chunks per gfx950 v_mfma_f32_16x16x32_bf16);
//   4. writes the FP32 accumulators, rounded to the storage type, into an LDS staging tile that
//      aliases the source rectangle, and stores it with 16-byte writes, contiguous along a row;
//   5. optionally accumulates the BN statistics (count, mean, m2) of the FP32 results.
// Tiles are handed out XCD by XCD: consecutive workgroup indices alternate over the 8 XCDs, so
// workgroup b walks the tiles of the contiguous range owned by XCD b % 8, which keeps the halo
// rows shared by neighbouring tiles inside one L2.
#pragma once
#include "dense_mfma.h"

namespace stda {

template <class T> struct S2Pad;
template <> struct S2Pad<float> { static constexpr int v = 4; };  // 16 bytes per padded row end
template <> struct S2Pad<bf16> { static constexpr int v = 8; };

template <class T, int OP, int K, int N, int NB, int TH, int TW, int WV = 4>
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
  static constexpr int R = MT / WV;                           // row tiles per wave per phase
  static constexpr int BLK = 64 * WV;                         // threads per workgroup
  static constexpr int KC = K / 16, NT = N / 16, NTB = NB / 16;
  static constexpr int TAPS = KS * KS;
  static constexpr int SRC_ELEMS = SH * SW * KP;
  static constexpr int OUT_ELEMS = TH * TW * OP_;
  static constexpr int TILE_ELEMS = SRC_ELEMS > OUT_ELEMS ? SRC_ELEMS : OUT_ELEMS;
  static constexpr int W_ELEMS = TAPS * K * NB;
  static constexpr int LDS_BYTES = (TILE_ELEMS + W_ELEMS) * ES;
  static_assert(K % 16 == 0 && N % NB == 0 && NB % 16 == 0, "channel counts");
  static_assert(MT % WV == 0 && R >= 1, "each wave needs whole row tiles of every phase");
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

template <class T, int OP, int K, int N, int NB, int TH, int TW, bool STATS, int WV = 4>
struct k_s2_tile_args {
  const T* src;
  const T* wfrag;
  T* dst;
  float* part;
  int B;
  int hd;
  int wd;
};
template <class T, int OP, int K, int N, int NB, int TH, int TW, bool STATS, int WV = 4>
__global__ __launch_bounds__(64 * WV) void k_s2_tile(SegL<k_s2_tile_args<T, OP, K, N, NB, TH, TW, STATS, WV>> L) {
  const SegB sb = seg_block(L);
  if (sb.x >= sb.gx) return;
  const int bx = sb.x, gx = sb.gx;  // workgroup index and count within the segment
  (void)gx;
  const k_s2_tile_args<T, OP, K, N, NB, TH, TW, STATS, WV>& a_ = L.a[sb.s];
  const T* __restrict__ const src = a_.src;
  const T* __restrict__ const wfrag = a_.wfrag;
  T* __restrict__ const dst = a_.dst;
  float* __restrict__ const part = a_.part;
  const int B = a_.B;
  const int hd = a_.hd;
  const int wd = a_.wd;
  typedef S2Cfg<T, OP, K, N, NB, TH, TW, WV> C;
  constexpr int BLK = C::BLK;
  typedef typename FragT<T>::type F;
  constexpr int KS = C::KS, KP = C::KP, SW = C::SW, SH = C::SH, R = C::R, NTB = C::NTB, KC = C::KC;
  constexpr bool PAIR2 = sizeof(T) == 2 && KC % 2 == 0;  // BF16 on the 16x16x32 instruction
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
    for (int u = threadIdx.x; u < UNITS; u += BLK) {
      const int ln = u & 63, q = u >> 6;
      const int ntb = q % NTB, ts = q / NTB;  // ts = tap * KC + s
      wl[u] = wf[((int64_t)ts * C::NT + cb * NTB + ntb) * 64 + ln];
    }
  }

  float mn[NTB], q2[NTB];  // STATS: mean and m2 of this lane's columns 16 j + m (Welford)
#pragma unroll
  for (int j = 0; j < NTB; ++j) mn[j] = q2[j] = 0.f;
  float cnt = 0.f;  // rows seen by this lane

  const int nty = (hd + TH - 1) / TH, ntx = (wd + TW - 1) / TW;
  const int64_t ntiles = (int64_t)B * nty * ntx;
  // XCD-contiguous tile ranges (falls back to a plain stride when the grid is not a multiple of 8)
  int64_t t_begin, t_end, t_step;
  if ((gx & 7) == 0) {
    const int xcd = bx & 7, l = bx >> 3, per = gx >> 3;
    const int64_t chunk = (ntiles + 7) / 8;
    t_begin = xcd * chunk + l;
    t_end = (xcd + 1) * chunk < ntiles ? (xcd + 1) * chunk : ntiles;
    t_step = per;
  } else {
    t_begin = bx;
    t_end = ntiles;
    t_step = gx;
  }

  // 2. source rectangle of tile t, HBM -> registers; the next tile's is loaded while this tile's
  // GEMM runs (software pipelining: the loads stay in flight across the LDS-only barriers)
  constexpr int CH = K / VE;  // 16-byte chunks per pixel
  constexpr int TOTAL = SH * SW * CH;
  constexpr int PER = (TOTAL + BLK - 1) / BLK;
  uint4 v[PER];
  auto load_src = [&](int64_t tt) {
    int lb, ly0, lx0;
    s2_tile_origin(tt, nty, ntx, TH, TW, lb, ly0, lx0);
    const int sy0 = C::DOWN ? 2 * ly0 - 1 : ly0 / 2 - C::SOFF;
    const int sx0 = C::DOWN ? 2 * lx0 - 1 : lx0 / 2 - C::SOFF;
    // buffer loads over the clip, reading 0 off the map and past the rectangle: no branch around
    // them, so every thread issues the same loads (and the stores after them are counted exactly)
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<T*>(src + (int64_t)lb * hs * ws * K), (short)0, hs * ws * K * (int)sizeof(T), 0x00020000);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + i * BLK;
      const int c = e % CH, px = e / CH;
      const int sy = sy0 + px / SW, sx = sx0 + px % SW;
      const bool ok = e < TOTAL && sy >= 0 && sy < hs && sx >= 0 && sx < ws;
      const u32x4_t q = __builtin_amdgcn_raw_buffer_load_b128(rs, ok ? ((sy * ws + sx) * K + c * VE) * (int)sizeof(T)
                                                                     : (int)0x80000000u, 0, 0);
      v[i] = make_uint4(q.x, q.y, q.z, q.w);
    }
  };
  if (t_begin < t_end) load_src(t_begin);

  for (int64_t t = t_begin; t < t_end; t += t_step) {
    int b, y0, x0;
    s2_tile_origin(t, nty, ntx, TH, TW, b, y0, x0);
    __syncthreads();  // previous tile's staging reads are done (and the weights are in LDS)
    // registers -> LDS
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + i * BLK;
      if (e < TOTAL) {
        const int c = e % CH, px = e / CH;
        *reinterpret_cast<uint4*>(tile_lds + px * KP + c * VE) = v[i];
      }
    }
    __syncthreads();
    if (t + t_step < t_end) load_src(t + t_step);
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
          if constexpr (PAIR2) {
            // BF16, K a multiple of 32: chunks s and s + 1 feed one 16x16x32 product
#pragma unroll
            for (int s = 0; s < KC; s += 2) {
              bf16x8 av[R];
#pragma unroll
              for (int r = 0; r < R; ++r)
                av[r] = pack8(*reinterpret_cast<const F*>(tile_lds + base[r] + 16 * s),
                              *reinterpret_cast<const F*>(tile_lds + base[r] + 16 * s + 16));
#pragma unroll
              for (int j = 0; j < NTB; ++j) {
                const bf16x8 bv = pack8(wl[(s * NTB + j) * 64], wl[((s + 1) * NTB + j) * 64]);
#pragma unroll
                for (int r = 0; r < R; ++r)
                  acc[ph][r][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[r], bv, acc[ph][r][j], 0, 0, 0);
              }
            }
          } else {
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
          float rk = 0.f;
          if (STATS && valid) {
            cnt += 1.f;
            rk = __builtin_amdgcn_rcpf(cnt);
          }
#pragma unroll
          for (int j = 0; j < NTB; ++j) {
            const float v = acc[ph][r][j][i];
            tile_lds[(ty * TW + tx) * C::OP_ + 16 * j + m] = from_f<T>(v);
            if (STATS && valid) wf_add(mn[j], q2[j], v, rk);
          }
        }
    }
    __syncthreads();
    // 5. staging -> global, 16-byte vectors, contiguous along each tile row.  Buffer stores over
    // this clip's output, an offset past its range (off the map or past the tile) dropping the
    // store: no branch around them, so every thread issues the same stores and the next tile's
    // wait for its source loads (issued before these) need not wait for these stores.  A clip's
    // output is at most 1 GiB here (4096 x 4096 pixels of 16 FP32 channels at full resolution).
    {
      constexpr int CH = NB / VE;
      constexpr int TOTAL = TH * TW * CH, NSI = (TOTAL + BLK - 1) / BLK;
      const __amdgpu_buffer_rsrc_t rd = __builtin_amdgcn_make_buffer_rsrc(
          dst + (int64_t)b * hd * wd * N, (short)0, hd * wd * N * (int)sizeof(T), 0x00020000);
#pragma unroll
      for (int k = 0; k < NSI; ++k) {
        const int e = threadIdx.x + k * BLK, ec = e < TOTAL ? e : TOTAL - 1;
        const int c = ec % CH, p = ec / CH;
        const int ty = p / TW, tx = p % TW;
        const int y = y0 + ty, x = x0 + tx;
        const bool ok = e < TOTAL && y < hd && x < wd;
        const uint4 q = *reinterpret_cast<const uint4*>(tile_lds + p * C::OP_ + c * VE);
        __builtin_amdgcn_raw_buffer_store_b128(u32x4_t{q.x, q.y, q.z, q.w}, rd,
                                               ok ? ((y * wd + x) * N + cb * NB + c * VE) * (int)sizeof(T)
                                                  : (int)0x80000000u,
                                               0, 0);
      }
    }
  }
  if (STATS) {
    // part[bx][n][2] = (mean, m2) (n = cb * NB + column), the block's count at
    // part[gx * 2 N + bx]: merge over the 4 lane groups, then the WV waves, in a
    // fixed order
    constexpr int ROW = 2 * NB + 1;
    static_assert(WV * ROW * 4 <= (int)sizeof(lds), "statistics scratch fits the tile buffer");
    __syncthreads();
    float* sm = reinterpret_cast<float*>(lds);  // WV x ROW floats, the tile is no longer needed
#pragma unroll
    for (int off = 16; off < 64; off <<= 1) {
      const float nb = __shfl_xor(cnt, off);
#pragma unroll
      for (int j = 0; j < NTB; ++j) {
        const float mb = __shfl_xor(mn[j], off), qb = __shfl_xor(q2[j], off);
        chan_merge(cnt, mn[j], q2[j], nb, mb, qb);
      }
      cnt += nb;
    }
    if (g == 0) {
#pragma unroll
      for (int j = 0; j < NTB; ++j) {
        sm[wave * ROW + 16 * j + m] = mn[j];
        sm[wave * ROW + NB + 16 * j + m] = q2[j];
      }
      if (m == 0) sm[wave * ROW + 2 * NB] = cnt;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < NB; c += BLK) {
      float na = sm[2 * NB], ma = sm[c], qa = sm[NB + c];
#pragma unroll
      for (int wv = 1; wv < WV; ++wv) {
        const float nb = sm[wv * ROW + 2 * NB];
        chan_merge(na, ma, qa, nb, sm[wv * ROW + c], sm[wv * ROW + NB + c]);
        na += nb;
      }
      part[((int64_t)bx * N + cb * NB + c) * 2] = ma;
      part[((int64_t)bx * N + cb * NB + c) * 2 + 1] = qa;
      if (cb == 0 && c == 0) part[(int64_t)gx * 2 * N + bx] = na;
    }
  }
}

}  // namespace stda

namespace stda {

// Weight gradients of the stage-2 dense layers on LDS tiles.
//
//   R[tap][ch][cl] = sum over low-resolution pixels (b, y, x) of
//                    Hi(b, 2y - 1 + ky, 2x - 1 + kx)[ch] * Lo(b, y, x)[cl],   tap = ky * KS + kx
//
// Conv3x3-s2 (encoder): Lo = output gradient (cl = o), Hi = layer input (ch = c), KS = 3.
// DeConv4x4-s2 (decoder): Lo = layer input (cl = c), Hi = output gradient (ch = o), KS = 4.
// A workgroup walks TH x TW low-resolution tiles (XCD-contiguous ranges, as the forward does) and
// stages, as FP32, Lo transposed to [cl][pixel] and the Hi rectangle of the tile split into its
// four parity planes [py][px][ch][Y][X], so that tap (ky, kx) reads plane (ky & 1, kx & 1) at
// (y + ky / 2, x + kx / 2): a unit-stride window.  The reduction over pixels is the MFMA's inner
// dimension: lane group g takes 4 consecutive pixels of a row (one 16-byte read of Lo; the Hi
// window is read as 4 scalars since the tap shift breaks 16-byte alignment).  FP32:
// v_mfma_f32_16x16x4f32, the 4 pixels feeding 4 MFMAs; BF16: v_mfma_f32_16x16x16bf16_1k with
// lane group g supplying pixels 4g .. 4g + 3 of 16 (values are BF16-exact, so truncating the
// staged FP32 packs them exactly).  Wave w owns the (tap, 16-channel ch tile) pairs w, w + 4, ...
// with all cl tiles, accumulating across its tiles; the result is written once per workgroup as
// part[blk][k * NCOL + n] in the layout of the weight's column map (encoder: k = tap * CH + ch,
// n = cl; decoder: k = cl, n = tap * CH + ch), reduced across workgroups afterwards in FP64.
template <class T, bool DEC, int CL, int CH, int TH, int TW>
struct WgCfg {
  static constexpr int KS = DEC ? 4 : 3, TAPS = KS * KS;
  static constexpr int SH = 2 * TH + KS - 2, SW = 2 * TW + KS - 2;  // Hi rectangle
  static constexpr int PY = TH + 1, PX = TW + 1;                    // parity-plane extent
  static constexpr int PXP = PX + 3;                                // plane row pitch (floats)
  static constexpr int PLANE = CH * PY * PXP;
  static constexpr int LP = TH * TW + 4;                            // Lo row pitch (floats)
  static constexpr int MTC = CH / 16, NTC = CL / 16;
  static constexpr int PAIRS = TAPS * MTC, PW_ = (PAIRS + 3) / 4;   // (tap, ch tile) pairs per wave
  static constexpr int LDS_FLOATS = CL * LP + 4 * PLANE;
  static_assert(TW % 4 == 0 && (TH * TW) % 16 == 0, "pixel groups of 4 inside a row, chunks of 16");
  static_assert(LDS_FLOATS * 4 <= 160 * 1024, "LDS of one workgroup");
};

template <class T, bool DEC, int CL, int CH, int TH, int TW>
struct k_s2_wgrad_args {
  const T* lo;
  const T* hi;
  float* part;
  int B;
  int h;
  int w;
};
template <class T, bool DEC, int CL, int CH, int TH, int TW>
__global__ __launch_bounds__(256) void k_s2_wgrad(SegL<k_s2_wgrad_args<T, DEC, CL, CH, TH, TW>> L) {
  const SegB sb = seg_block(L);
  if (sb.x >= sb.gx) return;
  const int bx = sb.x, gx = sb.gx;  // workgroup index and count within the segment
  (void)gx;
  const k_s2_wgrad_args<T, DEC, CL, CH, TH, TW>& a_ = L.a[sb.s];
  const T* __restrict__ const lo = a_.lo;
  const T* __restrict__ const hi = a_.hi;
  float* __restrict__ const part = a_.part;
  const int B = a_.B;
  const int h = a_.h;
  const int w = a_.w;
  typedef WgCfg<T, DEC, CL, CH, TH, TW> C;
  constexpr int KS = C::KS, PW_ = C::PW_, NTC = C::NTC, MTC = C::MTC, LP = C::LP, PXP = C::PXP, PY = C::PY;
  constexpr bool BF = sizeof(T) == 2;
  constexpr int VE = 16 / sizeof(T);
  __shared__ __attribute__((aligned(16))) float lds[C::LDS_FLOATS];
  float* const ls = lds;              // [CL][LP]
  float* const hs = lds + CL * LP;    // [4][CH][PY][PXP]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, i = lane & 15, g = lane >> 4;
  const int H2 = 2 * h, W2 = 2 * w;

  floatx4 acc[PW_][NTC];
#pragma unroll
  for (int u = 0; u < PW_; ++u)
#pragma unroll
    for (int j = 0; j < NTC; ++j) acc[u][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int nty = (h + TH - 1) / TH, ntx = (w + TW - 1) / TW;
  const int64_t ntiles = (int64_t)B * nty * ntx;
  int64_t t_begin, t_end, t_step;
  if ((gx & 7) == 0) {
    const int xcd = bx & 7, l = bx >> 3, per = gx >> 3;
    const int64_t chunk = (ntiles + 7) / 8;
    t_begin = xcd * chunk + l;
    t_end = (xcd + 1) * chunk < ntiles ? (xcd + 1) * chunk : ntiles;
    t_step = per;
  } else {
    t_begin = bx;
    t_end = ntiles;
    t_step = gx;
  }
  for (int64_t t = t_begin; t < t_end; t += t_step) {
    int b, y0, x0;
    s2_tile_origin(t, nty, ntx, TH, TW, b, y0, x0);
    __syncthreads();
    // Lo tile -> ls[cl][p] (zeros off the map)
    {
      constexpr int CHV = CL / VE, TOTAL = TH * TW * CHV;
      for (int e = threadIdx.x; e < TOTAL; e += STDA_BLOCK) {
        const int cv = e % CHV, p = e / CHV;
        const int y = y0 + p / TW, x = x0 + p % TW;
        float v[VE];
        if (y < h && x < w) {
          const T* src = lo + (((int64_t)b * h + y) * w + x) * CL + cv * VE;
#pragma unroll
          for (int q = 0; q < VE; q += 4) ld4(src + q, v + q);
        } else {
#pragma unroll
          for (int q = 0; q < VE; ++q) v[q] = 0.f;
        }
#pragma unroll
        for (int q = 0; q < VE; ++q) ls[(cv * VE + q) * LP + p] = v[q];
      }
    }
    // Hi rectangle -> parity planes hs[(py * 2 + px)][ch][Y][X]
    {
      constexpr int CHV = CH / VE, TOTAL = C::SH * C::SW * CHV;
      for (int e = threadIdx.x; e < TOTAL; e += STDA_BLOCK) {
        const int cv = e % CHV, px_ = e / CHV;
        const int ly = px_ / C::SW, lx = px_ % C::SW;
        const int sy = 2 * y0 - 1 + ly, sx = 2 * x0 - 1 + lx;
        float v[VE];
        if (sy >= 0 && sy < H2 && sx >= 0 && sx < W2) {
          const T* src = hi + (((int64_t)b * H2 + sy) * W2 + sx) * CH + cv * VE;
#pragma unroll
          for (int q = 0; q < VE; q += 4) ld4(src + q, v + q);
        } else {
#pragma unroll
          for (int q = 0; q < VE; ++q) v[q] = 0.f;
        }
        float* dst = hs + ((ly & 1) * 2 + (lx & 1)) * C::PLANE + (ly >> 1) * PXP + (lx >> 1);
#pragma unroll
        for (int q = 0; q < VE; ++q) dst[(cv * VE + q) * PY * PXP] = v[q];
      }
    }
    __syncthreads();
#pragma unroll 1
    for (int c16 = 0; c16 < TH * TW / 16; ++c16) {
      const int p0 = 16 * c16 + 4 * g, ty = p0 / TW, tx = p0 % TW;
      float4 bq[NTC];
#pragma unroll
      for (int j = 0; j < NTC; ++j) bq[j] = *reinterpret_cast<const float4*>(ls + (16 * j + i) * LP + p0);
#pragma unroll
      for (int u = 0; u < PW_; ++u) {
        const int q = wave + 4 * u;
        if (q >= C::PAIRS) continue;
        const int tap = q / MTC, mt = q % MTC, ky = tap / KS, kx = tap % KS;
        const float* a = hs + ((ky & 1) * 2 + (kx & 1)) * C::PLANE + ((16 * mt + i) * PY + ty + (ky >> 1)) * PXP +
                         tx + (kx >> 1);
        const float a0 = a[0], a1 = a[1], a2 = a[2], a3 = a[3];
#pragma unroll
        for (int j = 0; j < NTC; ++j) {
          if constexpr (BF) {
            const shortx4 av = {(short)(__float_as_uint(a0) >> 16), (short)(__float_as_uint(a1) >> 16),
                                (short)(__float_as_uint(a2) >> 16), (short)(__float_as_uint(a3) >> 16)};
            const shortx4 bv = {(short)(__float_as_uint(bq[j].x) >> 16), (short)(__float_as_uint(bq[j].y) >> 16),
                                (short)(__float_as_uint(bq[j].z) >> 16), (short)(__float_as_uint(bq[j].w) >> 16)};
            acc[u][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[u][j], 0, 0, 0);
          } else {
            acc[u][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, bq[j].x, acc[u][j], 0, 0, 0);
            acc[u][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, bq[j].y, acc[u][j], 0, 0, 0);
            acc[u][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2, bq[j].z, acc[u][j], 0, 0, 0);
            acc[u][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a3, bq[j].w, acc[u][j], 0, 0, 0);
          }
        }
      }
    }
  }
  // lane (i, g) holds D[4g + r][i]: ch = 16 mt + 4g + r, cl = 16 j + i
  constexpr int NCOL = DEC ? C::TAPS * CH : CL;
  float* out = part + (int64_t)bx * C::TAPS * CH * CL;
#pragma unroll
  for (int u = 0; u < PW_; ++u) {
    const int q = wave + 4 * u;
    if (q >= C::PAIRS) continue;
    const int tap = q / MTC, mt = q % MTC;
#pragma unroll
    for (int j = 0; j < NTC; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ch = 16 * mt + 4 * g + r, cl = 16 * j + i;
        const int64_t idx = DEC ? (int64_t)cl * NCOL + tap * CH + ch : ((int64_t)tap * CH + ch) * NCOL + cl;
        out[idx] = acc[u][j][r];
      }
  }
}

}  // namespace stda

namespace stda {

// Weight gradients of the stage-2 dense layers, vector-operand form (same R and part layout as
// k_s2_wgrad).  LDS holds the operands in the storage type: Lo as [cl][pixel] and the Hi
// rectangle as parity planes [slot][ch][Y][X] where a slot is a plane (py, px) together with a
// column shift s in {0, 1} (slot content at X = plane value at X + s).  Tap (ky, kx) reads slot
// (ky & 1, kx & 1, kx >> 1) at (y + ky / 2, x): the 4 consecutive pixels a lane group feeds to
// the matrix core are one aligned 8-byte (BF16) or 16-byte (FP32) read for both operands.  The
// shifted copy exists only for the planes a tap with kx >> 1 = 1 reads (px = 0 when KS = 3).
// Staging: a thread takes 4 channels x 4 consecutive pixels, issues the 4 loads, transposes in
// registers and writes 4 aligned vectors.
template <class T>
struct WgVec;
template <>
struct WgVec<float> {
  typedef float4 type;
  typedef float elem;
};
template <>
struct WgVec<bf16> {
  typedef shortx4 type;
  typedef unsigned short elem;
};

template <class T, bool DEC, int CL, int CH, int TH, int TW>
struct WgVCfg {
  static constexpr int KS = DEC ? 4 : 3, TAPS = KS * KS;
  static constexpr int SH = 2 * TH + KS - 2, SW = 2 * TW + KS - 2;
  static constexpr int PY = TH + 1;
  static constexpr int CS = PY * TW + 4;         // channel stride of a slot (elements)
  static constexpr int SLOTS = KS == 3 ? 6 : 8;  // 4 planes unshifted + the shifted ones read
  static constexpr int LP = TH * TW + 4;         // Lo channel stride (elements)
  static constexpr int MTC = CH / 16, NTC = CL / 16;
  static constexpr int PAIRS = TAPS * MTC, PW_ = (PAIRS + 3) / 4;
  static constexpr int ELEMS = CL * LP + SLOTS * CH * CS;
  static constexpr int LDS_BYTES = ELEMS * (int)sizeof(T);
  static_assert(TW % 4 == 0 && (TH * TW) % 16 == 0, "pixel groups of 4 inside a row, chunks of 16");
  static_assert(CL % 4 == 0 && CH % 4 == 0, "channel quads");
  static_assert(LDS_BYTES <= 160 * 1024, "LDS of one workgroup");
  // slot of plane p = 2 py + px with shift s
  __device__ static constexpr int slot(int p, int s) { return s == 0 ? p : 4 + (KS == 3 ? (p >> 1) : p); }
};

template <class T>
__device__ __forceinline__ void wg_store4(T* dst, const float v[4]);
template <>
__device__ __forceinline__ void wg_store4<float>(float* dst, const float v[4]) {
  *reinterpret_cast<float4*>(dst) = make_float4(v[0], v[1], v[2], v[3]);
}
template <>
__device__ __forceinline__ void wg_store4<bf16>(bf16* dst, const float v[4]) {
  // values are BF16-exact (they were loaded from BF16), so truncation packs them exactly
  const uint32_t lo = (__float_as_uint(v[0]) >> 16) | (__float_as_uint(v[1]) & 0xffff0000u);
  const uint32_t hi = (__float_as_uint(v[2]) >> 16) | (__float_as_uint(v[3]) & 0xffff0000u);
  *reinterpret_cast<uint2*>(dst) = make_uint2(lo, hi);
}

template <class T, bool DEC, int CL, int CH, int TH, int TW>
struct k_s2_wgrad_v_args {
  const T* lo;
  const T* hi;
  float* part;
  int B;
  int h;
  int w;
};
template <class T, bool DEC, int CL, int CH, int TH, int TW>
__global__ __launch_bounds__(256) void k_s2_wgrad_v(SegL<k_s2_wgrad_v_args<T, DEC, CL, CH, TH, TW>> L) {
  const SegB sb = seg_block(L);
  if (sb.x >= sb.gx) return;
  const int bx = sb.x, gx = sb.gx;  // workgroup index and count within the segment
  (void)gx;
  const k_s2_wgrad_v_args<T, DEC, CL, CH, TH, TW>& a_ = L.a[sb.s];
  const T* __restrict__ const lo = a_.lo;
  const T* __restrict__ const hi = a_.hi;
  float* __restrict__ const part = a_.part;
  const int B = a_.B;
  const int h = a_.h;
  const int w = a_.w;
  typedef WgVCfg<T, DEC, CL, CH, TH, TW> C;
  typedef typename WgVec<T>::type V;
  constexpr int KS = C::KS, PW_ = C::PW_, NTC = C::NTC, MTC = C::MTC, LP = C::LP, CS = C::CS, PY = C::PY;
  constexpr bool BF = sizeof(T) == 2;
  __shared__ __attribute__((aligned(16))) T lds[C::ELEMS];
  T* const ls = lds;            // [CL][LP]
  T* const hs = lds + CL * LP;  // [slot][CH][PY][TW] with channel stride CS
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, i = lane & 15, g = lane >> 4;
  const int H2 = 2 * h, W2 = 2 * w;

  floatx4 acc[PW_][NTC];
#pragma unroll
  for (int u = 0; u < PW_; ++u)
#pragma unroll
    for (int j = 0; j < NTC; ++j) acc[u][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int nty = (h + TH - 1) / TH, ntx = (w + TW - 1) / TW;
  const int64_t ntiles = (int64_t)B * nty * ntx;
  int64_t t_begin, t_end, t_step;
  if ((gx & 7) == 0) {
    const int xcd = bx & 7, l = bx >> 3, per = gx >> 3;
    const int64_t chunk = (ntiles + 7) / 8;
    t_begin = xcd * chunk + l;
    t_end = (xcd + 1) * chunk < ntiles ? (xcd + 1) * chunk : ntiles;
    t_step = per;
  } else {
    t_begin = bx;
    t_end = ntiles;
    t_step = gx;
  }
  if constexpr (BF) {
    // BF16: the operands stay packed from HBM to the matrix core.  The staging units of the next
    // tile are loaded (4 channels of a pixel = one 8-byte load) while this tile's products run, the
    // 4 x 4 transposes are byte permutes, and two 16-pixel chunks feed one
    // v_mfma_f32_16x16x32_bf16 (lane group g: pixels 4g .. 4g + 3 of each chunk, the same
    // reduction order for both operands).
    constexpr int LU = (CL / 4) * (TH * TW / 4), XQ = TW / 4, HU = C::SLOTS * (CH / 4) * PY * XQ;
    constexpr int PL = (LU + STDA_BLOCK - 1) / STDA_BLOCK, PH = (HU + STDA_BLOCK - 1) / STDA_BLOCK;
    uint2 lv[PL][4], hv[PH][4];  // [unit][pixel]: channels 4 cq .. 4 cq + 3 packed
    auto fetch = [&](int64_t tt) {
      int b, y0, x0;
      s2_tile_origin(tt, nty, ntx, TH, TW, b, y0, x0);
#pragma unroll
      for (int k = 0; k < PL; ++k) {
        const int e = threadIdx.x + k * STDA_BLOCK;
        const int cq = e % (CL / 4), p0 = 4 * (e / (CL / 4)), ty = p0 / TW, tx = p0 % TW, y = y0 + ty;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int x = x0 + tx + q;
          lv[k][q] = (e < LU && y < h && x < w)
                         ? *reinterpret_cast<const uint2*>(lo + (((int64_t)b * h + y) * w + x) * CL + 4 * cq)
                         : make_uint2(0u, 0u);
        }
      }
#pragma unroll
      for (int k = 0; k < PH; ++k) {
        const int e = threadIdx.x + k * STDA_BLOCK;
        int r = e;
        const int xq = r % XQ;
        r /= XQ;
        const int Y = r % PY;
        r /= PY;
        const int cq = r % (CH / 4), sl = r / (CH / 4);
        const int s = sl < 4 ? 0 : 1;
        const int pp = sl < 4 ? sl : (KS == 3 ? 2 * (sl - 4) : sl - 4);
        const int ly = 2 * Y + (pp >> 1), sy = 2 * y0 - 1 + ly;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int lx = 2 * (4 * xq + q + s) + (pp & 1), sx = 2 * x0 - 1 + lx;
          hv[k][q] = (e < HU && ly < C::SH && lx < C::SW && sy >= 0 && sy < H2 && sx >= 0 && sx < W2)
                         ? *reinterpret_cast<const uint2*>(hi + (((int64_t)b * H2 + sy) * W2 + sx) * CH + 4 * cq)
                         : make_uint2(0u, 0u);
        }
      }
    };
    // channel c of pixels 0..3 of a unit (u[q] holds channels 4 cq .. 4 cq + 3 of pixel q), as the
    // four BF16 values of one 8-byte LDS row segment
    auto column = [](const uint2 (&u)[4], int c) {
      const uint32_t sel = (c & 1) ? 0x07060302u : 0x05040100u;
      const uint32_t a0 = (c & 2) ? u[0].y : u[0].x, a1 = (c & 2) ? u[1].y : u[1].x;
      const uint32_t a2 = (c & 2) ? u[2].y : u[2].x, a3 = (c & 2) ? u[3].y : u[3].x;
      return make_uint2(__builtin_amdgcn_perm(a1, a0, sel), __builtin_amdgcn_perm(a3, a2, sel));
    };
    if (t_begin < t_end) fetch(t_begin);
    for (int64_t t = t_begin; t < t_end; t += t_step) {
      __syncthreads();  // the previous tile's products have read the LDS operands
#pragma unroll
      for (int k = 0; k < PL; ++k) {
        const int e = threadIdx.x + k * STDA_BLOCK;
        if (e >= LU) continue;
        const int cq = e % (CL / 4), p0 = 4 * (e / (CL / 4));
#pragma unroll
        for (int c = 0; c < 4; ++c) *reinterpret_cast<uint2*>(ls + (4 * cq + c) * LP + p0) = column(lv[k], c);
      }
#pragma unroll
      for (int k = 0; k < PH; ++k) {
        const int e = threadIdx.x + k * STDA_BLOCK;
        if (e >= HU) continue;
        int r = e;
        const int xq = r % XQ;
        r /= XQ;
        const int Y = r % PY;
        r /= PY;
        const int cq = r % (CH / 4), sl = r / (CH / 4);
#pragma unroll
        for (int c = 0; c < 4; ++c)
          *reinterpret_cast<uint2*>(hs + (sl * CH + 4 * cq + c) * CS + Y * TW + 4 * xq) = column(hv[k], c);
      }
      __syncthreads();
      if (t + t_step < t_end) fetch(t + t_step);
      constexpr int NCH = TH * TW / 16;
#pragma unroll 1
      for (int c32 = 0; c32 < NCH / 2; ++c32) {
        const int pa = 32 * c32 + 4 * g, pb = pa + 16;
        const int tya = pa / TW, txa = pa % TW, tyb = pb / TW, txb = pb % TW;
        bf16x8 bq[NTC];
#pragma unroll
        for (int j = 0; j < NTC; ++j)
          bq[j] = pack8(*reinterpret_cast<const shortx4*>(ls + (16 * j + i) * LP + pa),
                        *reinterpret_cast<const shortx4*>(ls + (16 * j + i) * LP + pb));
#pragma unroll
        for (int u = 0; u < PW_; ++u) {
          const int q = wave + 4 * u;
          if (q >= C::PAIRS) continue;
          const int tap = q / MTC, mt = q % MTC, ky = tap / KS, kx = tap % KS;
          const int sl = C::slot((ky & 1) * 2 + (kx & 1), kx >> 1);
          const T* hb = hs + (sl * CH + 16 * mt + i) * CS + (ky >> 1) * TW;
          const bf16x8 a = pack8(*reinterpret_cast<const shortx4*>(hb + tya * TW + txa),
                                 *reinterpret_cast<const shortx4*>(hb + tyb * TW + txb));
#pragma unroll
          for (int j = 0; j < NTC; ++j)
            acc[u][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bq[j], acc[u][j], 0, 0, 0);
        }
      }
      if constexpr (NCH % 2 == 1) {  // an odd last chunk on the 16-deep instruction
        const int p0 = 16 * (NCH - 1) + 4 * g, ty = p0 / TW, tx = p0 % TW;
        shortx4 bq[NTC];
#pragma unroll
        for (int j = 0; j < NTC; ++j) bq[j] = *reinterpret_cast<const shortx4*>(ls + (16 * j + i) * LP + p0);
#pragma unroll
        for (int u = 0; u < PW_; ++u) {
          const int q = wave + 4 * u;
          if (q >= C::PAIRS) continue;
          const int tap = q / MTC, mt = q % MTC, ky = tap / KS, kx = tap % KS;
          const int sl = C::slot((ky & 1) * 2 + (kx & 1), kx >> 1);
          const shortx4 a =
              *reinterpret_cast<const shortx4*>(hs + (sl * CH + 16 * mt + i) * CS + (ty + (ky >> 1)) * TW + tx);
#pragma unroll
          for (int j = 0; j < NTC; ++j)
            acc[u][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bq[j], acc[u][j], 0, 0, 0);
        }
      }
    }
  } else {
    for (int64_t t = t_begin; t < t_end; t += t_step) {
      int b, y0, x0;
      s2_tile_origin(t, nty, ntx, TH, TW, b, y0, x0);
      __syncthreads();
      // Staging: a unit is (4 channels, 4 consecutive pixels); every load of the thread's units is
      // issued before the first transpose and LDS write, so their latencies overlap.
      // Lo units: (channel quad, pixel quad of a tile row); Hi units: (slot, channel quad, plane row,
      // quad of plane columns).
      {
        constexpr int LU = (CL / 4) * (TH * TW / 4), XQ = TW / 4, HU = C::SLOTS * (CH / 4) * PY * XQ;
        constexpr int PL = (LU + STDA_BLOCK - 1) / STDA_BLOCK, PH = (HU + STDA_BLOCK - 1) / STDA_BLOCK;
        float lv[PL][4][4], hv[PH][4][4];  // [unit][pixel][channel]
  #pragma unroll
        for (int k = 0; k < PL; ++k) {
          const int e = threadIdx.x + k * STDA_BLOCK;
          const int cq = e % (CL / 4), p0 = 4 * (e / (CL / 4)), ty = p0 / TW, tx = p0 % TW, y = y0 + ty;
  #pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int x = x0 + tx + q;
            if (e < LU && y < h && x < w) ld4(lo + (((int64_t)b * h + y) * w + x) * CL + 4 * cq, lv[k][q]);
            else zero4(lv[k][q]);
          }
        }
  #pragma unroll
        for (int k = 0; k < PH; ++k) {
          const int e = threadIdx.x + k * STDA_BLOCK;
          int r = e;
          const int xq = r % XQ;
          r /= XQ;
          const int Y = r % PY;
          r /= PY;
          const int cq = r % (CH / 4), sl = r / (CH / 4);
          const int s = sl < 4 ? 0 : 1;
          const int p = sl < 4 ? sl : (KS == 3 ? 2 * (sl - 4) : sl - 4);
          const int ly = 2 * Y + (p >> 1), sy = 2 * y0 - 1 + ly;
  #pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int lx = 2 * (4 * xq + q + s) + (p & 1), sx = 2 * x0 - 1 + lx;
            if (e < HU && ly < C::SH && lx < C::SW && sy >= 0 && sy < H2 && sx >= 0 && sx < W2)
              ld4(hi + (((int64_t)b * H2 + sy) * W2 + sx) * CH + 4 * cq, hv[k][q]);
            else
              zero4(hv[k][q]);
          }
        }
  #pragma unroll
        for (int k = 0; k < PL; ++k) {
          const int e = threadIdx.x + k * STDA_BLOCK;
          if (e >= LU) continue;
          const int cq = e % (CL / 4), p0 = 4 * (e / (CL / 4));
  #pragma unroll
          for (int c = 0; c < 4; ++c) {
            const float col[4] = {lv[k][0][c], lv[k][1][c], lv[k][2][c], lv[k][3][c]};
            wg_store4<T>(ls + (4 * cq + c) * LP + p0, col);
          }
        }
  #pragma unroll
        for (int k = 0; k < PH; ++k) {
          const int e = threadIdx.x + k * STDA_BLOCK;
          if (e >= HU) continue;
          int r = e;
          const int xq = r % XQ;
          r /= XQ;
          const int Y = r % PY;
          r /= PY;
          const int cq = r % (CH / 4), sl = r / (CH / 4);
  #pragma unroll
          for (int c = 0; c < 4; ++c) {
            const float col[4] = {hv[k][0][c], hv[k][1][c], hv[k][2][c], hv[k][3][c]};
            wg_store4<T>(hs + (sl * CH + 4 * cq + c) * CS + Y * TW + 4 * xq, col);
          }
        }
      }
      __syncthreads();
  #pragma unroll 1
      for (int c16 = 0; c16 < TH * TW / 16; ++c16) {
        const int p0 = 16 * c16 + 4 * g, ty = p0 / TW, tx = p0 % TW;
        V bq[NTC];
  #pragma unroll
        for (int j = 0; j < NTC; ++j) bq[j] = *reinterpret_cast<const V*>(ls + (16 * j + i) * LP + p0);
  #pragma unroll
        for (int u = 0; u < PW_; ++u) {
          const int q = wave + 4 * u;
          if (q >= C::PAIRS) continue;
          const int tap = q / MTC, mt = q % MTC, ky = tap / KS, kx = tap % KS;
          const int sl = C::slot((ky & 1) * 2 + (kx & 1), kx >> 1);
          const V a = *reinterpret_cast<const V*>(hs + (sl * CH + 16 * mt + i) * CS + (ty + (ky >> 1)) * TW + tx);
  #pragma unroll
          for (int j = 0; j < NTC; ++j) {
            if constexpr (BF) {
              acc[u][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, bq[j], acc[u][j], 0, 0, 0);
            } else {
              acc[u][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, bq[j].x, acc[u][j], 0, 0, 0);
              acc[u][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, bq[j].y, acc[u][j], 0, 0, 0);
              acc[u][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, bq[j].z, acc[u][j], 0, 0, 0);
              acc[u][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, bq[j].w, acc[u][j], 0, 0, 0);
            }
          }
        }
      }
    }
  }
  constexpr int NCOL = DEC ? C::TAPS * CH : CL;
  float* out = part + (int64_t)bx * C::TAPS * CH * CL;
#pragma unroll
  for (int u = 0; u < PW_; ++u) {
    const int q = wave + 4 * u;
    if (q >= C::PAIRS) continue;
    const int tap = q / MTC, mt = q % MTC;
#pragma unroll
    for (int j = 0; j < NTC; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int ch = 16 * mt + 4 * g + r, cl = 16 * j + i;
        const int64_t idx = DEC ? (int64_t)cl * NCOL + tap * CH + ch : ((int64_t)tap * CH + ch) * NCOL + cl;
        out[idx] = acc[u][j][r];
      }
  }
}

}  // namespace stda
