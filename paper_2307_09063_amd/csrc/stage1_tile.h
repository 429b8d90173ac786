// Stage 1 of the mobile encoder / decoder blocks on LDS tiles (gfx950).
//
// Stage 1 (first equation group of the mobile block): u = BN_p(PW(x)) + BN_d(DW3x3(x)) + BN_x(x),
// x1 = ReLU(u); PW is a dense C x C pointwise layer, DW a depthwise 3x3 (transposed, i.e. with a
// flipped kernel, in the decoder).  A block stages a TH x TW pixel tile of x plus a halo into
// LDS with coalesced 16-byte loads (zeros outside the map) and computes every pixel of the tile
// from LDS; the grid loops over the tiles of all clips.  Thread mapping inside a tile: item =
// (pixel, group of 4 channels), channel group fastest, so a thread keeps one channel group for
// its whole life.  LDS tiles are [pixel][C] floats laid out by S1Lds (see there) so that the
// access patterns avoid bank conflicts: one thread per (pixel, chunk) reading float4s, and
// matrix-core operands reading one channel of 16 consecutive pixels.
#pragma once
#include "net_kernels.h"

namespace stda {

template <int C>
struct S1Tile;
template <>
struct S1Tile<16> {
  static constexpr int TH = 8, TW = 16;
};
template <>
struct S1Tile<32> {
  static constexpr int TH = 8, TW = 8;
};
template <>
struct S1Tile<64> {
  static constexpr int TH = 4, TW = 4;
};

template <int C>
struct S1Geo {
  static constexpr int TH = S1Tile<C>::TH, TW = S1Tile<C>::TW, G = C / 4;
};

// LDS layout of an NPIX-pixel [pixel][C] tile.  64 channels: rows of C floats whose 16-byte chunk
// q sits in slot q ^ (px & 15), so that 16 consecutive pixels cover all 64 banks in both access
// patterns.  16 and 32 channels: planar by 16-byte chunk, plane q holding chunk q of every pixel
// (px * 4 floats into the plane), planes PL floats apart with PL = 16 (16 channels) or 8 (32
// channels) modulo the 64 banks.  Then the quarter-wave of a 16-byte access (4 or 2 consecutive
// pixels x all chunks), a matrix-core operand (one channel of 16 consecutive pixels) and a
// weight-gradient operand (16 channels of 4 pixels) each touch distinct banks, and a tap's
// offset stays a constant the compiler folds into the instruction.
template <int C, int NPIX>
struct S1Lds {
  static constexpr bool SWZ = C == 64;
  static constexpr int TGT = C == 16 ? 16 : 8;
  static constexpr int PL = NPIX * 4 + (TGT - (NPIX * 4) % 64 + 64) % 64;
  static constexpr int SIZE = SWZ ? NPIX * C : (C / 4 - 1) * PL + NPIX * 4;  // no pad after the last plane
};
// Float offset of chunk q (channels 4q .. 4q + 3) of LDS pixel px, and of channel c.
template <int C, int NPIX>
__device__ __forceinline__ int s1c(int px, int q) {
  if constexpr (S1Lds<C, NPIX>::SWZ) return px * C + ((q ^ (px & (C / 4 - 1))) << 2);
  else return q * S1Lds<C, NPIX>::PL + (px << 2);
}
template <int C, int NPIX>
__device__ __forceinline__ int s1e(int px, int c) {
  return s1c<C, NPIX>(px, c >> 2) + (c & 3);
}
// Channels 4q .. 4q + 3 of pixel px0 + dpx of a tile: in the planar layouts a pixel step is a
// fixed float offset, so a neighbourhood is one base address plus constant offsets (immediate
// offsets of the LDS reads); the swizzled layout computes each address.
template <int C, int NPIX>
__device__ __forceinline__ float4 s1_nbr(const float* lds, int px0, int q, int dpx) {
  if constexpr (S1Lds<C, NPIX>::SWZ) return *reinterpret_cast<const float4*>(lds + s1c<C, NPIX>(px0 + dpx, q));
  else return *reinterpret_cast<const float4*>(lds + s1c<C, NPIX>(px0, q) + 4 * dpx);
}

// Rows y0-HALO .. y0+TH+HALO-1 and columns x0-HALO .. x0+TW+HALO-1 of clip b -> lds, pixel
// (row, col) of the haloed tile at LDS pixel row * (TW + 2 HALO) + col.
// BATCH: every load of the thread is issued before the first LDS write, so that their latencies
// overlap (at the cost of the registers holding them; measured per kernel, see the callers).
template <class T, int C, int TH, int TW, int HALO, bool BATCH = true>
__device__ __forceinline__ void load_tile(const T* __restrict__ X, int b, int y0, int x0, int h, int w, float* lds) {
  constexpr int RW = TW + 2 * HALO, RH = TH + 2 * HALO, G = C / 4, N = RH * RW * G;
  if constexpr (!BATCH) {
    for (int e = threadIdx.x; e < N; e += STDA_BLOCK) {
      const int q = e % G, px = e / G;
      const int y = y0 - HALO + px / RW, x = x0 - HALO + px % RW;
      float v[4];
      if (y >= 0 && y < h && x >= 0 && x < w)
        ld4(X + (((int64_t)b * h + y) * w + x) * C + 4 * q, v);
      else
        zero4(v);
      *reinterpret_cast<float4*>(lds + s1c<C, RH * RW>(px, q)) = make_float4(v[0], v[1], v[2], v[3]);
    }
    return;
  }
  constexpr int K = (N + STDA_BLOCK - 1) / STDA_BLOCK;
  float v[K][4];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = threadIdx.x + k * STDA_BLOCK;
    const int q = e % G, px = e / G;
    const int y = y0 - HALO + px / RW, x = x0 - HALO + px % RW;
    if (e < N && y >= 0 && y < h && x >= 0 && x < w)
      ld4(X + (((int64_t)b * h + y) * w + x) * C + 4 * q, v[k]);
    else
      zero4(v[k]);
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = threadIdx.x + k * STDA_BLOCK;
    if (e < N)
      *reinterpret_cast<float4*>(lds + s1c<C, RH * RW>(e / G, e % G)) = make_float4(v[k][0], v[k][1], v[k][2], v[k][3]);
  }
}

// FP32, planar layouts: the same tile fetched by buffer loads that write LDS directly, one
// instruction per 64 consecutive pixels of one 4-channel plane (a plane holds its pixels as
// consecutive 16-byte chunks, the order in which a load's 64 lanes write).  The LDS layout is that
// of NPIXL >= the tile's pixels, a multiple of 64, so that every lane of every load writes inside
// its plane: no lane is masked off, and each wave issues the same loads on every path (the
// compiler's waits for loads issued before these then leave these in flight).  Issued without
// VGPRs and without a wait: the caller waits for its own wave's loads (wait_vmem) and
// then synchronises the workgroup before the tile is read; barriers in between must leave vector
// memory in flight (lds_barrier).  A pixel off the map, or past the tile, gets an offset beyond
// the clip's buffer range, which the range check turns into zeros.  A clip is at most 4096 x 4096
// pixels of 16 channels here (1 GiB), inside the 2 GiB a buffer range can describe.
template <int C, int TH, int TW, int HALO, int NPIXL>
__device__ __forceinline__ void load_tile_dma(const float* X, int b, int y0, int x0, int h, int w, float* lds) {
  constexpr int RW = TW + 2 * HALO, RH = TH + 2 * HALO, NPIX = RH * RW, G = C / 4;
  constexpr int NCH = NPIXL / 64;  // 64-pixel chunks of a plane
  static_assert(NPIXL % 64 == 0 && NPIXL >= NPIX && !S1Lds<C, NPIXL>::SWZ, "planar layout of whole 64-pixel chunks");
  static_assert((G * NCH) % (STDA_BLOCK / 64) == 0, "the same number of loads in every wave");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int bytes = h * w * (C * 4);
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(X + (int64_t)b * h * w * C), (short)0, bytes, 0x00020000);
#pragma unroll
  for (int i = 0; i < G * NCH / (STDA_BLOCK / 64); ++i) {
    const int j = wave + i * (STDA_BLOCK / 64), q = j / NCH, p0 = (j % NCH) * 64, px = p0 + lane;
    const int y = y0 - HALO + px / RW, x = x0 - HALO + px % RW;
    const bool in = px < NPIX && y >= 0 && y < h && x >= 0 && x < w;
    const int off = in ? ((y * w + x) * C + 4 * q) * 4 : (int)0x80000000u;
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, lds_ptr(lds + s1c<C, NPIXL>(p0, q)), 16, off, 0, 0, 0);
  }
}

// The tile's pixels in storage form (BF16, or FP32 where a second x buffer does not fit) fetched
// by buffer loads that write LDS directly into a staging buffer (NPIXL pixels of C values, pixel
// after pixel as in HBM; a load's 64 lanes write 64 consecutive 16-byte chunks), for
// stage1_put_raw to convert into load_tile's FP32 layout.  Waits, synchronisation and out-of-map
// zeros as for load_tile_dma.
template <class T, int C, int TH, int TW, int HALO, int NPIXL>
__device__ __forceinline__ void load_tile_dma_raw(const T* X, int b, int y0, int x0, int h, int w, uint32_t* stg) {
  constexpr int RW = TW + 2 * HALO, RH = TH + 2 * HALO, NPIX = RH * RW;
  constexpr int CH = C * (int)sizeof(T) / 16, PPI = 64 / CH, NI = NPIXL / PPI;  // chunks per pixel, pixels per load
  static_assert(64 % CH == 0 && NPIXL % PPI == 0 && NPIXL >= NPIX, "whole loads of whole pixels");
  static_assert(NI % (STDA_BLOCK / 64) == 0, "the same number of loads in every wave");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int bytes = h * w * (C * (int)sizeof(T));
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(X + (int64_t)b * h * w * C), (short)0, bytes, 0x00020000);
#pragma unroll
  for (int i = 0; i < NI / (STDA_BLOCK / 64); ++i) {
    const int j = wave + i * (STDA_BLOCK / 64), px = j * PPI + lane / CH, hc = lane % CH;
    const int y = y0 - HALO + px / RW, x = x0 - HALO + px % RW;
    const bool in = px < NPIX && y >= 0 && y < h && x >= 0 && x < w;
    const int off = in ? (y * w + x) * (C * (int)sizeof(T)) + hc * 16 : (int)0x80000000u;
    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, lds_ptr(stg + j * 256), 16, off, 0, 0, 0);
  }
}
// The staged tile of NPIX pixels -> FP32 LDS tile in the layout of S1Lds<C, NPIXL>.
template <class T, int C, int NPIX, int NPIXL>
__device__ __forceinline__ void stage1_put_raw(const uint32_t* stg, float* lds) {
  constexpr int G = C / 4;
  const T* st = reinterpret_cast<const T*>(stg);
  for (int e = threadIdx.x; e < NPIX * G; e += STDA_BLOCK) {
    const int px = e / G, q = e % G;
    const typename Raw4<T>::type r = *reinterpret_cast<const typename Raw4<T>::type*>(st + px * C + 4 * q);
    float v[4];
    raw_cvt4(r, v);
    *reinterpret_cast<float4*>(lds + s1c<C, NPIXL>(px, q)) = make_float4(v[0], v[1], v[2], v[3]);
  }
}

// The same tile in two halves, for software pipelining across a grid-stride tile loop: fetch()
// issues this thread's loads into registers in storage form (they stay in flight until put()),
// put() converts them and writes the LDS tile in load_tile's layout.
template <class T, int C, int TH, int TW, int HALO>
struct TileRegs {
  static constexpr int RW = TW + 2 * HALO, RH = TH + 2 * HALO, G = C / 4, N = RH * RW * G;
  static constexpr int K = (N + STDA_BLOCK - 1) / STDA_BLOCK;
  typename Raw4<T>::type v[K];
  __device__ __forceinline__ void fetch(const T* __restrict__ X, int b, int y0, int x0, int h, int w) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int e = threadIdx.x + k * STDA_BLOCK;
      const int q = e % G, px = e / G;
      const int y = y0 - HALO + px / RW, x = x0 - HALO + px % RW;
      if (e < N && y >= 0 && y < h && x >= 0 && x < w)
        raw_ld4(X + (((int64_t)b * h + y) * w + x) * C + 4 * q, v[k]);
      else
        raw_zero4(v[k]);
    }
  }
  __device__ __forceinline__ void put(float* lds) const {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int e = threadIdx.x + k * STDA_BLOCK;
      if (e < N) {
        float f[4];
        raw_cvt4(v[k], f);
        *reinterpret_cast<float4*>(lds + s1c<C, RH * RW>(e / G, e % G)) = make_float4(f[0], f[1], f[2], f[3]);
      }
    }
  }
};

__device__ __forceinline__ void tile_coords(int tile, int h, int w, int TH, int TW, int& b, int& y0, int& x0) {
  const int ty = (h + TH - 1) / TH, tx = (w + TW - 1) / TW;
  b = tile / (ty * tx);
  const int r = tile - b * ty * tx;
  y0 = (r / tx) * TH;
  x0 = (r % tx) * TW;
}

typedef float floatx4_t __attribute__((ext_vector_type(4)));

// store(i, n, sum_k A(i, k) B(k, n)) for an M x N x K product held in LDS, on the matrix cores
// (v_mfma_f32_16x16x4f32); A and B are addressing functors.  The block's 4 waves take 16 x 16
// output tiles in turn.  Caller synchronises around it.
template <int M, int N, int K, class AF, class BF, class SF>
__device__ __forceinline__ void lds_gemm_s(AF A, BF B, SF store) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, i = lane & 15, g = lane >> 4;
  for (int t = wave; t < (M / 16) * (N / 16); t += 4) {
    const int m0 = (t / (N / 16)) * 16, n0 = (t % (N / 16)) * 16;
    floatx4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int k = 0; k < K; k += 4)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A(m0 + i, k + g), B(k + g, n0 + i), acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) store(m0 + 4 * g + r, n0 + i, acc[r]);
  }
}

// The same product stored row-major into Cm with row stride ldc.
template <int M, int N, int K, class AF, class BF>
__device__ __forceinline__ void lds_gemm(AF A, BF B, float* Cm, int ldc) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, i = lane & 15, g = lane >> 4;
  for (int t = wave; t < (M / 16) * (N / 16); t += 4) {
    const int m0 = (t / (N / 16)) * 16, n0 = (t % (N / 16)) * 16;
    floatx4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int k = 0; k < K; k += 4)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A(m0 + i, k + g), B(k + g, n0 + i), acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) Cm[(m0 + 4 * g + r) * ldc + n0 + i] = acc[r];
  }
}

// Depthwise branch (4 channels) of the pixel at padded LDS position (r, c) of a tile with rows of RW
// pixels.  wr: this thread's 4 channels of the 9 taps, held in registers.
template <int C, int NPIX, int RW>
__device__ __forceinline__ void s1_dw_lds(const float* xt, int r, int c, int c0, const float (&wr)[9][4], float dv[4]) {
  zero4(dv);
  const int p0 = (r - 1) * RW + c - 1;  // top-left neighbour
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const float4 v = s1_nbr<C, NPIX>(xt, p0, c0 >> 2, (t / 3) * RW + t % 3);
    dv[0] += wr[t][0] * v.x;
    dv[1] += wr[t][1] * v.y;
    dv[2] += wr[t][2] * v.z;
    dv[3] += wr[t][3] * v.w;
  }
}

// Channels c0 .. c0 + 3 of the 9 depthwise taps, from LDS into registers.
template <int C>
__device__ __forceinline__ void s1_dw_regs(const float* wd, int c0, float (&wr)[9][4]) {
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const float4 q = *reinterpret_cast<const float4*>(wd + t * C + c0);
    wr[t][0] = q.x;
    wr[t][1] = q.y;
    wr[t][2] = q.z;
    wr[t][3] = q.w;
  }
}

// Forward.  MODE 0: per-block (mean, m2) of the three BN inputs, part[blk][3][C][2], and the
// block's count at part[blocks * 6 C + blk] (blocks = the segment's workgroups; see
// block_chan_stats).  MODE 1: X1 = ReLU(BN_p(p) + BN_d(d) + BN_x(x)) and, if M1 is not null, the
// ReLU decisions X1 > 0 as one bit per element (M1[pixel][C / 8], channel c at byte c / 8, bit
// c % 8), which is all the adjoint needs of X1.
template <class T, int C, bool DEC, int MODE>
struct k_s1_tile_args {
  const T* X;
  T* X1;
  uint8_t* M1;
  float* part;
  S1Params prm;
  int B;
  int h;
  int w;
};
template <class T, int C, bool DEC, int MODE>
__global__ __launch_bounds__(256) void k_s1_tile(SegL<k_s1_tile_args<T, C, DEC, MODE>> L) {
  const SegB sb = seg_block(L);
  if (sb.x >= sb.gx) return;
  const int bx = sb.x, gx = sb.gx;  // workgroup index and count within the segment
  (void)gx;
  const k_s1_tile_args<T, C, DEC, MODE>& a_ = L.a[sb.s];
  const T* __restrict__ const X = a_.X;
  T* __restrict__ const X1 = a_.X1;
  uint8_t* __restrict__ const M1 = a_.M1;
  float* __restrict__ const part = a_.part;
  const S1Params& prm = a_.prm;
  const int B = a_.B;
  const int h = a_.h;
  const int w = a_.w;
  typedef S1Geo<C> Gm;
  constexpr int TH = Gm::TH, TW = Gm::TW, G = Gm::G, RW = TW + 2;
  constexpr int XN = (TH + 2) * RW, PN = TH * TW;  // pixels of the x tile (halo 1) and of the tile
  __shared__ float xt[S1Lds<C, XN>::SIZE];
  __shared__ float pt[S1Lds<C, PN>::SIZE];  // pointwise branch of the tile (matrix cores)
  __shared__ float wp[C * C];
  __shared__ float wd[9 * C];
  __shared__ float sm[MODE == 0 ? 4 * (6 * C + 1) : 1];
  __shared__ float red[MODE == 0 ? 6 * C + 1 : 1];
  // BF16 (DMAB): the next tile's x is fetched in storage form by buffer loads into an LDS staging
  // buffer during a tile and converted at the start of the tile it belongs to; only where the
  // staging buffer keeps four workgroups (of 40 KiB at most) per CU.
  constexpr int LDS_BASE =
      4 * (S1Lds<C, XN>::SIZE + S1Lds<C, PN>::SIZE + C * C + 9 * C + (MODE == 0 ? 5 * (6 * C + 1) : 2));
  constexpr int SPPI = 64 * 16 / (C * (int)sizeof(T));                // pixels per staging load
  constexpr int XSL = (XN + 4 * SPPI - 1) / (4 * SPPI) * (4 * SPPI);  // staged pixels (whole loads in every wave)
  // (Not the 16-channel statistics pass, whose register prefetch below measured faster.)
  constexpr bool DMAB =
      sizeof(T) == 2 && !(MODE == 0 && C == 16) && LDS_BASE + XSL * C * (int)sizeof(T) <= 40 * 1024;
  __shared__ uint32_t xst[DMAB ? XSL * C * sizeof(T) / 4 : 1];
  stage1_load_weights<C, DEC>(prm.wpw, prm.wdw, wp, wd);
  const int c0 = (threadIdx.x % G) * 4;
  float wr[9][4];
  s1_dw_regs<C>(wd, c0, wr);
  float mn[3][4], q2[3][4];  // MODE 0: mean and m2 of the p, d, x branches (Welford)
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    zero4(mn[s]);
    zero4(q2[s]);
  }
  float cnt = 0.f;  // pixels seen by this thread
  float sc[3][4], sh[3][4];
  if (MODE == 1)
#pragma unroll
    for (int k = 0; k < 3; ++k) bn_affine4(prm.stats[k], prm.gamma[k], prm.beta[k], C, c0, sc[k], sh[k]);
  const int ntiles = B * ((h + TH - 1) / TH) * ((w + TW - 1) / TW);
  // PIPE: the x tile of the block's next tile is fetched while this one is computed.  It costs a
  // wave per SIMD, which pays (measured) only for the BF16 16-channel statistics pass.
  constexpr bool PIPE = !DMAB && MODE == 0 && C == 16 && sizeof(T) == 2;
  TileRegs<T, C, TH, TW, 1> nx;
  if (PIPE && bx < ntiles) {
    int b, y0, x0;
    tile_coords(bx, h, w, TH, TW, b, y0, x0);
    nx.fetch(X, b, y0, x0, h, w);
  }
  if constexpr (DMAB)
    if (bx < ntiles) {
      int b, y0, x0;
      tile_coords(bx, h, w, TH, TW, b, y0, x0);
      load_tile_dma_raw<T, C, TH, TW, 1, XSL>(X, b, y0, x0, h, w, xst);
    }
  for (int tile = bx; tile < ntiles; tile += gx) {
    int b, y0, x0;
    tile_coords(tile, h, w, TH, TW, b, y0, x0);
    if constexpr (DMAB) wait_vmem();  // this wave's part of the staged tile is in LDS
    __syncthreads();
    if constexpr (DMAB) {
      stage1_put_raw<T, C, XN, XN>(xst, xt);
      __syncthreads();
    } else if constexpr (PIPE) {
      nx.put(xt);
      __syncthreads();
      if (tile + gx < ntiles) {
        int nb, ny0, nx0;
        tile_coords(tile + gx, h, w, TH, TW, nb, ny0, nx0);
        nx.fetch(X, nb, ny0, nx0, h, w);
      }
    } else {
      load_tile<T, C, TH, TW, 1, C != 32>(X, b, y0, x0, h, w, xt);  // batched where it measured faster
      __syncthreads();
    }
    // pt[p][o] = sum_c x[p][c] wp[c][o]; tile pixel p = r*TW + cc sits at padded (r + 1, cc + 1)
    lds_gemm_s<TH * TW, C, C>([&](int p, int k) { return xt[s1e<C, XN>((p / TW + 1) * RW + p % TW + 1, k)]; },
                              [&](int k, int n) { return wp[k * C + n]; },
                              [&](int p, int n, float v) { pt[s1e<C, PN>(p, n)] = v; });
    if constexpr (DMAB) {
      // the next tile's x (after the last tile this tile again, never read), in flight until
      // that tile starts; issued after this tile's last LDS writes, which would otherwise wait
      int nb, ny0, nx0;
      tile_coords(tile + gx < ntiles ? tile + gx : tile, h, w, TH, TW, nb, ny0, nx0);
      load_tile_dma_raw<T, C, TH, TW, 1, XSL>(X, nb, ny0, nx0, h, w, xst);
      lds_barrier();
    } else {
      __syncthreads();
    }
    for (int e = threadIdx.x; e < TH * TW * G; e += STDA_BLOCK) {
      const int px = e / G, r = px / TW, cc = px % TW;
      const int y = y0 + r, x = x0 + cc;
      if (y >= h || x >= w) continue;
      float pv[4], dv[4], xv[4];
      const float4 pq = *reinterpret_cast<const float4*>(pt + s1c<C, PN>(px, c0 >> 2));
      pv[0] = pq.x;
      pv[1] = pq.y;
      pv[2] = pq.z;
      pv[3] = pq.w;
      const float4 xq = *reinterpret_cast<const float4*>(xt + s1c<C, XN>((r + 1) * RW + cc + 1, c0 >> 2));
      xv[0] = xq.x;
      xv[1] = xq.y;
      xv[2] = xq.z;
      xv[3] = xq.w;
      s1_dw_lds<C, XN, RW>(xt, r + 1, cc + 1, c0, wr, dv);
      if (MODE == 0) {
        cnt += 1.f;
        const float rk = __builtin_amdgcn_rcpf(cnt);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          wf_add(mn[0][j], q2[0][j], pv[j], rk);
          wf_add(mn[1][j], q2[1][j], dv[j], rk);
          wf_add(mn[2][j], q2[2][j], xv[j], rk);
        }
      } else {
        float o[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          o[j] = fmaxf(pv[j] * sc[0][j] + sh[0][j] + dv[j] * sc[1][j] + sh[1][j] + xv[j] * sc[2][j] + sh[2][j], 0.f);
        const int64_t pix = ((int64_t)b * h + y) * w + x;
        st4(X1 + pix * C + c0, o);
        if (M1) {
          // this thread's 4 decisions; the neighbouring lane holds the other half of the byte (the
          // two lanes share the pixel, so both are active here)
          const int nib = (o[0] > 0.f) | ((o[1] > 0.f) << 1) | ((o[2] > 0.f) << 2) | ((o[3] > 0.f) << 3);
          const int hi = __shfl_xor(nib, 1);
          if (!(c0 & 4)) M1[pix * (C / 8) + (c0 >> 3)] = (uint8_t)(nib | (hi << 4));
        }
      }
    }
  }
  if constexpr (DMAB) wait_vmem();  // the last (unused) fetch has landed
  if (MODE == 0) {
    block_chan_stats<G, 3>(cnt, mn, q2, sm, red);
    for (int q = threadIdx.x; q < 3 * C; q += STDA_BLOCK) {
      part[(int64_t)bx * 6 * C + 2 * q] = red[q];               // mean of (branch q / C, channel q % C)
      part[(int64_t)bx * 6 * C + 2 * q + 1] = red[3 * C + q];   // m2
    }
    if (threadIdx.x == 0) part[(int64_t)gx * 6 * C + bx] = red[6 * C];
  }
}

// Backward statistics: du = dX1 [X1 > 0] (the decisions read from the bit mask M1 the forward
// wrote); part[blk][4][C] = sum du, sum du*phat, sum du*dhat, sum du*xhat (branch outputs
// recomputed from the tile).
template <class T, int C, bool DEC>
struct k_s1_bwd_stats_tile_args {
  const T* X;
  const uint8_t* M1;
  const T* dX1;
  float* part;
  S1Params prm;
  int B;
  int h;
  int w;
};
template <class T, int C, bool DEC>
__global__ __launch_bounds__(256) void k_s1_bwd_stats_tile(SegL<k_s1_bwd_stats_tile_args<T, C, DEC>> L) {
  const SegB sb = seg_block(L);
  if (sb.x >= sb.gx) return;
  const int bx = sb.x, gx = sb.gx;  // workgroup index and count within the segment
  (void)gx;
  const k_s1_bwd_stats_tile_args<T, C, DEC>& a_ = L.a[sb.s];
  const T* __restrict__ const X = a_.X;
  const uint8_t* __restrict__ const M1 = a_.M1;
  const T* __restrict__ const dX1 = a_.dX1;
  float* __restrict__ const part = a_.part;
  const S1Params& prm = a_.prm;
  const int B = a_.B;
  const int h = a_.h;
  const int w = a_.w;
  typedef S1Geo<C> Gm;
  constexpr int TH = Gm::TH, TW = Gm::TW, G = Gm::G, RW = TW + 2;
  constexpr int XN = (TH + 2) * RW, PN = TH * TW;
  __shared__ float xt[S1Lds<C, XN>::SIZE];
  __shared__ float pt[S1Lds<C, PN>::SIZE];
  __shared__ float wp[C * C];
  __shared__ float wd[9 * C];
  __shared__ float sm[4 * 4 * C];
  __shared__ float red[4 * C];
  // BF16 (DMAB): the next tile's x is fetched in storage form by buffer loads into an LDS staging
  // buffer during a tile and converted at the start of the tile it belongs to; the thread's items
  // (at most two) load their x1 decisions and dx1 at the tile start, before that fetch is issued,
  // so that waiting for them does not wait for it.  Only where the staging buffer keeps three
  // workgroups (of 53 KiB at most) per CU: the kernel's registers allow no more than three above
  // 16 channels, and at 16 channels it still fits four.
  constexpr int NI = TH * TW * G;
  constexpr int LDS_BASE = 4 * (S1Lds<C, XN>::SIZE + S1Lds<C, PN>::SIZE + C * C + 9 * C + 20 * C);
  constexpr int SPPI = 64 * 16 / (C * (int)sizeof(T));                // pixels per staging load
  constexpr int XSL = (XN + 4 * SPPI - 1) / (4 * SPPI) * (4 * SPPI);  // staged pixels (whole loads in every wave)
  constexpr bool DMAB =
      sizeof(T) == 2 && NI <= 2 * STDA_BLOCK && LDS_BASE + XSL * C * (int)sizeof(T) <= 160 * 1024 / 3;
  __shared__ uint32_t xst[DMAB ? XSL * C * sizeof(T) / 4 : 1];
  stage1_load_weights<C, DEC>(prm.wpw, prm.wdw, wp, wd);
  const int c0 = (threadIdx.x % G) * 4;
  float wr[9][4];
  s1_dw_regs<C>(wd, c0, wr);
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
  const int ntiles = B * ((h + TH - 1) / TH) * ((w + TW - 1) / TW);
  // PIPE: the x tile of the block's next tile is fetched while this one is computed (measured
  // faster above 16 channels; at 16 it costs the kernel a wave per SIMD and time)
  constexpr bool PIPE = !DMAB && C > 16;
  TileRegs<T, C, TH, TW, 1> nx;
  if (PIPE && bx < ntiles) {
    int b, y0, x0;
    tile_coords(bx, h, w, TH, TW, b, y0, x0);
    nx.fetch(X, b, y0, x0, h, w);
  }
  if constexpr (DMAB)
    if (bx < ntiles) {
      int b, y0, x0;
      tile_coords(bx, h, w, TH, TW, b, y0, x0);
      load_tile_dma_raw<T, C, TH, TW, 1, XSL>(X, b, y0, x0, h, w, xst);
    }
  for (int tile = bx; tile < ntiles; tile += gx) {
    int b, y0, x0;
    tile_coords(tile, h, w, TH, TW, b, y0, x0);
    // BF16 above 16 channels: x1 and dx1 of the thread's next item loaded one item ahead, in
    // storage form (the first item's loads overlap the staging and the product); otherwise each
    // item loads its own in place (measured faster there: the 16-channel tiles lose a wave per SIMD)
    constexpr bool PF = sizeof(T) == 2 && C > 16 && !DMAB;
    typedef typename Raw4<T>::type R4;
    R4 ng, ng2;
    uint32_t nm, nm2;  // the byte of M1 holding this thread's 4 decisions (ng2, nm2: DMAB's second item)
    auto item_load_to = [&](int e, R4& g, uint32_t& m) {
      const int px = e / G, y = y0 + px / TW, x = x0 + px % TW;
      if (e < NI && y < h && x < w) {
        const int64_t off = (((int64_t)b * h + y) * w + x) * C + c0;
        m = M1[off >> 3];  // byte (pixel, c0 / 8) of the mask: C / 8 bytes per pixel
        raw_ld4(dX1 + off, g);
      } else {
        m = 0;
        raw_zero4(g);
      }
    };
    auto item_load = [&](int e) { item_load_to(e, ng, nm); };
    if constexpr (DMAB) {
      wait_vmem();  // this wave's part of the staged tile is in LDS
      item_load(threadIdx.x);
      if constexpr (NI > STDA_BLOCK) item_load_to(threadIdx.x + STDA_BLOCK, ng2, nm2);
    }
    if constexpr (PF) item_load(threadIdx.x);
    __syncthreads();
    if constexpr (DMAB) {
      stage1_put_raw<T, C, XN, XN>(xst, xt);
      __syncthreads();
    } else if constexpr (PIPE) {
      nx.put(xt);
      __syncthreads();
      if (tile + gx < ntiles) {
        int nb, ny0, nx0;
        tile_coords(tile + gx, h, w, TH, TW, nb, ny0, nx0);
        nx.fetch(X, nb, ny0, nx0, h, w);
      }
    } else {
      load_tile<T, C, TH, TW, 1, C != 16>(X, b, y0, x0, h, w, xt);  // batched where it measured faster
      __syncthreads();
    }
    lds_gemm_s<TH * TW, C, C>([&](int p, int k) { return xt[s1e<C, XN>((p / TW + 1) * RW + p % TW + 1, k)]; },
                              [&](int k, int n) { return wp[k * C + n]; },
                              [&](int p, int n, float v) { pt[s1e<C, PN>(p, n)] = v; });
    if constexpr (DMAB) {
      // the next tile's x (after the last tile this tile again, never read), in flight until
      // that tile starts; issued after this tile's last LDS writes, which would otherwise wait
      int nb, ny0, nx0;
      tile_coords(tile + gx < ntiles ? tile + gx : tile, h, w, TH, TW, nb, ny0, nx0);
      load_tile_dma_raw<T, C, TH, TW, 1, XSL>(X, nb, ny0, nx0, h, w, xst);
      lds_barrier();
    } else {
      __syncthreads();
    }
    for (int e = threadIdx.x; e < NI; e += STDA_BLOCK) {
      const int px = e / G, r = px / TW, cc = px % TW;
      const int y = y0 + r, x = x0 + cc;
      float g[4];
      uint32_t m;
      if constexpr (PF) {
        m = nm;
        raw_cvt4(ng, g);
        if (e + STDA_BLOCK < NI) item_load(e + STDA_BLOCK);
      } else if constexpr (DMAB) {
        const bool first = e < STDA_BLOCK;
        m = first ? nm : nm2;
        raw_cvt4(first ? ng : ng2, g);
      }
      if (y >= h || x >= w) continue;
      float pv[4], dv[4], xv[4];
      const float4 pq = *reinterpret_cast<const float4*>(pt + s1c<C, PN>(px, c0 >> 2));
      pv[0] = pq.x;
      pv[1] = pq.y;
      pv[2] = pq.z;
      pv[3] = pq.w;
      const float4 xq = *reinterpret_cast<const float4*>(xt + s1c<C, XN>((r + 1) * RW + cc + 1, c0 >> 2));
      xv[0] = xq.x;
      xv[1] = xq.y;
      xv[2] = xq.z;
      xv[3] = xq.w;
      s1_dw_lds<C, XN, RW>(xt, r + 1, cc + 1, c0, wr, dv);
      if constexpr (!PF && !DMAB) {
        const int64_t off = (((int64_t)b * h + y) * w + x) * C + c0;
        m = M1[off >> 3];
        ld4(dX1 + off, g);
      }
      m >>= (c0 & 4);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const float du = (m >> j) & 1u ? g[j] : 0.f;
        acc[0][j] += du;
        acc[1][j] += du * (pv[j] - mu[0][j]) * is[0][j];
        acc[2][j] += du * (dv[j] - mu[1][j]) * is[1][j];
        acc[3][j] += du * (xv[j] - mu[2][j]) * is[2][j];
      }
    }
  }
  if constexpr (DMAB) wait_vmem();  // the last (unused) fetch has landed
  block_chan_reduce_shfl<G, 4>(acc, sm, red);
  for (int q = threadIdx.x; q < 4 * C; q += STDA_BLOCK) part[(int64_t)bx * 4 * C + q] = red[q];
}

// Fused backward of stage 1.  With du = dX1 [X1 > 0] (decisions from the bit mask M1 of the
// forward) and the BN adjoint coefficients
// k[s][c] = (sum du, sum du*phat, sum du*dhat, sum du*xhat) / n:
//   dP = g_p is_p (du - k0 - phat k1), dD = g_d is_d (du - k0 - dhat k2),
//   dX = g_x is_x (du - k0 - xhat k3) + dXr + PW^T(dP) + DW^T(dD) (+ skip gradient),
// plus the pointwise weight gradient sum_p x[c](p) dP[o](p) -> pwpart[blk][c][o] and the
// depthwise one sum_p x[c](p + off_t) dD[c](p) -> dwpart[blk][tap][c] (the weight's own tap
// index, flipped in the decoder; accumulated as each tile pixel's dD is formed, from the 3x3
// neighbourhood of x that its depthwise recompute has just read).  Per tile: x on a 2-pixel halo,
// dD on a 1-pixel halo, dP and du in LDS (never in HBM; du is formed once, with dD, and read back
// for dX); the three pointwise
// products (p = x Wp, dP Wp^T, x^T dP) run on the matrix cores, the last one accumulating in
// registers across tiles.  Tiles are TH x TW pixels; MINW waves per SIMD bound the registers.
template <class T, int C, bool DEC, bool SKIP, int TH, int TW, int MINW, bool LC = false>
struct k_s1_bwd_fused_args {
  const T* X;
  const uint8_t* M1;
  const T* dX1;
  const T* dXr;
  const T* skip;
  const float* coef;
  S1Params prm;
  T* dX;
  float* pwpart;
  float* dwpart;
  int B;
  int h;
  int w;
};
template <class T, int C, bool DEC, bool SKIP, int TH, int TW, int MINW, bool LC = false>
__global__ __launch_bounds__(256, MINW) void k_s1_bwd_fused(SegL<k_s1_bwd_fused_args<T, C, DEC, SKIP, TH, TW, MINW, LC>> L) {
  const SegB sb = seg_block(L);
  if (sb.x >= sb.gx) return;
  const int bx = sb.x, gx = sb.gx;  // workgroup index and count within the segment
  (void)gx;
  const k_s1_bwd_fused_args<T, C, DEC, SKIP, TH, TW, MINW, LC>& a_ = L.a[sb.s];
  const T* __restrict__ const X = a_.X;
  const uint8_t* __restrict__ const M1 = a_.M1;
  const T* __restrict__ const dX1 = a_.dX1;
  const T* __restrict__ const dXr = a_.dXr;
  const T* __restrict__ const skip = a_.skip;
  const float* __restrict__ const coef = a_.coef;
  const S1Params& prm = a_.prm;
  T* __restrict__ const dX = a_.dX;
  float* __restrict__ const pwpart = a_.pwpart;
  float* __restrict__ const dwpart = a_.dwpart;
  const int B = a_.B;
  const int h = a_.h;
  const int w = a_.w;
  constexpr int G = C / 4, M = TH * TW;
  static_assert(M % 16 == 0, "matrix-core row tiles of 16 pixels");
  constexpr int XW = TW + 4, DWd = TW + 2;  // row widths of the x tile (halo 2) and dD tile (halo 1)
  constexpr int NT = (C / 16) * (C / 16), NTW = (NT + 3) / 4;  // pointwise-gradient tiles (per wave)
  constexpr int XN = (TH + 4) * XW, DN = (TH + 2) * DWd;  // pixels of the x and dD tiles
  // Not LC: the next tile's x is fetched by buffer loads into LDS during a tile.  FP32 at 16
  // channels (DMA): straight into a second x buffer, the x tiles laid out for whole 64-pixel
  // chunks (XNL pixels).  BF16, and FP32 at 64 channels (DMAB): in storage form into a staging
  // buffer, converted into the x tile at the start of the tile it belongs to (FP32 at 32 channels:
  // neither buffer fits beside the tile's others at two workgroups per CU).
  // Each only where the added buffer keeps MINW workgroups' LDS within the CU's 160 KiB.
  constexpr int LDS_REST = 4 * (S1Lds<C, DN>::SIZE + 3 * S1Lds<C, M>::SIZE + C * C + 18 * C);  // ddt .. cf
  constexpr int LDS_CAP = 160 * 1024 / MINW, XN64 = (XN + 63) / 64 * 64;
  constexpr int SPPI = 64 * 16 / (C * (int)sizeof(T));                // pixels per staging load
  constexpr int XSL = (XN + 4 * SPPI - 1) / (4 * SPPI) * (4 * SPPI);  // staged pixels (whole loads in every wave)
  constexpr bool DMA =
      std::is_same<T, float>::value && C == 16 && !LC && LDS_REST + 8 * S1Lds<C, XN64>::SIZE <= LDS_CAP;
  constexpr bool DMAB = !LC && !DMA && (sizeof(T) == 2 || C == 64) &&
                        LDS_REST + 4 * S1Lds<C, XN>::SIZE + XSL * C * (int)sizeof(T) <= LDS_CAP;
  constexpr int XNL = DMA ? XN64 : XN;
  constexpr int XT = S1Lds<C, XNL>::SIZE;
  static_assert(XT >= 4 * 9 * C + 9 * C && XT >= 4 * 256, "reduction scratch aliases the x tile");
  __shared__ float xt[XT];
  __shared__ float xt2[DMA ? XT : 1];
  __shared__ uint32_t xst[DMAB ? XSL * C * sizeof(T) / 4 : 1];
  __shared__ float ddt[S1Lds<C, DN>::SIZE];
  __shared__ float dpt[S1Lds<C, M>::SIZE];
  __shared__ float dut[S1Lds<C, M>::SIZE];
  __shared__ float qt[S1Lds<C, M>::SIZE];
  __shared__ float wp[C * C];
  __shared__ float wd[9 * C];
  // the three BN adjoints as affine maps of (du, branch value): cf[3 s + 0/1/2][c] = a, b, e with
  // grad = a du + b v + e, for s = 0 pointwise (v = p), 1 depthwise (v = d), 2 identity (v = x)
  __shared__ float cf[9 * C];
  float* sm = xt;  // used only after the tile loop
  float* red = xt + 4 * 9 * C;
  if (threadIdx.x < 3 * C) {
    const int s = threadIdx.x / C, c = threadIdx.x % C;
    const float mu = prm.stats[s][c], is = prm.stats[s][C + c], ga = prm.gamma[s][c];
    const float k0 = coef[c], ks = coef[(s + 1) * C + c];
    const float a = ga * is;
    cf[(3 * s) * C + c] = a;
    cf[(3 * s + 1) * C + c] = -a * is * ks;
    cf[(3 * s + 2) * C + c] = a * (is * ks * mu - k0);
  }
  stage1_load_weights<C, DEC>(prm.wpw, prm.wdw, wp, wd);  // ends with a barrier
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, li = lane & 15, lg = lane >> 4;
  const int c0 = (threadIdx.x % G) * 4;
  // LC: the depthwise taps and the BN-adjoint coefficients are read from LDS where they are used
  // (72 registers fewer per thread, for a third wave per SIMD); otherwise held in registers
  float wr[LC ? 1 : 9][4];
  float cfr[LC ? 1 : 9][4];  // this thread's 4 channels of the 9 coefficient rows
  if constexpr (!LC) {
    s1_dw_regs<C>(wd, c0, wr);
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const float4 t = *reinterpret_cast<const float4*>(cf + q * C + c0);
      cfr[q][0] = t.x;
      cfr[q][1] = t.y;
      cfr[q][2] = t.z;
      cfr[q][3] = t.w;
    }
  }
  auto W4 = [&](int t) {
    if constexpr (LC) return *reinterpret_cast<const float4*>(wd + t * C + c0);
    else return make_float4(wr[t][0], wr[t][1], wr[t][2], wr[t][3]);
  };
  auto CF4 = [&](int q) {
    if constexpr (LC) return *reinterpret_cast<const float4*>(cf + q * C + c0);
    else return make_float4(cfr[q][0], cfr[q][1], cfr[q][2], cfr[q][3]);
  };
  float dwacc[9][4];
#pragma unroll
  for (int t = 0; t < 9; ++t) zero4(dwacc[t]);
  floatx4_t pwacc[NTW];
#pragma unroll
  for (int u = 0; u < NTW; ++u) pwacc[u] = floatx4_t{0.f, 0.f, 0.f, 0.f};
  auto xpx = [&](int p) { return (p / TW + 2) * XW + p % TW + 2; };  // tile pixel -> x-tile LDS pixel

  const int ntiles = B * ((h + TH - 1) / TH) * ((w + TW - 1) / TW);
  // Tile loop.  With DMA a tile's x was fetched during the previous tile (or before the loop) and
  // the next tile's is fetched into the other buffer during this one: two tiles per iteration, the
  // first in xt, the second in xt2, unrolled so that each copy names its buffers and reads of the
  // current one do not wait for the loads into the other.
  if constexpr (DMA || DMAB)
    if (bx < ntiles) {
      int b, y0, x0;
      tile_coords(bx, h, w, TH, TW, b, y0, x0);
      if constexpr (DMA) load_tile_dma<C, TH, TW, 2, XNL>(X, b, y0, x0, h, w, xt);
      else load_tile_dma_raw<T, C, TH, TW, 2, XSL>(X, b, y0, x0, h, w, xst);
    }
  constexpr int NU = DMA ? 2 : 1;
  for (int tile0 = bx; tile0 < ntiles; tile0 += NU * gx)
#pragma unroll
  for (int half = 0; half < NU; ++half) {
    const int tile = tile0 + half * gx;
    if (half > 0 && tile >= ntiles) break;
    float* const xc = half ? xt2 : xt;   // this tile's x
    float* const xnx = half ? xt : xt2;  // the next tile's (DMA)
    (void)xnx;
    int b, y0, x0;
    tile_coords(tile, h, w, TH, TW, b, y0, x0);
    // the ReLU decisions and dx1 of the thread's dD-phase items (zero off the map), loaded ahead:
    // BF16 at 16 channels all of them (at most 3) at the tile start, so that their latencies
    // overlap each other, the staging and the first product (measured faster there; FP32, whose
    // x tile is already fetched a tile ahead, gained nothing for 16 more registers); otherwise one
    // item ahead, the first item's loads overlapping the staging and the first product, each later
    // one the previous item.  Not at 64 channels, whose tiles have no registers to spare: there
    // each item loads its own.
    constexpr int NA = (TH + 2) * DWd * G, NAI = (NA + STDA_BLOCK - 1) / STDA_BLOCK;
    constexpr bool PF = C < 64 && !LC;  // (LC: registers go to a third wave instead)
    constexpr bool PALL = PF && C == 16 && NAI <= 3 && sizeof(T) == 2;
    constexpr int NPF = PALL ? NAI : 1, NUNR = PALL ? NAI : 1;
    typedef typename Raw4<T>::type R4;  // held in storage form until used
    R4 ng[NPF];
    uint32_t nm[NPF];  // the byte of M1 holding this thread's 4 decisions
    // loaded ahead by buffer loads over this clip, which read 0 off the map: no branch around
    // them, so every thread issues the same loads and a wait for one item's operands need not
    // wait for the later items'
    const int64_t cpx = (int64_t)b * h * w;  // the clip's first pixel
    const __amdgpu_buffer_rsrc_t rm1 = __builtin_amdgcn_make_buffer_rsrc(const_cast<uint8_t*>(M1 + cpx * (C / 8)),
                                                                         (short)0, h * w * (C / 8), 0x00020000);
    const __amdgpu_buffer_rsrc_t rdx1 = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(dX1 + cpx * C), (short)0,
                                                                          h * w * C * (int)sizeof(T), 0x00020000);
    auto a2_load = [&](int e, int k) {
      const int px = e / G, y = y0 - 1 + px / DWd, x = x0 - 1 + px % DWd;
      const bool in = e < NA && y >= 0 && y < h && x >= 0 && x < w;
      const int off = (y * w + x) * C + c0;  // element offset in the clip
      // byte (pixel, c0 / 8) of the mask: C / 8 bytes per pixel
      nm[k] = __builtin_amdgcn_raw_buffer_load_b8(rm1, in ? off >> 3 : (int)0x80000000u, 0, 0);
      raw_bld4(rdx1, in ? off * (int)sizeof(T) : (int)0x80000000u, ng[k]);
    };
    auto a2_first = [&]() {
#pragma unroll
      for (int k = 0; k < NPF; ++k) a2_load(threadIdx.x + k * STDA_BLOCK, k);
    };
    if constexpr (DMA) {
      wait_vmem();  // this wave's part of the tile is in LDS
      if constexpr (PF) a2_first();
      __syncthreads();  // and every other wave's
    } else if constexpr (DMAB) {
      wait_vmem();  // this wave's part of the staged tile is in LDS
      if constexpr (PF) a2_first();
      __syncthreads();  // and every other wave's
      stage1_put_raw<T, C, XN, XNL>(xst, xc);
      __syncthreads();
    } else {
      if constexpr (PF) a2_first();
      __syncthreads();
      load_tile<T, C, TH, TW, 2, !LC>(X, b, y0, x0, h, w, xc);  // LC: one load at a time (register peak)
      __syncthreads();
    }
    // A1: pointwise branch of the tile, qt = x Wp
    lds_gemm_s<M, C, C>([&](int p, int kk) { return xc[s1e<C, XNL>(xpx(p), kk)]; },
                        [&](int kk, int n) { return wp[kk * C + n]; },
                        [&](int p, int n, float v) { qt[s1e<C, M>(p, n)] = v; });
    __syncthreads();
    // A2: dD on the tile + halo 1, dP on the tile (zero off the map)
#pragma unroll NUNR
    for (int i = 0; i < NAI; ++i) {
      const int e = threadIdx.x + i * STDA_BLOCK;
      if (e >= NA) break;
      const int px = e / G, r = px / DWd, cc = px % DWd;  // position in the dD tile
      const int y = y0 - 1 + r, x = x0 - 1 + cc;
      const bool center = r >= 1 && r <= TH && cc >= 1 && cc <= TW;
      float g[4];
      uint32_t m;
      if constexpr (PF) {
        m = nm[PALL ? i : 0];
        raw_cvt4(ng[PALL ? i : 0], g);
        if constexpr (!PALL)
          if (e + STDA_BLOCK < NA) a2_load(e + STDA_BLOCK, 0);
      }
      float od[4], op[4], uv[4];
      zero4(od);
      zero4(op);
      zero4(uv);
      if (y >= 0 && y < h && x >= 0 && x < w) {
        if constexpr (!PF) {
          const int64_t off = (((int64_t)b * h + y) * w + x) * C + c0;
          m = M1[off >> 3];
          ld4(dX1 + off, g);
        }
        m >>= (c0 & 4);
        float dv[4];
        float4 xn[9];
        zero4(dv);
#pragma unroll
        for (int t = 0; t < 9; ++t) {
          xn[t] = s1_nbr<C, XNL>(xc, r * XW + cc, c0 >> 2, (t / 3) * XW + t % 3);
          const float4 w4 = W4(t);
          dv[0] += w4.x * xn[t].x;
          dv[1] += w4.y * xn[t].y;
          dv[2] += w4.z * xn[t].z;
          dv[3] += w4.w * xn[t].w;
        }
        float pv[4] = {0.f, 0.f, 0.f, 0.f};
        if (center) {
          const float4 pq = *reinterpret_cast<const float4*>(qt + s1c<C, M>((r - 1) * TW + cc - 1, c0 >> 2));
          pv[0] = pq.x;
          pv[1] = pq.y;
          pv[2] = pq.z;
          pv[3] = pq.w;
        }
        const float4 pa4 = CF4(0), pb4 = CF4(1), pe4 = CF4(2), da4 = CF4(3), db4 = CF4(4), de4 = CF4(5);
        const float pa[4] = {pa4.x, pa4.y, pa4.z, pa4.w}, pb[4] = {pb4.x, pb4.y, pb4.z, pb4.w};
        const float pe[4] = {pe4.x, pe4.y, pe4.z, pe4.w}, da[4] = {da4.x, da4.y, da4.z, da4.w};
        const float db[4] = {db4.x, db4.y, db4.z, db4.w}, de[4] = {de4.x, de4.y, de4.z, de4.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float du = (m >> j) & 1u ? g[j] : 0.f;
          uv[j] = du;
          od[j] = da[j] * du + db[j] * dv[j] + de[j];
          op[j] = pa[j] * du + pb[j] * pv[j] + pe[j];
        }
        if (center)  // depthwise weight gradient: x(q + off_t) dD(q) over the tile's pixels q
#pragma unroll
          for (int t = 0; t < 9; ++t) {
            dwacc[t][0] += xn[t].x * od[0];
            dwacc[t][1] += xn[t].y * od[1];
            dwacc[t][2] += xn[t].z * od[2];
            dwacc[t][3] += xn[t].w * od[3];
          }
      }
      *reinterpret_cast<float4*>(ddt + s1c<C, DN>(px, c0 >> 2)) = make_float4(od[0], od[1], od[2], od[3]);
      if (center) {
        const int cp = s1c<C, M>((r - 1) * TW + cc - 1, c0 >> 2);
        *reinterpret_cast<float4*>(dpt + cp) = make_float4(op[0], op[1], op[2], op[3]);
        *reinterpret_cast<float4*>(dut + cp) = make_float4(uv[0], uv[1], uv[2], uv[3]);
      }
    }
    // dXr and the skip gradient of the thread's next dX-phase pixel pair (below 64 channels), one
    // pair ahead: the first pair's loads overlap the two products that follow
    constexpr int NB2 = (M / 2) * G;
    R4 nr[2], ns[2];
    const __amdgpu_buffer_rsrc_t rdxr = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(dXr + cpx * C), (short)0,
                                                                          h * w * C * (int)sizeof(T), 0x00020000);
    const __amdgpu_buffer_rsrc_t rskp = __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(SKIP ? skip + cpx * C : dXr),
                                                                          (short)0, h * w * C * (int)sizeof(T), 0x00020000);
    auto b2_load = [&](int e) {  // buffer loads as above
      const int px = 2 * (e / G), y = y0 + px / TW, x = x0 + px % TW;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const bool in = e < NB2 && y < h && x + s < w;
        const int off = in ? ((y * w + x + s) * C + c0) * (int)sizeof(T) : (int)0x80000000u;
        raw_bld4(rdxr, off, nr[s]);
        if (SKIP) raw_bld4(rskp, off, ns[s]);
        else raw_zero4(ns[s]);
      }
    };
    constexpr bool PF2 = !LC;  // dX phase: load one pair ahead (else each pair loads its own)
    if constexpr (C < 64 && PF2) b2_load(threadIdx.x);
    __syncthreads();
    // B1: pointwise transpose, qt[p][c] = sum_o dP[p][o] wp[c][o]
    lds_gemm_s<M, C, C>([&](int p, int o) { return dpt[s1e<C, M>(p, o)]; }, [&](int o, int n) { return wp[n * C + o]; },
                        [&](int p, int n, float v) { qt[s1e<C, M>(p, n)] = v; });
    if constexpr (DMA || DMAB) {
      // the next tile's x, into the other buffer (DMAB: the staging buffer, free once this tile's
      // x was converted), in flight until that tile starts (after the last tile this tile again,
      // never read: every path issues the same loads, so waits for loads issued before them need
      // not wait for these).  Issued after this tile's last LDS writes, which would otherwise wait
      // for them.
      int nb, ny0, nx0;
      tile_coords(tile + gx < ntiles ? tile + gx : tile, h, w, TH, TW, nb, ny0, nx0);
      if constexpr (DMA) load_tile_dma<C, TH, TW, 2, XNL>(X, nb, ny0, nx0, h, w, xnx);
      else load_tile_dma_raw<T, C, TH, TW, 2, XSL>(X, nb, ny0, nx0, h, w, xst);
    }
    // C: pointwise weight gradient, dWp[c][o] += sum_p x[p][c] dP[p][o] (registers, across tiles);
    // with a single 16 x 16 tile (16 channels) the 4 waves take a quarter of the pixels each
    if constexpr (NT == 1) {
      constexpr int MQ = M / 4;
      const int pb = wave * MQ;
#pragma unroll 4
      for (int p = 0; p < MQ; p += 4)
        pwacc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(xc[s1e<C, XNL>(xpx(pb + p + lg), li)], dpt[s1e<C, M>(pb + p + lg, li)],
                                                        pwacc[0], 0, 0, 0);
    } else {
#pragma unroll
      for (int u = 0; u < NTW; ++u) {
        const int t = wave + 4 * u;
        if (t < NT) {
          const int m0 = (t / (C / 16)) * 16, n0 = (t % (C / 16)) * 16;
#pragma unroll 4
          for (int p = 0; p < M; p += 4)
            pwacc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(xc[s1e<C, XNL>(xpx(p + lg), m0 + li)],
                                                            dpt[s1e<C, M>(p + lg, n0 + li)], pwacc[u], 0, 0, 0);
        }
      }
    }
    if constexpr (DMA || DMAB) lds_barrier();
    else __syncthreads();
    // B2: dX on the tile.  C < 64: two horizontally adjacent pixels per item, whose 3 x 3
    // neighbourhoods of dD share 6 of the 12 values read; C = 64 keeps one pixel per item, since the
    // pair does not fit its register budget.
    if constexpr (C < 64) {
      static_assert(TW % 2 == 0, "pixel pairs inside a tile row");
      for (int e = threadIdx.x; e < NB2; e += STDA_BLOCK) {
        const int px = 2 * (e / G), r = px / TW, cc = px % TW;  // pixels px, px + 1 of tile row r
        const int y = y0 + r, x = x0 + cc;
        float rp[2][4], sp2[2][4];
        if constexpr (!PF2) b2_load(e);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          raw_cvt4(nr[s], rp[s]);
          raw_cvt4(ns[s], sp2[s]);
        }
        if constexpr (PF2)
          if (e + STDA_BLOCK < NB2) b2_load(e + STDA_BLOCK);
        if (y >= h || x >= w) continue;
        const bool second = x + 1 < w;
        const int64_t off = (((int64_t)b * h + y) * w + x) * C + c0;
        float acc[2][4];
        const float4 xa4 = CF4(6), xb4 = CF4(7), xe4 = CF4(8);
        const float xa[4] = {xa4.x, xa4.y, xa4.z, xa4.w}, xb[4] = {xb4.x, xb4.y, xb4.z, xb4.w};
        const float xe[4] = {xe4.x, xe4.y, xe4.z, xe4.w};
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          if (s == 1 && !second) break;
          const float* rr = rp[s];
          const float4 xq = *reinterpret_cast<const float4*>(xc + s1c<C, XNL>(xpx(px + s), c0 >> 2));
          const float4 qc = *reinterpret_cast<const float4*>(qt + s1c<C, M>(px + s, c0 >> 2));
          const float4 uc = *reinterpret_cast<const float4*>(dut + s1c<C, M>(px + s, c0 >> 2));
          const float xv[4] = {xq.x, xq.y, xq.z, xq.w}, qv[4] = {qc.x, qc.y, qc.z, qc.w}, du[4] = {uc.x, uc.y, uc.z, uc.w};
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[s][j] = xa[j] * du[j] + xb[j] * xv[j] + xe[j] + rr[j] + qv[j];
          if (SKIP)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[s][j] += sp2[s][j];
        }
        // depthwise transpose: dx[c](q) += sum_t dD[c](q - off_t) wd[t][c]; dD is 0 off the map.
        // Row dy of the pair reads dD tile columns cc .. cc + 3 (k = 0..3); the first pixel takes
        // column k with tap dx = 1 - k, the second with dx = 2 - k (taps in the order t = 0..8).
#pragma unroll
        for (int dyi = 0; dyi < 3; ++dyi) {
          const int dy = dyi - 1;
          float4 col[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) col[k] = s1_nbr<C, DN>(ddt, r * DWd + cc, c0 >> 2, (1 - dy) * DWd + k);
#pragma unroll
          for (int k = 2; k >= 0; --k) {
            const float4 w4 = W4(dyi * 3 + 2 - k);
            acc[0][0] += w4.x * col[k].x;
            acc[0][1] += w4.y * col[k].y;
            acc[0][2] += w4.z * col[k].z;
            acc[0][3] += w4.w * col[k].w;
          }
#pragma unroll
          for (int k = 3; k >= 1; --k) {
            const float4 w4 = W4(dyi * 3 + 3 - k);
            acc[1][0] += w4.x * col[k].x;
            acc[1][1] += w4.y * col[k].y;
            acc[1][2] += w4.z * col[k].z;
            acc[1][3] += w4.w * col[k].w;
          }
        }
        st4(dX + off, acc[0]);
        if (second) st4(dX + off + C, acc[1]);
      }
    } else {
      for (int e = threadIdx.x; e < M * G; e += STDA_BLOCK) {
        const int px = e / G, r = px / TW, cc = px % TW;
        const int y = y0 + r, x = x0 + cc;
        if (y >= h || x >= w) continue;
        const int64_t off = (((int64_t)b * h + y) * w + x) * C + c0;
        float rr[4], acc[4];
        ld4(dXr + off, rr);
        const float4 xq = *reinterpret_cast<const float4*>(xc + s1c<C, XNL>(xpx(px), c0 >> 2));
        const float4 qc = *reinterpret_cast<const float4*>(qt + s1c<C, M>(px, c0 >> 2));
        const float4 uc = *reinterpret_cast<const float4*>(dut + s1c<C, M>(px, c0 >> 2));
        const float xv[4] = {xq.x, xq.y, xq.z, xq.w}, qv[4] = {qc.x, qc.y, qc.z, qc.w}, du[4] = {uc.x, uc.y, uc.z, uc.w};
        const float4 xa4 = CF4(6), xb4 = CF4(7), xe4 = CF4(8);
        const float xa[4] = {xa4.x, xa4.y, xa4.z, xa4.w}, xb[4] = {xb4.x, xb4.y, xb4.z, xb4.w};
        const float xe[4] = {xe4.x, xe4.y, xe4.z, xe4.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = xa[j] * du[j] + xb[j] * xv[j] + xe[j] + rr[j] + qv[j];
        if (SKIP) {
          float sv[4];
          ld4(skip + off, sv);
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[j] += sv[j];
        }
        // depthwise transpose: dx[c](q) += sum_t dD[c](q - off_t) wd[t][c]; dD is 0 off the map
#pragma unroll
        for (int t = 0; t < 9; ++t) {
          const int dy = t / 3 - 1, dx = t % 3 - 1;
          const float4 v = *reinterpret_cast<const float4*>(ddt + s1c<C, DN>((r + 1 - dy) * DWd + cc + 1 - dx, c0 >> 2));
          const float4 w4 = W4(t);
          acc[0] += w4.x * v.x;
          acc[1] += w4.y * v.y;
          acc[2] += w4.z * v.z;
          acc[3] += w4.w * v.w;
        }
        st4(dX + off, acc);
      }
    }
  }
  if constexpr (DMA || DMAB) wait_vmem();  // the last (unused) fetch has landed
  __syncthreads();
  block_chan_reduce_shfl<G, 9>(dwacc, sm, red);
  for (int q = threadIdx.x; q < 9 * C; q += STDA_BLOCK) {
    const int t = q / C, c = q % C;
    const int tw = DEC ? 8 - t : t;
    dwpart[(int64_t)bx * 9 * C + tw * C + c] = red[q];
  }
  // pointwise gradient tile (m0, n0): lane holds D[4 lg + r][li] -> (c = m0 + 4 lg + r, o = n0 + li)
  float* pw = pwpart + (int64_t)bx * C * C;
  if constexpr (NT == 1) {
    // the four waves' partial tiles, summed in wave order
    __syncthreads();  // the reduction scratch above is no longer read
#pragma unroll
    for (int r = 0; r < 4; ++r) sm[wave * 256 + (4 * lg + r) * 16 + li] = pwacc[0][r];
    __syncthreads();
    const int q = threadIdx.x;  // 256 = 16 x 16 entries
    pw[q] = ((sm[q] + sm[256 + q]) + sm[512 + q]) + sm[768 + q];
    return;
  }
  for (int t = 0; t < NT; ++t) {
    const int m0 = (t / (C / 16)) * 16, n0 = (t % (C / 16)) * 16;
#pragma unroll
    for (int u = 0; u < NTW; ++u)
      if (wave + 4 * u == t)
#pragma unroll
        for (int r = 0; r < 4; ++r) pw[(m0 + 4 * lg + r) * C + n0 + li] = pwacc[u][r];
  }
}

}  // namespace stda
