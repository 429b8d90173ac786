// Input module (Conv3x3 p1, 3 -> 16 on the channel concatenation of frames t, t-1, t-2, then BN
// and ReLU) on LDS tiles (gfx950).
//
// A block stages the three planar input maps of a TH x TW pixel tile plus a 1-pixel halo in LDS;
// the convolution is an M x 16 x 28 GEMM (M = tile pixels, k = c*9 + tap, k = 27 zero) on the
// matrix cores, reading the im2col operand straight from the staged planes.  The pre-BN output
// is never stored: every pass recomputes it.
//   MODE 0  TRAIN statistics: part[blk][16][2] = (mean, m2) of the block's conv outputs and
//           the block's count at part[blocks * 32 + blk] (blocks = the segment's workgroups)
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
struct k_stem_tile_args {
  StemArgs a;
  const T* dS;
  const T* S;
  T* out;
  int B;
  int H;
  int W;
};
template <class T, int MODE>
__global__ __launch_bounds__(256) void k_stem_tile(SegL<k_stem_tile_args<T, MODE>> L) {
  const SegB sb = seg_block(L);
  if (sb.x >= sb.gx) return;
  const int bx = sb.x, gx = sb.gx;  // workgroup index and count within the segment
  (void)gx;
  const k_stem_tile_args<T, MODE>& a_ = L.a[sb.s];
  const StemArgs& a = a_.a;
  const T* __restrict__ const dS = a_.dS;
  const T* __restrict__ const S = a_.S;
  T* __restrict__ const out = a_.out;
  const int B = a_.B;
  const int H = a_.H;
  const int W = a_.W;
  constexpr int TH = 8, TW = 32, M = TH * TW, C = 16, G = 4, PS = C + 4, XR = TH + 2, XC = TW + 2;
  constexpr int NX = 3 * XR * XC, NXL = (NX + 255) / 256 * 256;  // staged values (NXL: whole loads in every wave)
  __shared__ float xs[NXL];
  __shared__ float wk[C * 28];
  __shared__ float tt[M * PS];   // conv output of the tile (then dTp in MODE 3)
  __shared__ float sm[4 * (2 * C + 1)];
  __shared__ float red[2 * C + 1];
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
  float acc[2][4];  // MODE 2 sums; MODE 0: mean and m2 of channels c0 .. c0 + 3 (Welford)
  zero4(acc[0]);
  zero4(acc[1]);
  float cnt = 0.f;  // MODE 0: pixels seen by this thread
  // MODE 3: every wave accumulates the weight gradient of a quarter of each tile's pixels, columns
  // k = 0..15 and 16..31 (two independent chains); the waves are summed at the end
  floatx4_t wacc0 = {0.f, 0.f, 0.f, 0.f}, wacc1 = {0.f, 0.f, 0.f, 0.f};
  // offset in xs of im2col column k (channel c = k / 9, tap t = k % 9) relative to the pixel's own
  // top-left; -1 for the zero column k = 27
  auto koff_of = [](int kk) { return kk < 27 ? ((kk / 9) * XR + (kk % 9) / 3) * XC + kk % 3 : -1; };
  int koff[7];  // conv GEMM: column k = 4 s + lg of step s
#pragma unroll
  for (int s = 0; s < 7; ++s) koff[s] = koff_of(4 * s + lg);
  const int wo0 = koff_of(li), wo1 = koff_of(16 + li);  // weight gradient: columns li, 16 + li
  const int ntiles = B * ((H + TH - 1) / TH) * ((W + TW - 1) / TW);
  // MODE 0..2 (DMAX): the next tile's three planes are fetched by buffer loads that write LDS
  // directly (one value per lane, 64 consecutive values of the staged layout per load) once this
  // tile's product has read them; the fetch is in flight during this tile's items and is waited
  // for at the next tile's start.  A value off the map gets an offset past the clip's buffer range,
  // which the range check turns into 0.  (MODE 3 reads the planes again for its weight gradient.)
  constexpr bool DMAX = MODE <= 2;
  auto xs_fetch = [&](int t) {
    int fb, fy0, fx0;
    tile_coords(t, H, W, TH, TW, fb, fy0, fx0);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(a.x + (int64_t)fb * 3 * H * W),
                                                                        (short)0, 3 * H * W * 4, 0x00020000);
#pragma unroll
    for (int i = 0; i < NXL / STDA_BLOCK; ++i) {
      const int j = wave + i * (STDA_BLOCK / 64), q = j * 64 + lane;
      const int c = q / (XR * XC), r = (q / XC) % XR, cc = q % XC;
      const int y = fy0 - 1 + r, x = fx0 - 1 + cc;
      const bool in = q < NX && y >= 0 && y < H && x >= 0 && x < W;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, lds_ptr(xs + j * 64), 4, in ? ((c * H + y) * W + x) * 4 : (int)0x80000000u,
                                               0, 0, 0);
    }
  };
  if constexpr (DMAX)
    if (bx < ntiles) xs_fetch(bx);
  for (int tile = bx; tile < ntiles; tile += gx) {
    int b, y0, x0;
    tile_coords(tile, H, W, TH, TW, b, y0, x0);
    if constexpr (DMAX) wait_vmem();  // this wave's part of the planes is in LDS (before the loads below)
    // MODE 3: the three planes of the tile plus halo, loaded into registers first (then dS and S
    // below), so that writing them to LDS waits for these loads only (the product does not wait
    // for dS and S)
    constexpr int KX = (NX + STDA_BLOCK - 1) / STDA_BLOCK;
    float xv[DMAX ? 1 : KX];
    if constexpr (!DMAX) {  // buffer loads: 0 off the map, no branch around the loads
      const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(a.x + (int64_t)b * 3 * H * W),
                                                                          (short)0, 3 * H * W * 4, 0x00020000);
#pragma unroll
      for (int k = 0; k < KX; ++k) {
        const int q = threadIdx.x + k * STDA_BLOCK;
        const int c = q / (XR * XC), r = (q / XC) % XR, cc = q % XC;
        const int y = y0 - 1 + r, x = x0 - 1 + cc;
        const bool in = q < NX && y >= 0 && y < H && x >= 0 && x < W;
        xv[k] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rx, in ? ((c * H + y) * W + x) * 4 : (int)0x80000000u, 0, 0));
      }
    }
    // adjoint modes: this thread's dS and S, loaded before the staging and the GEMM so that
    // their latency overlaps them; buffer loads (0 off the map), so that every thread issues the
    // same loads and the planes' wait above need not wait for these
    constexpr int KI = M * G / STDA_BLOCK;
    static_assert(M * G % STDA_BLOCK == 0, "whole items per thread");
    typename Raw4<T>::type pg[KI], ps[KI];  // storage form: converted where used
    if constexpr (MODE >= 2) {
      const int cb = H * W * C * (int)sizeof(T);  // bytes of one clip (at most 1 GiB here)
      const __amdgpu_buffer_rsrc_t rg =
          __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(dS + (int64_t)b * H * W * C), (short)0, cb, 0x00020000);
      const __amdgpu_buffer_rsrc_t rsv =
          __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(S + (int64_t)b * H * W * C), (short)0, cb, 0x00020000);
#pragma unroll
      for (int k = 0; k < KI; ++k) {
        const int px = (threadIdx.x + k * STDA_BLOCK) / G, y = y0 + px / TW, x = x0 + px % TW;
        const int off = y < H && x < W ? ((y * W + x) * C + c0) * (int)sizeof(T) : (int)0x80000000u;
        raw_bld4(rg, off, pg[k]);
        raw_bld4(rsv, off, ps[k]);
      }
    }
    __syncthreads();  // the previous tile's readers of xs and tt are done
    if constexpr (!DMAX) {
#pragma unroll
      for (int k = 0; k < KX; ++k) {
        const int q = threadIdx.x + k * STDA_BLOCK;
        if (q < NX) xs[q] = xv[k];
      }
      __syncthreads();
    }
    {
      // conv GEMM tt[p][o] = sum_k im2col(p, k) w[o][k] on the matrix cores: wave w takes the
      // 16-pixel row tiles w, w + 4, w + 8, w + 12, as NCH independent chains at a time (four in
      // the forward modes; one in the adjoint modes, whose registers already hold dS and S)
      constexpr int NCH = MODE < 2 ? 4 : 1;
#pragma unroll 1
      for (int t0 = wave; t0 < M / 16; t0 += 4 * NCH) {
        floatx4_t cacc[NCH];
        int pbase[NCH];
#pragma unroll
        for (int u = 0; u < NCH; ++u) {
          const int p = 16 * (t0 + 4 * u) + li;
          pbase[u] = (p / TW) * XC + p % TW;
          cacc[u] = floatx4_t{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int s = 0; s < 7; ++s) {
          const float bv = wk[li * 28 + 4 * s + lg];
#pragma unroll
          for (int u = 0; u < NCH; ++u)
            cacc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(koff[s] >= 0 ? xs[koff[s] + pbase[u]] : 0.f, bv, cacc[u], 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < NCH; ++u)
#pragma unroll
          for (int r = 0; r < 4; ++r) tt[(16 * (t0 + 4 * u) + 4 * lg + r) * PS + li] = cacc[u][r];
      }
    }
    __syncthreads();
    if constexpr (DMAX) xs_fetch(tile + gx < ntiles ? tile + gx : tile);  // (after the last tile: unused)
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
        cnt += 1.f;
        const float rk = __builtin_amdgcn_rcpf(cnt);
#pragma unroll
        for (int j = 0; j < 4; ++j) wf_add(acc[0][j], acc[1][j], t[j], rk);
      } else if (MODE == 1) {
        if (!in) continue;
        float o[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) o[j] = fmaxf(t[j] * sc[j] + sh[j], 0.f);
        st4(out + off, o);
      } else {
        float g[4], s[4];
        raw_cvt4(pg[k], g);
        raw_cvt4(ps[k], s);
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
      // dW[o][k] += sum_p dTp[p][o] im2col(p, k) over this wave's quarter of the pixels
      const int pb = wave * (M / 4);
#pragma unroll 4
      for (int p = 0; p < M / 4; p += 4) {
        const int q = pb + p + lg, qb = (q / TW) * XC + q % TW;
        const float av = tt[q * PS + li];
        wacc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, xs[wo0 + qb], wacc0, 0, 0, 0);
        wacc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, wo1 >= 0 ? xs[wo1 + qb] : 0.f, wacc1, 0, 0, 0);
      }
    }
  }
  if constexpr (DMAX) wait_vmem();  // the last (unused) fetch has landed
  if (MODE == 0) {
    float mn[1][4], q2[1][4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      mn[0][j] = acc[0][j];
      q2[0][j] = acc[1][j];
    }
    block_chan_stats<G, 1>(cnt, mn, q2, sm, red);
    for (int q = threadIdx.x; q < 2 * C; q += STDA_BLOCK) {
      const int s = q / C, c = q % C;  // red: [mean 16][m2 16] -> part [16][2]
      a.part[(int64_t)bx * 2 * C + c * 2 + s] = red[q];
    }
    if (threadIdx.x == 0) a.part[(int64_t)gx * 2 * C + bx] = red[2 * C];
  }
  if (MODE == 2) {
    block_chan_reduce_shfl<G, 2>(acc, sm, red);
    for (int q = threadIdx.x; q < 2 * C; q += STDA_BLOCK) a.part[(int64_t)bx * 2 * C + q] = red[q];  // [2][16]
  }
  if (MODE == 3) {
    // lane holds D[4 lg + r][li] = dW[o = 4 lg + r][k = li (wacc0) | 16 + li (wacc1)]; the four
    // waves' tiles meet in LDS (aliasing tt) and are summed in wave order
    static_assert(4 * 2 * 256 <= M * PS, "wave partials fit the tile buffer");
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      tt[((wave * 2 + 0) * 16 + 4 * lg + r) * 16 + li] = wacc0[r];
      tt[((wave * 2 + 1) * 16 + 4 * lg + r) * 16 + li] = wacc1[r];
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 2 * 256; q += STDA_BLOCK) {
      const int hf = q / 256, o = (q / 16) % 16, ki = q % 16, kk = 16 * hf + ki;
      auto wv = [&](int w) { return tt[((w * 2 + hf) * 16 + o) * 16 + ki]; };
      const float v = ((wv(0) + wv(1)) + wv(2)) + wv(3);
      if (kk < 27) a.part[(int64_t)bx * 27 * C + kk * C + o] = v;
    }
  }
}

}  // namespace stda
