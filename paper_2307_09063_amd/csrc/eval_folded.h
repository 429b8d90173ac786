// Folded-weight EVAL inference of Radar-STDA (gfx950).
//
// In EVAL mode every batch normalisation is a fixed per-channel affine map x -> a x + b with
// a = gamma / sqrt(var + eps) and b = beta - mean a (running statistics).  Folding them into the
// adjacent weights (the re-parameterisation the mobile block of Sec. IV-C inherits from
// MobileOne) leaves, per block,
//   stage 1:  x1 = ReLU(PW'(x) + DW'(x) + b1),  PW' = a_p PW + diag(a_x),  DW' = a_d DW,
//             b1 = b_p + b_d + b_x  (the identity branch becomes the diagonal of the 1x1 weight);
//   stage 2:  y  = ReLU(conv'(x1) + b_m) + conv_res(x),  conv' = a_m conv (per output channel);
// and the input module s0 = ReLU(conv'(x) + b').  k_fold_eval writes the folded parameters into
// a vector of the flat parameter layout (the batch-norm scales set to 1 and the shifts to the
// folded biases), so that the input-module and stage-1 kernels run on it with identity
// statistics; k_s2_eval runs all of stage 2 as one launch.
#pragma once
#include "dense_mfma.h"

namespace stda {

// Jobs of k_fold_eval (blockIdx.x): 0 the input module; 1..4 stage 1 of block k; 5..8 the stage-2
// main convolution of block k; 9 the identity statistics ([mean 0][invstd 1] for 16, 32 and 64
// channels, back to back).  wf must already hold a copy of w (the entries not listed keep it).
struct FoldArgs {
  NetOffsets no;
  int cin[4], cout[4], dec[4];
  int64_t ids;  // element offset of the identity statistics in wf's buffer
};

__device__ __forceinline__ void bn_fold(const float* __restrict__ w, const float* __restrict__ running,
                                        int64_t g_off, int64_t b_off, int64_t bn_off, int C, int c, float& a,
                                        float& b) {
  const float mu = running[bn_off + c], var = running[bn_off + C + c];
  a = w[g_off + c] / sqrtf(var + BN_EPS);
  b = w[b_off + c] - mu * a;
}

__global__ __launch_bounds__(256) void k_fold_eval(const float* __restrict__ w, const float* __restrict__ running,
                                                   float* __restrict__ wf, FoldArgs fa) {
  const int job = blockIdx.x;
  const NetOffsets& no = fa.no;
  if (job == 0) {
    for (int i = threadIdx.x; i < 16 * 27; i += blockDim.x) {
      float a, b;
      bn_fold(w, running, no.stem_g, no.stem_b, 0, 16, i / 27, a, b);
      wf[no.stem_w + i] = w[no.stem_w + i] * a;
    }
    for (int o = threadIdx.x; o < 16; o += blockDim.x) {
      float a, b;
      bn_fold(w, running, no.stem_g, no.stem_b, 0, 16, o, a, b);
      wf[no.stem_g + o] = 1.f;
      wf[no.stem_b + o] = b;
    }
  } else if (job <= 4) {
    const int k = job - 1, C = fa.cin[k], dec = fa.dec[k];
    const BlockOffsets& bo = no.blk[k];
    // 1x1: encoder weight [out][in], decoder (transposed) [in][out]; output channel o
    for (int i = threadIdx.x; i < C * C; i += blockDim.x) {
      const int r = i / C, q = i % C, o = dec ? q : r;
      float ap, bp, ax, bx;
      bn_fold(w, running, bo.pw_g, bo.pw_b, bo.bn_pw, C, o, ap, bp);
      bn_fold(w, running, bo.id_g, bo.id_b, bo.bn_id, C, o, ax, bx);
      wf[bo.pw_w + i] = w[bo.pw_w + i] * ap + (r == q ? ax : 0.f);
    }
    for (int i = threadIdx.x; i < 9 * C; i += blockDim.x) {  // depthwise [C][1][3][3]
      float ad, bd;
      bn_fold(w, running, bo.dw_g, bo.dw_b, bo.bn_dw, C, i / 9, ad, bd);
      wf[bo.dw_w + i] = w[bo.dw_w + i] * ad;
    }
    for (int c = threadIdx.x; c < C; c += blockDim.x) {
      float ap, bp, ad, bd, ax, bx;
      bn_fold(w, running, bo.pw_g, bo.pw_b, bo.bn_pw, C, c, ap, bp);
      bn_fold(w, running, bo.dw_g, bo.dw_b, bo.bn_dw, C, c, ad, bd);
      bn_fold(w, running, bo.id_g, bo.id_b, bo.bn_id, C, c, ax, bx);
      wf[bo.pw_g + c] = 1.f;
      wf[bo.dw_g + c] = 1.f;
      wf[bo.id_g + c] = 0.f;  // the identity branch lives in the 1x1 weight's diagonal
      wf[bo.pw_b + c] = bp + bd + bx;
      wf[bo.dw_b + c] = 0.f;
      wf[bo.id_b + c] = 0.f;
    }
  } else if (job <= 8) {
    const int k = job - 5, Ci = fa.cin[k], Co = fa.cout[k], dec = fa.dec[k];
    const BlockOffsets& bo = no.blk[k];
    const int taps = dec ? 16 : 9;
    // encoder [Cout][Cin][3][3], decoder (transposed) [Cin][Cout][4][4]
    for (int i = threadIdx.x; i < Ci * Co * taps; i += blockDim.x) {
      const int o = dec ? (i / taps) % Co : i / (Ci * taps);
      float a, b;
      bn_fold(w, running, bo.main_g, bo.main_b, bo.bn_main, Co, o, a, b);
      wf[bo.main_w + i] = w[bo.main_w + i] * a;
    }
    for (int o = threadIdx.x; o < Co; o += blockDim.x) {
      float a, b;
      bn_fold(w, running, bo.main_g, bo.main_b, bo.bn_main, Co, o, a, b);
      wf[bo.main_g + o] = 1.f;
      wf[bo.main_b + o] = b;
    }
  } else {
    float* ids = wf + fa.ids;
    for (int i = threadIdx.x; i < 2 * (16 + 32 + 64); i += blockDim.x) {
      // [0 x16][1 x16][0 x32][1 x32][0 x64][1 x64]
      const int seg = i < 32 ? 0 : (i < 96 ? 1 : 2), base = seg == 0 ? 0 : (seg == 1 ? 32 : 96);
      const int C = 16 << seg;
      ids[i] = (i - base) < C ? 0.f : 1.f;
    }
  }
}

// Element offset of the [mean 0][invstd 1] identity statistics of width C in the block above.
__host__ __device__ constexpr int fold_ids_off(int C) { return C == 16 ? 0 : (C == 32 ? 32 : 96); }
constexpr int kFoldIds = 2 * (16 + 32 + 64);

// Stage 2 of a folded mobile block:  y = ReLU(conv'(x1) + bias) + conv_res(x),  stored in the
// storage type, and per (clip, phase, row tile) channel sums of the stored y for the ECA average:
// gap[((clip * PH + phase) * tiles + tile) * N + n].  The two convolutions have the same
// geometry (x1 and x have the same width and map size), so each tap's A-fragment address serves
// both sources; the wave keeps two accumulator chains.  One wave computes 16 R rows of one clip's
// output (phase) grid with all N output channels; grid (clips x row tiles, phases).  Weights in
// MFMA fragment order as for k_dense_mfma.
template <class T, int OP, int K, int N, int R>
struct k_s2_eval_args {
  const T* x1;
  const T* x;
  const T* wmain;
  const T* wres;
  const float* bias;
  T* y;
  float* gap;
  int hd;
  int wd;
  int tiles;
};
template <class T, int OP, int K, int N, int R>
__global__ __launch_bounds__(256) void k_s2_eval(SegL<k_s2_eval_args<T, OP, K, N, R>> L) {
  const SegB sb = seg_block(L);
  if (sb.x >= sb.gx) return;
  const int bx = sb.x, gx = sb.gx;  // workgroup index and count within the segment
  (void)gx;
  const k_s2_eval_args<T, OP, K, N, R>& a_ = L.a[sb.s];
  const T* __restrict__ const x1 = a_.x1;
  const T* __restrict__ const x = a_.x;
  const T* __restrict__ const wmain = a_.wmain;
  const T* __restrict__ const wres = a_.wres;
  const float* __restrict__ const bias = a_.bias;
  T* __restrict__ const y = a_.y;
  float* __restrict__ const gap = a_.gap;
  const int hd = a_.hd;
  const int wd = a_.wd;
  const int tiles = a_.tiles;
  typedef typename FragT<T>::type F;
  constexpr int KS = OpGeo<OP>::KS;
  constexpr bool DOWN = OpGeo<OP>::DOWN;
  constexpr int NT = N / 16, KC = K / 16;
  constexpr bool PAIR2 = sizeof(T) == 2 && KC % 2 == 0;
  __shared__ float sm[4][N];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, m = lane & 15, g = lane >> 4;
  const int ph = blockIdx.y, py = DOWN ? 0 : ph >> 1, px = DOWN ? 0 : ph & 1;
  const int b = bx / tiles, tx = bx - b * tiles;  // clip, row tile of the clip
  const int hr = DOWN ? hd : hd / 2, wr = DOWN ? wd : wd / 2;  // the clip's GEMM row grid
  const int hs = DOWN ? 2 * hd : hd / 2, ws = DOWN ? 2 * wd : wd / 2;
  const int64_t Pc = (int64_t)hr * wr;
  const F* wm = reinterpret_cast<const F*>(wmain);
  const F* wq = reinterpret_cast<const F*>(wres);
  const int64_t pbase = ((int64_t)tx * 4 + wave) * 16 * R;
  int prow[R], pcol[R];
  bool pv[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int64_t p = pbase + 16 * r + m;
    pv[r] = p < Pc;
    prow[r] = pv[r] ? (int)(p / wr) : 0;
    pcol[r] = pv[r] ? (int)(p % wr) : 0;
  }
  floatx4 am[R][NT], ar[R][NT];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) am[r][nt] = ar[r][nt] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int a = 0; a < (DOWN ? KS : 2); ++a) {
    const int ky = DOWN ? a : ((py + 1) & 1) + 2 * a;
    if (ky >= KS) continue;
#pragma unroll
    for (int c = 0; c < (DOWN ? KS : 2); ++c) {
      const int kx = DOWN ? c : ((px + 1) & 1) + 2 * c;
      if (kx >= KS) continue;
      const int tap = ky * KS + kx;
      int64_t so[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int sy = DOWN ? 2 * prow[r] - 1 + ky : (2 * prow[r] + py + 1 - ky) / 2;
        const int sx = DOWN ? 2 * pcol[r] - 1 + kx : (2 * pcol[r] + px + 1 - kx) / 2;
        const bool ok = pv[r] && sy >= 0 && sy < hs && sx >= 0 && sx < ws;
        so[r] = ok ? (((int64_t)b * hs + sy) * ws + sx) * K + 4 * g : -1;
      }
      if constexpr (PAIR2) {
#pragma unroll
        for (int s = 0; s < KC; s += 2) {
          bf16x8 a1[R], a2[R];
#pragma unroll
          for (int r = 0; r < R; ++r) {
            a1[r] = so[r] >= 0 ? pack8(*reinterpret_cast<const F*>(x1 + so[r] + 16 * s),
                                       *reinterpret_cast<const F*>(x1 + so[r] + 16 * s + 16))
                               : pack8(frag_zero<F>(), frag_zero<F>());
            a2[r] = so[r] >= 0 ? pack8(*reinterpret_cast<const F*>(x + so[r] + 16 * s),
                                       *reinterpret_cast<const F*>(x + so[r] + 16 * s + 16))
                               : pack8(frag_zero<F>(), frag_zero<F>());
          }
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const int i0 = ((tap * KC + s) * NT + nt) * 64 + lane, i1 = ((tap * KC + s + 1) * NT + nt) * 64 + lane;
            const bf16x8 bm = pack8(wm[i0], wm[i1]), bq = pack8(wq[i0], wq[i1]);
#pragma unroll
            for (int r = 0; r < R; ++r) {
              am[r][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[r], bm, am[r][nt], 0, 0, 0);
              ar[r][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[r], bq, ar[r][nt], 0, 0, 0);
            }
          }
        }
      } else {
#pragma unroll
        for (int s = 0; s < KC; ++s) {
          F a1[R], a2[R];
#pragma unroll
          for (int r = 0; r < R; ++r) {
            a1[r] = so[r] >= 0 ? *reinterpret_cast<const F*>(x1 + so[r] + 16 * s) : frag_zero<F>();
            a2[r] = so[r] >= 0 ? *reinterpret_cast<const F*>(x + so[r] + 16 * s) : frag_zero<F>();
          }
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const int i0 = ((tap * KC + s) * NT + nt) * 64 + lane;
            const F bm = wm[i0], bq = wq[i0];
#pragma unroll
            for (int r = 0; r < R; ++r) {
              am[r][nt] = mfma_chunk(a1[r], bm, am[r][nt]);
              ar[r][nt] = mfma_chunk(a2[r], bq, ar[r][nt]);
            }
          }
        }
      }
    }
  }
  // epilogue: lane holds rows 4g + i of each 16-row sub-tile, channel 16 nt + m
  float bn[NT], gs[NT];
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    bn[nt] = bias[16 * nt + m];
    gs[nt] = 0.f;
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t p = pbase + 16 * r + 4 * g + i;
      if (p >= Pc) continue;
      const int yy = (int)(p / wr), xx = (int)(p % wr);
      const int64_t dp = DOWN ? ((int64_t)b * hd + yy) * wd + xx : ((int64_t)b * hd + 2 * yy + py) * wd + 2 * xx + px;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const float v = fmaxf(am[r][nt][i] + bn[nt], 0.f) + ar[r][nt][i];
        y[dp * N + 16 * nt + m] = from_f<T>(v);
        gs[nt] += stored<T>(v);  // the average is taken over the values as stored
      }
    }
  // channel sums over the 4 lane groups, then the 4 waves, in a fixed order
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    float s = gs[nt];
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    if (g == 0) sm[wave][16 * nt + m] = s;
  }
  __syncthreads();
  float* out = gap + (((int64_t)b * gridDim.y + ph) * tiles + tx) * N;
  for (int c = threadIdx.x; c < N; c += blockDim.x) out[c] = ((sm[0][c] + sm[1][c]) + sm[2][c]) + sm[3][c];
}

}  // namespace stda
