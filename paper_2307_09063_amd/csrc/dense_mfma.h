// Dense stride-2 layers of the mobile blocks on the matrix cores (gfx950 MFMA).
//
// Implicit GEMM: out[p][n] = sum over taps t and input channels k of src(p, t)[k] * W[t][k][n].
// One wave computes 16*R GEMM rows (pixels) x all N output channels; a block is 4 waves and
// loops over row tiles.  A fragments are gathered straight from NHWC rows: lane (m, g) of a
// 16-row sub-tile loads channels 16s + 4g .. +3 of its pixel (one 16-byte FP32 or 8-byte BF16
// load).  B fragments are pre-arranged per call in "fragment order" (lane-contiguous), so a
// wave reads one coalesced 1 KB (FP32) / 512 B (BF16) block per (tap, 16-channel chunk, 16
// output channels); every block reads the same weights, which therefore stay in L1/L2.
//
// FP32: v_mfma_f32_16x16x4f32.  The four channels a lane holds feed four consecutive MFMAs
// (k-index e of the lane group g is channel 4g + e): a fixed permutation of the reduction order
// applied identically to A and B.  BF16: lane group g supplies channels 4g .. 4g + 3 of a
// 16-channel chunk; with 32 or more input channels two chunks of a tap feed one gfx950
// v_mfma_f32_16x16x32_bf16, with 16 one chunk feeds v_mfma_f32_16x16x16bf16_1k.  Accumulation is
// FP32 in both cases.
//
// Up-sampling operators (DeConv4x4-s2 forward, Conv3x3-s2 adjoint) run one output phase
// (row parity, column parity) per grid.y so that all rows of a block share their taps.
#pragma once
#include <type_traits>

#include "net_kernels.h"

namespace stda {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef short shortx4 __attribute__((ext_vector_type(4)));

template <class T>
struct FragT;
template <>
struct FragT<float> {
  typedef float4 type;
};
template <>
struct FragT<bf16> {
  typedef shortx4 type;
};

__device__ __forceinline__ floatx4 mfma_chunk(const float4 a, const float4 b, floatx4 c) {
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, c, 0, 0, 0);
  return c;
}
__device__ __forceinline__ floatx4 mfma_chunk(const shortx4 a, const shortx4 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Two 4-value BF16 operands as the 8 values one lane feeds v_mfma_f32_16x16x32_bf16 (gfx950).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short shortx8 __attribute__((ext_vector_type(8)));
__device__ __forceinline__ bf16x8 pack8(const shortx4 a, const shortx4 b) {
  return __builtin_bit_cast(bf16x8, __builtin_shufflevector(a, b, 0, 1, 2, 3, 4, 5, 6, 7));
}

template <class F>
__device__ __forceinline__ F frag_zero() {
  F z;
  if constexpr (std::is_same<F, float4>::value) {
    z = make_float4(0.f, 0.f, 0.f, 0.f);
  } else {
    z = shortx4{0, 0, 0, 0};
  }
  return z;
}

// Fragment-order weights: frag[((tap * KC + s) * NT + nt) * 64 + lane][e] = W[tap][16 s + 4 g + e]
// [16 nt + m] (lane = 16 g + m), from [tap][K][N] FP32 layouts; one job per layout.
struct FragJob {
  int64_t src, dst;  // element offsets of the [tap][K][N] layout and of the fragment buffer
  int taps, K, N;
};
struct FragJobs {
  int n;
  FragJob j[16];
};
template <class T>
__global__ void k_prep_frag(const float* __restrict__ wl, T* __restrict__ frag, FragJobs jobs) {
  const FragJob J = jobs.j[blockIdx.y];
  const int KC = J.K / 16, NT = J.N / 16;
  const int64_t total = (int64_t)J.taps * KC * NT * 64 * 4;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int e = (int)(i & 3);
    int64_t r = i >> 2;
    const int lane = (int)(r & 63);
    r >>= 6;
    const int nt = (int)(r % NT);
    r /= NT;
    const int s = (int)(r % KC);
    const int tap = (int)(r / KC);
    const int k = 16 * s + 4 * (lane >> 4) + e, n = 16 * nt + (lane & 15);
    frag[J.dst + i] = from_f<T>(wl[J.src + ((int64_t)tap * J.K + k) * J.N + n]);
  }
}

template <class T, int OP, int K, int N, int R, bool STATS>
struct k_dense_mfma_args {
  const T* src;
  const T* wfrag;
  T* dst;
  float* part;
  int B;
  int hd;
  int wd;
};
template <class T, int OP, int K, int N, int R, bool STATS>
__global__ __launch_bounds__(256) void k_dense_mfma(SegL<k_dense_mfma_args<T, OP, K, N, R, STATS>> L) {
  const SegB sb = seg_block(L);
  if (sb.x >= sb.gx) return;
  const int bx = sb.x, gx = sb.gx;  // workgroup index and count within the segment
  (void)gx;
  const k_dense_mfma_args<T, OP, K, N, R, STATS>& a_ = L.a[sb.s];
  const T* __restrict__ const src = a_.src;
  const T* __restrict__ const wfrag = a_.wfrag;
  T* __restrict__ const dst = a_.dst;
  float* __restrict__ const part = a_.part;
  const int B = a_.B;
  const int hd = a_.hd;
  const int wd = a_.wd;
  typedef typename FragT<T>::type F;
  constexpr int KS = OpGeo<OP>::KS;
  constexpr bool DOWN = OpGeo<OP>::DOWN;
  constexpr int NT = N / 16, KC = K / 16;
  constexpr bool PAIR2 = sizeof(T) == 2 && KC % 2 == 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, m = lane & 15, g = lane >> 4;
  const int py = DOWN ? 0 : (int)(blockIdx.y >> 1), px = DOWN ? 0 : (int)(blockIdx.y & 1);
  const int hr = DOWN ? hd : hd / 2, wr = DOWN ? wd : wd / 2;  // GEMM row grid
  const int hs = DOWN ? 2 * hd : hd / 2, ws = DOWN ? 2 * wd : wd / 2;
  const int64_t P = (int64_t)B * hr * wr;
  const int64_t tiles = (P + 64 * R - 1) / (64 * R);
  const F* wf = reinterpret_cast<const F*>(wfrag);
  // the unrolled tap loop lets the compiler keep every weight fragment of the layer in registers
  // across tiles; that pays while they fit (up to 256 dwords a lane)
  constexpr int WDW = (DOWN ? KS * KS : 4) * KC * NT * (int)(sizeof(F) / 4);
  constexpr bool HOIST_W = WDW <= 256;
  float mn[NT], q2[NT];  // STATS: mean and m2 of this lane's columns 16 nt + m (Welford)
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) mn[nt] = q2[nt] = 0.f;
  float cnt = 0.f;  // rows seen by this lane

  for (int64_t tile = bx; tile < tiles; tile += gx) {
    const int64_t pbase = (tile * 4 + wave) * 16 * R;
    int pb[R], prow[R], pcol[R];
    bool pv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t p = pbase + 16 * r + m;
      pv[r] = p < P;
      pix3(pv[r] ? p : 0, hr, wr, pb[r], prow[r], pcol[r]);
    }
    floatx4 acc[R][NT];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[r][nt] = floatx4{0.f, 0.f, 0.f, 0.f};

    // one tap (ky, kx) of the GEMM's k loop
    auto do_tap = [&](const int ky, const int kx) {
      const int tap = ky * KS + kx;
      int64_t so[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int sy = DOWN ? 2 * prow[r] - 1 + ky : (2 * prow[r] + py + 1 - ky) / 2;
        const int sx = DOWN ? 2 * pcol[r] - 1 + kx : (2 * pcol[r] + px + 1 - kx) / 2;
        const bool ok = pv[r] && sy >= 0 && sy < hs && sx >= 0 && sx < ws;
        so[r] = ok ? (((int64_t)pb[r] * hs + sy) * ws + sx) * K + 4 * g : -1;
      }
      if constexpr (PAIR2) {
        // BF16, K a multiple of 32: chunks s and s + 1 of the tap feed one 16x16x32 product
#pragma unroll
        for (int s = 0; s < KC; s += 2) {
          bf16x8 av[R];
#pragma unroll
          for (int r = 0; r < R; ++r)
            av[r] = so[r] >= 0 ? pack8(*reinterpret_cast<const F*>(src + so[r] + 16 * s),
                                       *reinterpret_cast<const F*>(src + so[r] + 16 * s + 16))
                               : pack8(frag_zero<F>(), frag_zero<F>());
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const bf16x8 bv = pack8(wf[((tap * KC + s) * NT + nt) * 64 + lane], wf[((tap * KC + s + 1) * NT + nt) * 64 + lane]);
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[r], bv, acc[r][nt], 0, 0, 0);
          }
        }
      } else {
#pragma unroll
        for (int s = 0; s < KC; ++s) {
          F av[R];
#pragma unroll
          for (int r = 0; r < R; ++r)
            av[r] = so[r] >= 0 ? *reinterpret_cast<const F*>(src + so[r] + 16 * s) : frag_zero<F>();
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            const F bv = wf[((tap * KC + s) * NT + nt) * 64 + lane];
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r][nt] = mfma_chunk(av[r], bv, acc[r][nt]);
          }
        }
      }
    };
    // taps of this phase: KS x KS (stride-2 convolution) or 2 x 2 (one phase of a transposed one)
    constexpr int NA = DOWN ? KS : 2;
    if constexpr (HOIST_W) {
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        const int ky = DOWN ? a : ((py + 1) & 1) + 2 * a;
        if (ky >= KS) continue;
#pragma unroll
        for (int c = 0; c < NA; ++c) {
          const int kx = DOWN ? c : ((px + 1) & 1) + 2 * c;
          if (kx >= KS) continue;
          do_tap(ky, kx);
        }
      }
    } else {
      // a runtime tap loop: the weight fragments are read per tile (from cache) instead of being
      // held across tiles, which for this many taps would not fit the registers
#pragma unroll 1
      for (int t = 0; t < NA * NA; ++t) {
        const int a = t / NA, c = t % NA;
        const int ky = DOWN ? a : ((py + 1) & 1) + 2 * a, kx = DOWN ? c : ((px + 1) & 1) + 2 * c;
        if (ky < KS && kx < KS) do_tap(ky, kx);
      }
    }
    // epilogue: lane holds rows 4g + i of each 16-row sub-tile, channel 16 nt + m
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t p = pbase + 16 * r + 4 * g + i;
        if (p >= P) continue;
        int64_t dp = p;
        if (!DOWN) {
          int b, y, x;
          pix3(p, hr, wr, b, y, x);
          dp = ((int64_t)b * hd + 2 * y + py) * wd + 2 * x + px;
        }
        float rk = 0.f;
        if (STATS) {
          cnt += 1.f;
          rk = __builtin_amdgcn_rcpf(cnt);
        }
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const float v = acc[r][nt][i];
          dst[dp * N + 16 * nt + m] = from_f<T>(v);
          if (STATS) wf_add(mn[nt], q2[nt], v, rk);
        }
      }
  }
  if (STATS) {
    // part[blk][N][2] = (mean, m2), the block's count at part[blocks * 2 N + blk]: merge over the
    // 4 lane groups (same channel), then over the 4 waves, in a fixed order
    __shared__ float sm[4][2 * N + 1];
#pragma unroll
    for (int off = 16; off < 64; off <<= 1) {
      const float nb = __shfl_xor(cnt, off);
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const float mb = __shfl_xor(mn[nt], off), qb = __shfl_xor(q2[nt], off);
        chan_merge(cnt, mn[nt], q2[nt], nb, mb, qb);
      }
      cnt += nb;
    }
    if (g == 0) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        sm[wave][16 * nt + m] = mn[nt];
        sm[wave][N + 16 * nt + m] = q2[nt];
      }
      if (m == 0) sm[wave][2 * N] = cnt;
    }
    __syncthreads();
    const int64_t blk = (int64_t)blockIdx.y * gx + bx;
    for (int c = threadIdx.x; c < N; c += STDA_BLOCK) {
      float na = sm[0][2 * N], ma = sm[0][c], qa = sm[0][N + c];
#pragma unroll
      for (int wv = 1; wv < 4; ++wv) {
        chan_merge(na, ma, qa, sm[wv][2 * N], sm[wv][c], sm[wv][N + c]);
        na += sm[wv][2 * N];
      }
      part[blk * 2 * N + 2 * c] = ma;
      part[blk * 2 * N + 2 * c + 1] = qa;
      if (c == 0) part[(int64_t)gx * gridDim.y * 2 * N + blk] = na;
    }
  }
}

}  // namespace stda


