// Detection step on restored RD maps (gfx950): CA-CFAR peak detection, the count of reference
// peaks it finds, and the EVM of Sec. V-B.
//
// CA-CFAR (square-law, cell averaging).  The statistic of a cell is p = m^2.  Its training cells
// are those of the (2(gr+tr)+1) x (2(gd+td)+1) window around it outside the (2gr+1) x (2gd+1)
// guard window; the Doppler axis (columns) wraps around, rows outside the map do not count.  With
// N training cells summing to S, the cell is a detection when p > alpha(N) S / N with
// alpha(N) = N (pfa^(-1/N) - 1), the factor that gives false-alarm probability pfa on
// exponentially distributed noise.
//
// A workgroup owns a TH x TW tile of one map.  It stages p (FP64, exact squares of the FP32
// values) of the tile plus its window halo in LDS (columns wrapped), forms the two horizontal
// box sums (widths 2(gd+td)+1 and 2gd+1) of every halo row, then the vertical box sums of those,
// so the training sum of a cell is box(outer) - box(guard): O(window height + width) per cell.
// Detection counts go through integer atomics (order-independent).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/stda.h"

namespace {

constexpr int kTH = 16, kTW = 64, kMaxHalo = STDA_CFAR_MAX_HALO;
constexpr int kRows = kTH + 2 * kMaxHalo, kCols = kTW + 2 * kMaxHalo;

__global__ __launch_bounds__(256) void k_zero_i32(int32_t* p, int n) {
  for (int i = threadIdx.x; i < n; i += 256) p[i] = 0;
}

__global__ __launch_bounds__(256) void k_cfar(const float* __restrict__ maps, int H, int W, int gr, int gd, int tr,
                                              int td, double pfa, uint8_t* __restrict__ det,
                                              const uint8_t* __restrict__ om, int32_t* __restrict__ counts) {
  __shared__ double p[kRows * kCols];
  __shared__ double h1[kRows * kTW];  // outer-width row sums
  __shared__ double h2[kRows * kTW];  // guard-width row sums
  __shared__ int cnt[2];
  const int R = gr + tr, D = gd + td;
  const int rows = kTH + 2 * R, cols = kTW + 2 * D;
  const int y0 = blockIdx.y * kTH, x0 = blockIdx.x * kTW;
  const int64_t base = (int64_t)blockIdx.z * H * W;
  if (threadIdx.x < 2) cnt[threadIdx.x] = 0;
  for (int e = threadIdx.x; e < rows * cols; e += 256) {
    const int r = e / cols, c = e % cols;
    const int y = y0 - R + r;
    int x = (x0 - D + c) % W;
    if (x < 0) x += W;
    double v = 0.0;
    if (y >= 0 && y < H) {
      const double m = (double)maps[base + (int64_t)y * W + x];
      v = m * m;
    }
    p[r * kCols + c] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < rows * kTW; e += 256) {
    const int r = e / kTW, c = e % kTW;
    const double* row = p + r * kCols + c + D;  // column c of the tile
    double s1 = 0.0, s2 = 0.0;
    for (int dx = -D; dx <= D; ++dx) s1 += row[dx];
    for (int dx = -gd; dx <= gd; ++dx) s2 += row[dx];
    h1[r * kTW + c] = s1;
    h2[r * kTW + c] = s2;
  }
  __syncthreads();
  int my_det = 0, my_hit = 0;
  for (int e = threadIdx.x; e < kTH * kTW; e += 256) {
    const int ty = e / kTW, tx = e % kTW;
    const int y = y0 + ty, x = x0 + tx;
    if (y >= H || x >= W) continue;
    double b1 = 0.0, b2 = 0.0;
    for (int dy = -R; dy <= R; ++dy) b1 += h1[(ty + R + dy) * kTW + tx];
    for (int dy = -gr; dy <= gr; ++dy) b2 += h2[(ty + R + dy) * kTW + tx];
    // training cells: rows of the outer / guard windows that lie inside the map
    const int r1 = min(y + R, H - 1) - max(y - R, 0) + 1;
    const int r2 = min(y + gr, H - 1) - max(y - gr, 0) + 1;
    const double n = (double)(r1 * (2 * D + 1) - r2 * (2 * gd + 1));
    const double alpha = n * (pow(pfa, -1.0 / n) - 1.0);
    const double cut = p[(ty + R) * kCols + tx + D];
    const bool d = cut > alpha * (b1 - b2) / n;
    const int64_t idx = base + (int64_t)y * W + x;
    det[idx] = d ? 1 : 0;
    my_det += d ? 1 : 0;
    if (om && d && om[idx]) ++my_hit;
  }
  if (counts) {
    if (my_det) atomicAdd(&cnt[0], my_det);
    if (my_hit) atomicAdd(&cnt[1], my_hit);
    __syncthreads();
    if (threadIdx.x == 0) {
      if (cnt[0]) atomicAdd(&counts[2 * blockIdx.z], cnt[0]);
      if (cnt[1]) atomicAdd(&counts[2 * blockIdx.z + 1], cnt[1]);
    }
  }
}

// EVM (Sec. V-B) of one map per workgroup: mean over the O cells of |clean - est| / |clean|,
// FP64 sums in a fixed order; 0 when the map has no O cell.
__global__ __launch_bounds__(256) void k_evm(const float* __restrict__ est, const float* __restrict__ clean,
                                             const uint8_t* __restrict__ om, int64_t hw, double* __restrict__ out) {
  __shared__ double s[2][256];
  const int64_t base = (int64_t)blockIdx.x * hw;
  double acc = 0.0, n = 0.0;
  for (int64_t i = threadIdx.x; i < hw; i += 256) {
    if (!om[base + i]) continue;
    const double c = (double)clean[base + i], e = (double)est[base + i];
    acc += fabs(c - e) / fabs(c);
    n += 1.0;
  }
  s[0][threadIdx.x] = acc;
  s[1][threadIdx.x] = n;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) {
      s[0][threadIdx.x] += s[0][threadIdx.x + k];
      s[1][threadIdx.x] += s[1][threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = s[1][0] > 0.0 ? s[0][0] / s[1][0] : 0.0;
}

}  // namespace

extern "C" {

int stda_cfar(const float* maps, int n_maps, int H, int W, int guard_r, int guard_d, int train_r, int train_d,
              double pfa, uint8_t* det, const uint8_t* o_mask, int32_t* counts, hipStream_t stream) {
  if (!maps || !det || n_maps < 1 || n_maps > 65535 || H < 1 || W < 1) return STDA_E_INVALID;
  if (guard_r < 0 || guard_d < 0 || train_r < 0 || train_d < 0 || (train_r == 0 && train_d == 0)) return STDA_E_INVALID;
  if (!(pfa > 0.0 && pfa < 1.0)) return STDA_E_INVALID;
  if (guard_r + train_r > kMaxHalo || guard_d + train_d > kMaxHalo) return STDA_E_SHAPE;
  if (2 * (guard_r + train_r) + 1 > H || 2 * (guard_d + train_d) + 1 > W) return STDA_E_SHAPE;
  if (counts) {
    k_zero_i32<<<1, 256, 0, stream>>>(counts, 2 * n_maps);
    if (hipGetLastError() != hipSuccess) return STDA_E_HIP;
  }
  const dim3 grid((W + kTW - 1) / kTW, (H + kTH - 1) / kTH, n_maps);
  k_cfar<<<grid, 256, 0, stream>>>(maps, H, W, guard_r, guard_d, train_r, train_d, pfa, det, o_mask, counts);
  return hipGetLastError() == hipSuccess ? STDA_OK : STDA_E_HIP;
}

int stda_evm(const float* est, const float* clean, const uint8_t* o_mask, int n_maps, int H, int W, double* out_dev,
             hipStream_t stream) {
  if (!est || !clean || !o_mask || !out_dev || n_maps < 1 || H < 1 || W < 1) return STDA_E_INVALID;
  k_evm<<<n_maps, 256, 0, stream>>>(est, clean, o_mask, (int64_t)H * W, out_dev);
  return hipGetLastError() == hipSuccess ? STDA_OK : STDA_E_HIP;
}

}  // extern "C"
