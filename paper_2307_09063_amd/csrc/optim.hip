// AdamW with decoupled weight decay and step annealing over the flat FP32 master buffer (gfx950).
// The hyper-parameters and the step counter live in device memory (stda_adamw_state), so a
// captured graph of a training step replays with the right step count and learning rate: the
// update kernel reads the counter, a one-thread kernel after it advances the counter.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/stda.h"

namespace {

__device__ __forceinline__ uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__global__ __launch_bounds__(256) void k_adamw(float* __restrict__ w, const float* __restrict__ g,
                                               float* __restrict__ m, float* __restrict__ v, int64_t n,
                                               const stda_adamw_state* __restrict__ st, uint16_t* __restrict__ wb) {
  const stda_adamw_state s = *st;
  const int t = s.t + 1;  // this step, 1-based
  const double lr = s.step_size > 0 ? s.lr * pow(s.gamma, (double)(s.t / s.step_size)) : s.lr;
  // scalar coefficients in FP64 once per thread: bias corrections folded into the step size and
  // the denominator, 1 - beta formed before rounding to FP32
  const double c1 = 1.0 - pow(s.beta1, (double)t), c2 = 1.0 - pow(s.beta2, (double)t);
  const float step = (float)(lr / c1), rc2 = (float)(1.0 / sqrt(c2)), decay = (float)(1.0 - lr * s.weight_decay);
  const float b1 = (float)s.beta1, b2 = (float)s.beta2, ob1 = (float)(1.0 - s.beta1), ob2 = (float)(1.0 - s.beta2);
  const float eps = (float)s.eps;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float gi = g[i];
    const float mi = b1 * m[i] + ob1 * gi;
    const float vi = b2 * v[i] + ob2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] * decay - step * mi / (sqrtf(vi) * rc2 + eps);
    w[i] = wi;
    if (wb) wb[i] = bf16_rne(wi);
  }
}

__global__ void k_adamw_tick(stda_adamw_state* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) st->t += 1;
}

}  // namespace

extern "C" {

int stda_adamw_step(float* w, const float* dw, float* m, float* v, int64_t n, stda_adamw_state* state,
                    uint16_t* w_bf16, hipStream_t stream) {
  if (!w || !dw || !m || !v || !state || n < 0) return STDA_E_INVALID;
  if (n > 0) {
    const int64_t blocks = (n + 255) / 256;
    k_adamw<<<(unsigned)(blocks < 1024 ? blocks : 1024), 256, 0, stream>>>(w, dw, m, v, n, state, w_bf16);
    if (hipGetLastError() != hipSuccess) return STDA_E_HIP;
  }
  k_adamw_tick<<<1, 64, 0, stream>>>(state);
  return hipGetLastError() == hipSuccess ? STDA_OK : STDA_E_HIP;
}

}  // extern "C"
