// FMCW range-Doppler map synthesizer on gfx950.
//
// Signal model: Radar-STDA (arXiv 2307.09063) Sec. III-A, Eq. (discrete signal) for a target
// tone, Eq. (IF signal) for the superposition of targets, interferers and complex white
// Gaussian noise.  RD processing: Sec. III-B, Eq. (column transform) over fast time, then
// Eq. (row transform) over slow time.  Each map is converted to dB, floored 80 dB below its
// maximum and min-max scaled to [0, 1].
//
// Three kernels per call, each map slot being one of the three interfered frames or the
// clean frame t:
//   A  per (clip, slot, chirp group): synthesize s(n, m) with exact 32-bit fixed-point phases,
//      apply both Hann windows, N-point radix-2 FFT in LDS, write the range spectrum.
//   B  per (clip, slot, range-bin group): M-point FFT in LDS, move zero Doppler to column M/2,
//      20 log10 |Y| into the output map, per-block max / min.
//   C  per (clip, slot): floor at (max - 80 dB), min-max scale, in place.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "../../include/stda.h"

namespace {

constexpr int RD_PTS = 1024;  // complex points per block in LDS
constexpr float FLOOR_DB = 80.0f;

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
struct U4 {
  uint32_t x, y, z, w;
};
__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return U4{c0, c1, c2, c3};
}

// exp(j 2 pi u / 2^32) in FP32 from a 32-bit fixed-point phase.
__device__ __forceinline__ void cis_u32(uint32_t u, float& c, float& s) {
  const float x = (float)(int32_t)u * 4.656612873077392578125e-10f;  // 2^-31: angle = pi x
  sincospif(x, &s, &c);
}

__device__ __forceinline__ float2 synth_sample(const rd_scene& sc, int frame, bool with_intf, int n, int m,
                                               uint32_t seed, uint32_t clip_id, float sig) {
  float re = 0.f, im = 0.f;
  const int nt = sc.n_tones[frame];
  for (int k = 0; k < nt; ++k) {
    const rd_tone t = sc.tone[frame][k];
    const uint32_t u = t.fr * (uint32_t)n + t.fd * (uint32_t)m + t.ph;
    float c, s;
    cis_u32(u, c, s);
    re += t.amp * c;
    im += t.amp * s;
  }
  if (with_intf) {
    const int ni = sc.n_intf[frame];
    for (int i = 0; i < ni; ++i) {
      const rd_intf f = sc.intf[frame][i];
      // start beat frequency of chirp m: linear in m, or the aggressor's sawtooth (span wrap)
      int64_t g = f.f0 + (int64_t)m * f.dl;
      if (f.wrap > 0) {
        int64_t r = (f.s0 + (int64_t)m * f.dl) % f.wrap;
        if (r < 0) r += f.wrap;
        g = f.f0 + r;
      }
      const int64_t F = 2 * f.q * n + g;  // beat frequency, exact
      if (F > -2147483648LL && F < 2147483648LL) {
        const uint32_t phi = f.coherent ? f.ph0 + (uint32_t)m * f.phd
                                        : philox((uint32_t)m, (uint32_t)i, (uint32_t)frame, 1u, seed, clip_id).x;
        const uint64_t P = (uint64_t)g * (uint64_t)n + (uint64_t)f.q * (uint64_t)((int64_t)n * n) + (uint64_t)phi;
        float c, s;
        cis_u32((uint32_t)P, c, s);
        re += f.amp * c;
        im += f.amp * s;
      }
    }
  }
  const U4 r = philox((uint32_t)n, (uint32_t)m, (uint32_t)frame, 0u, seed, clip_id);
  const float u1 = ((float)(r.x >> 9) + 0.5f) * 1.1920928955078125e-07f;  // 2^-23
  const float u2 = (float)(r.y >> 8) * 5.9604644775390625e-08f;           // 2^-24
  const float rad = sqrtf(-2.0f * logf(u1));
  float sn, cs;
  sincospif(2.0f * u2, &sn, &cs);
  re += sig * rad * cs;
  im += sig * rad * sn;
  return make_float2(re, im);
}

__device__ __forceinline__ float hann(int i, int n) { return 0.5f * (1.0f - cospif(2.0f * (float)i / (float)n)); }

__device__ __forceinline__ int bitrev(int i, int lg) { return (int)(__brev((unsigned)i) >> (32 - lg)); }

// count independent length-n FFTs (forward, e^{-j...}) on bit-reversed data in LDS.
__device__ void fft_lds(float2* buf, int n, int lg, int count) {
  const int half_total = (n / 2) * count;
  for (int s = 1; s <= lg; ++s) {
    const int L = 1 << (s - 1);  // half size of the butterflies of this stage
    for (int b = threadIdx.x; b < half_total; b += blockDim.x) {
      const int f = b / (n / 2), j = b % (n / 2);
      const int grp = j / L, k = j % L;
      const int i0 = f * n + grp * 2 * L + k, i1 = i0 + L;
      float sw, cw;
      sincospif(-(float)k / (float)L, &sw, &cw);
      const float2 a = buf[i0], c = buf[i1];
      const float tr = c.x * cw - c.y * sw, ti = c.x * sw + c.y * cw;
      buf[i0] = make_float2(a.x + tr, a.y + ti);
      buf[i1] = make_float2(a.x - tr, a.y - ti);
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_rd_range(const rd_scene* __restrict__ scenes, int N, int lgN, int M, int cpb,
                                                  uint32_t seed, int clip_base, float sig, float2* __restrict__ Y1) {
  __shared__ float2 buf[RD_PTS];
  const int slot = blockIdx.y, clip = blockIdx.z, m0 = blockIdx.x * cpb;
  const int frame = slot < 3 ? slot : 0;
  const bool with_intf = slot < 3;
  const rd_scene& sc = scenes[clip];
  const uint32_t cid = (uint32_t)(clip_base + clip);
  for (int e = threadIdx.x; e < cpb * N; e += blockDim.x) {
    const int mm = e / N, n = e % N, m = m0 + mm;
    float2 v = synth_sample(sc, frame, with_intf, n, m, seed, cid, sig);
    const float wgt = hann(n, N) * hann(m, M);
    buf[mm * N + bitrev(n, lgN)] = make_float2(v.x * wgt, v.y * wgt);
  }
  __syncthreads();
  fft_lds(buf, N, lgN, cpb);
  float2* out = Y1 + (((int64_t)clip * 4 + slot) * N) * M;
  for (int e = threadIdx.x; e < cpb * N; e += blockDim.x) {
    const int p = e / cpb, mm = e % cpb;
    out[(int64_t)p * M + m0 + mm] = buf[mm * N + p];
  }
}

__global__ __launch_bounds__(256) void k_rd_doppler(const float2* __restrict__ Y1, int N, int M, int lgM, int rpb,
                                                    float* __restrict__ x_out, float* __restrict__ clean_out,
                                                    float2* __restrict__ mxmn) {
  __shared__ float2 buf[RD_PTS];
  __shared__ float smx[256], smn[256];
  const int slot = blockIdx.y, clip = blockIdx.z, p0 = blockIdx.x * rpb;
  const float2* in = Y1 + (((int64_t)clip * 4 + slot) * N + p0) * M;
  for (int e = threadIdx.x; e < rpb * M; e += blockDim.x) {
    const int r = e / M, m = e % M;
    buf[r * M + bitrev(m, lgM)] = in[(int64_t)r * M + m];
  }
  __syncthreads();
  fft_lds(buf, M, lgM, rpb);
  float* map = slot < 3 ? x_out + (((int64_t)clip * 3 + slot) * N) * M : clean_out + ((int64_t)clip * N) * M;
  float mx = -INFINITY, mn = INFINITY;
  for (int e = threadIdx.x; e < rpb * M; e += blockDim.x) {
    const int r = e / M, q = e % M;
    const float2 v = buf[r * M + q];
    const float db = 10.0f * log10f(v.x * v.x + v.y * v.y);  // 20 log10 |Y|; -inf for 0
    map[(int64_t)(p0 + r) * M + ((q + M / 2) & (M - 1))] = db;
    mx = fmaxf(mx, db);
    mn = fminf(mn, db);
  }
  smx[threadIdx.x] = mx;
  smn[threadIdx.x] = mn;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      smx[threadIdx.x] = fmaxf(smx[threadIdx.x], smx[threadIdx.x + s]);
      smn[threadIdx.x] = fminf(smn[threadIdx.x], smn[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) mxmn[((int64_t)clip * 4 + slot) * gridDim.x + blockIdx.x] = make_float2(smx[0], smn[0]);
}

__global__ __launch_bounds__(256) void k_rd_normalise(int N, int M, int nparts, const float2* __restrict__ mxmn,
                                                      float* __restrict__ x_out, float* __restrict__ clean_out) {
  const int slot = blockIdx.y, clip = blockIdx.z;
  __shared__ float s_fl, s_mn, s_scale;
  if (threadIdx.x == 0) {
    float mx = -INFINITY, mnr = INFINITY;
    const float2* q = mxmn + ((int64_t)clip * 4 + slot) * nparts;
    for (int i = 0; i < nparts; ++i) {
      mx = fmaxf(mx, q[i].x);
      mnr = fminf(mnr, q[i].y);
    }
    const float fl = mx - FLOOR_DB;
    const float mn = fmaxf(mnr, fl);
    s_fl = fl;
    s_mn = mn;
    s_scale = (mx > mn && mx > -INFINITY) ? 1.0f / (mx - mn) : 0.0f;
  }
  __syncthreads();
  float* map = slot < 3 ? x_out + (((int64_t)clip * 3 + slot) * N) * M : clean_out + ((int64_t)clip * N) * M;
  const int64_t total = (int64_t)N * M;
  const float fl = s_fl, mn = s_mn, sc = s_scale;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const float v = fmaxf(map[i], fl);
    map[i] = sc == 0.0f ? 0.0f : (v - mn) * sc;
  }
}

int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

}  // namespace

extern "C" {

size_t rd_synth_workspace_size(int n_clips, int N, int M) {
  if (n_clips < 1 || N < 1 || M < 1) return 0;
  const int rpb = std::max(1, std::min(M > 0 ? RD_PTS / M : 1, N));
  const size_t parts = (size_t)n_clips * 4 * (size_t)(N / rpb);
  return ((size_t)n_clips * 4 * N * M * sizeof(float2) + 255) / 256 * 256 + parts * sizeof(float2);
}

int rd_synth(const rd_scene* scenes, int n_clips, int N, int M, uint32_t seed, float noise_sigma, int clip_base,
             float* x_out, float* clean_out, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!scenes || !x_out || !ws || n_clips < 1 || clip_base < 0) return STDA_E_INVALID;
  if (N < 8 || M < 8 || N > RD_PTS || M > RD_PTS || (N & (N - 1)) || (M & (M - 1))) return STDA_E_SHAPE;
  if (ws_bytes < rd_synth_workspace_size(n_clips, N, M)) return STDA_E_WORKSPACE;
  const int slots = clean_out ? 4 : 3;
  const int cpb = std::min(RD_PTS / N, M);
  const int rpb = std::min(RD_PTS / M, N);
  float2* Y1 = reinterpret_cast<float2*>(ws);
  float2* mxmn = reinterpret_cast<float2*>((char*)ws + ((size_t)n_clips * 4 * N * M * sizeof(float2) + 255) / 256 * 256);
  const float sig = noise_sigma * 0.70710678118654752f;
  k_rd_range<<<dim3(M / cpb, slots, n_clips), 256, 0, stream>>>(scenes, N, ilog2(N), M, cpb, seed, clip_base, sig, Y1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return STDA_E_HIP;
  k_rd_doppler<<<dim3(N / rpb, slots, n_clips), 256, 0, stream>>>(Y1, N, M, ilog2(M), rpb, x_out, clean_out, mxmn);
  e = hipGetLastError();
  if (e != hipSuccess) return STDA_E_HIP;
  const int nb = (int)std::min<int64_t>(64, ((int64_t)N * M + 1023) / 1024);
  k_rd_normalise<<<dim3(nb, slots, n_clips), 256, 0, stream>>>(N, M, N / rpb, mxmn, x_out, clean_out);
  e = hipGetLastError();
  if (e != hipSuccess) return STDA_E_HIP;
  return STDA_OK;
}

size_t rd_synth_host_workspace_size(int n_clips, int N, int M) {
  const size_t base = rd_synth_workspace_size(n_clips, N, M);
  if (base == 0) return 0;
  return (base + 255) / 256 * 256 + (size_t)n_clips * sizeof(rd_scene);
}

int rd_synth_host(const rd_scene* scenes_host, int n_clips, int N, int M, uint32_t seed, float noise_sigma,
                  int clip_base, float* x_out, float* clean_out, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!scenes_host || !x_out || !ws || n_clips < 1 || clip_base < 0) return STDA_E_INVALID;
  if (N < 8 || M < 8 || N > RD_PTS || M > RD_PTS || (N & (N - 1)) || (M & (M - 1))) return STDA_E_SHAPE;
  if (ws_bytes < rd_synth_host_workspace_size(n_clips, N, M)) return STDA_E_WORKSPACE;
  const size_t base = (rd_synth_workspace_size(n_clips, N, M) + 255) / 256 * 256;
  rd_scene* dev = reinterpret_cast<rd_scene*>(static_cast<char*>(ws) + base);
  // the table is in the workspace, and the host array free to reuse, when this returns
  if (hipMemcpyAsync(dev, scenes_host, (size_t)n_clips * sizeof(rd_scene), hipMemcpyHostToDevice, stream) != hipSuccess)
    return STDA_E_HIP;
  if (hipStreamSynchronize(stream) != hipSuccess) return STDA_E_HIP;
  return rd_synth(dev, n_clips, N, M, seed, noise_sigma, clip_base, x_out, clean_out, ws, base, stream);
}

}  // extern "C"
