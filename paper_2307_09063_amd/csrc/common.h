// Shared device helpers of the Radar-STDA HIP library: storage types, 4-channel vector
// loads/stores for NHWC rows, per-channel block reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "seg.h"

#define STDA_BLOCK 256

namespace stda {

// Workgroup barrier over LDS data only: this wave's LDS accesses complete, then s_barrier.  Unlike
// __syncthreads it leaves vector-memory loads in flight, among them loads that write LDS for a
// later phase (whose issuer waits for them and synchronises again before they are read).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }
// An LDS address as the LDS address space's pointer (the destination operand of loads that write
// LDS directly).
__device__ __forceinline__ __attribute__((address_space(3))) void* lds_ptr(const void* p) {
  return (__attribute__((address_space(3))) void*)(p);
}
// Wait until every vector-memory access this wave issued has completed (s_waitcnt vmcnt(0); in
// the gfx9 encoding vmcnt sits in bits 3:0 and 15:14, expcnt 6:4 and lgkmcnt 11:8 are left at
// their maxima, i.e. not waited for).
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// BF16 storage: raw 16-bit pattern, converted to/from FP32 at every load/store.
struct bf16 {
  uint16_t v;
};

__device__ __forceinline__ float to_f(float x) { return x; }
__device__ __forceinline__ float to_f(bf16 x) { return __uint_as_float((uint32_t)x.v << 16); }

template <class T> __device__ __forceinline__ T from_f(float x);
template <> __device__ __forceinline__ float from_f<float>(float x) { return x; }
// Round to nearest even; NaN stays a quiet NaN.  gfx950 converts in hardware (v_cvt_pk_bf16_f32,
// two values per instruction); its results equal the bitwise round-to-nearest-even on every
// non-NaN FP32 pattern.
typedef __bf16 bf16x2_hw __attribute__((ext_vector_type(2)));
typedef float f32x2_hw __attribute__((ext_vector_type(2)));
template <> __device__ __forceinline__ bf16 from_f<bf16>(float x) { return bf16{__builtin_bit_cast(uint16_t, (__bf16)x)}; }
// a in the low half, b in the high half
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_hw{a, b}, bf16x2_hw));
}
__device__ __forceinline__ float round_bf16(float x) { return to_f(from_f<bf16>(x)); }
// The value a store of type T keeps.
template <class T> __device__ __forceinline__ float stored(float x) { return to_f(from_f<T>(x)); }

// Four consecutive channels of an NHWC row (16-byte aligned for FP32, 8-byte for BF16).
__device__ __forceinline__ void ld4(const float* p, float v[4]) {
  float4 q = *reinterpret_cast<const float4*>(p);
  v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
}
__device__ __forceinline__ void ld4(const bf16* p, float v[4]) {
  uint2 q = *reinterpret_cast<const uint2*>(p);
  v[0] = __uint_as_float(q.x << 16);
  v[1] = __uint_as_float(q.x & 0xffff0000u);
  v[2] = __uint_as_float(q.y << 16);
  v[3] = __uint_as_float(q.y & 0xffff0000u);
}
__device__ __forceinline__ void st4(float* p, const float v[4]) {
  *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void st4(bf16* p, const float v[4]) {
  uint2 q;
  q.x = pack_bf16x2(v[0], v[1]);
  q.y = pack_bf16x2(v[2], v[3]);
  *reinterpret_cast<uint2*>(p) = q;
}
__device__ __forceinline__ void zero4(float v[4]) { v[0] = v[1] = v[2] = v[3] = 0.f; }

// Four channels held in their storage form (a load in flight is not waited for until raw_cvt4
// converts it): float4 for FP32, the packed pairs for BF16.
template <class T> struct Raw4;
template <> struct Raw4<float> { typedef float4 type; };
template <> struct Raw4<bf16> { typedef uint2 type; };
__device__ __forceinline__ void raw_ld4(const float* p, float4& r) { r = *reinterpret_cast<const float4*>(p); }
__device__ __forceinline__ void raw_ld4(const bf16* p, uint2& r) { r = *reinterpret_cast<const uint2*>(p); }
// The same four channels by a buffer load at byte offset off (an offset past the buffer's range
// reads 0): no branch around the load, so every thread issues the same loads.
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void raw_bld4(__amdgpu_buffer_rsrc_t rs, int off, float4& r) {
  const u32x4_t q = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
  r = make_float4(__uint_as_float(q.x), __uint_as_float(q.y), __uint_as_float(q.z), __uint_as_float(q.w));
}
__device__ __forceinline__ void raw_bld4(__amdgpu_buffer_rsrc_t rs, int off, uint2& r) {
  const u32x2_t q = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
  r = make_uint2(q.x, q.y);
}
__device__ __forceinline__ void raw_zero4(float4& r) { r = make_float4(0.f, 0.f, 0.f, 0.f); }
__device__ __forceinline__ void raw_zero4(uint2& r) { r = make_uint2(0u, 0u); }
__device__ __forceinline__ void raw_cvt4(const float4& r, float v[4]) {
  v[0] = r.x; v[1] = r.y; v[2] = r.z; v[3] = r.w;
}
__device__ __forceinline__ void raw_cvt4(const uint2& r, float v[4]) {
  v[0] = __uint_as_float(r.x << 16);
  v[1] = __uint_as_float(r.x & 0xffff0000u);
  v[2] = __uint_as_float(r.y << 16);
  v[3] = __uint_as_float(r.y & 0xffff0000u);
}

// Per-channel block reduction for the (pixel, channel-group) thread mapping: thread t owns
// channels 4*(t % G) .. +3 of some pixel; NS statistics per channel.  Sums the NS*4 values
// of all threads with the same channel group in a fixed order and writes
// out[s * C + c] (C = 4 G) from threads t < C.  `sm` holds STDA_BLOCK * NS * 4 floats.
template <int G, int NS>
__device__ __forceinline__ void block_channel_sums(const float (&v)[NS][4], float* sm, float* out) {
  const int t = threadIdx.x;
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int j = 0; j < 4; ++j) sm[(s * 4 + j) * STDA_BLOCK + t] = v[s][j];
  __syncthreads();
  constexpr int C = 4 * G;
  for (int i = t; i < NS * C; i += STDA_BLOCK) {
    const int s = i / C, c = i % C;
    const int g = c >> 2, j = c & 3;
    const float* row = sm + (s * 4 + j) * STDA_BLOCK;
    float acc = 0.f;
    for (int p = g; p < STDA_BLOCK; p += G) acc += row[p];
    out[s * C + c] = acc;
  }
  __syncthreads();
}

// Scale / shift of a batch-norm layer from its (mean, invstd) and affine parameters.
__device__ __forceinline__ void bn_affine4(const float* stats, const float* gamma, const float* beta,
                                           int C, int c0, float sc[4], float sh[4]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float m = stats[c0 + j], is = stats[C + c0 + j];
    sc[j] = gamma[c0 + j] * is;
    sh[j] = beta[c0 + j] - m * sc[j];
  }
}

}  // namespace stda
