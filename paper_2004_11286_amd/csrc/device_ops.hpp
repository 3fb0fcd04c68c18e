// device_ops.hpp -- gfx950 device primitives used by the node functions:
// stochastic-rounding conversions to 16-bit and FP32 storage, buffer accesses,
// streaming loads and stores, and a compiler barrier.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mclbm {

typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Convert with stochastic rounding: rounds to one of the two neighbouring 16-bit
// values with probability proportional to proximity, using the upper 16 bits of
// rnd (v_cvt_sr_f16_f32 / v_cvt_sr_bf16_f32). Representable values are exact.
__device__ inline _Float16 cvt_sr_f16(float x, uint32_t rnd)
{
  f16x2 o = {};
  o = __builtin_amdgcn_cvt_sr_f16_f32(o, x, rnd, false);
  return o[0];
}

__device__ inline __bf16 cvt_sr_bf16(float x, uint32_t rnd)
{
  bf16x2 o = {};
  o = __builtin_amdgcn_cvt_sr_bf16_f32(o, x, rnd, false);
  return o[0];
}

// Round x, a value in units of the storage quantum, to a 16-bit integer
// stochastically: floor(x + r) with r uniform in [0, 1) from the upper 24 bits of
// rnd (the sum is formed in FP32, so r is resolved to 2^-9 of a unit at |x| near
// 2^15), clamped to +-32767.
__device__ inline int16_t cvt_sr_i16(float x, uint32_t rnd)
{
  const float r = (float)(rnd >> 8) * 0x1p-24f;
  const int v = (int)floorf(x + r);
  return (int16_t)min(max(v, -32767), 32767);
}

// The same rounding in fewer instructions, for the step kernels: y = a b + 32768 +
// r with r = k / 256 (k the 8 random bits), formed by one FMA whose addend is the
// float 32768 with k in its low mantissa byte (its unit there is 2^-8: FP32
// resolves no finer fraction at 2^15 anyway). Truncating y >= 0 is its floor, so
// the result is floor(a b + r), clamped to +-32767; y itself goes to the caller's
// range tracking.
__device__ inline int16_t fma_sr_i16(float a, float b, uint32_t k8, float& y)
{
  y = fmaf(a, b, __uint_as_float(0x47000000u | k8));
  const int u = (int)y;
  return (int16_t)(min(max(u, 1), 65535) - 32768);
}

// Convert an FP64 value to FP32 with stochastic rounding: a uniform random
// number (the upper 24 bits of rnd) is added below the 29 mantissa bits that
// FP32 drops, and those bits are then cut: the magnitude is rounded up with
// probability equal to the dropped fraction, so the result is unbiased (its
// expectation is x, to 2^-24 of a unit in the last place). The conversion of
// the cut value is exact for every x in FP32's normal range.
__device__ inline float cvt_sr_f32(double x, uint32_t rnd)
{
  uint64_t b = (uint64_t)__double_as_longlong(x);
  b += (uint64_t)(rnd >> 8) << 5;
  b &= ~(((uint64_t)1 << 29) - 1);
  return (float)__longlong_as_double((long long)b);
}

// Buffer accesses to one direction's array of a lattice (n values from base). The
// resource (base address and byte size, in scalar registers) is the same for the
// whole wavefront: the blocks of a launch each lie in one tube, and base and n
// are that tube's. Each lane adds a 32-bit byte offset, so an access costs no
// per-lane address arithmetic, where a global access through a 64-bit per-lane
// address costs a 64-bit multiply-add or shift-add each. The hardware's range
// check returns zero for loads and drops stores past the array's end. Word 3 of
// the resource is the raw (untyped) buffer format of the gfx9 family.
enum { BUF_CACHED = 0, BUF_NT = 2 };   // cache policy: default, or the nontemporal hint

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes)
{
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

template <typename T, int AUX = BUF_CACHED>
__device__ __forceinline__ T buf_load(const T* base, uint32_t n, uint32_t idx)
{
  const __amdgpu_buffer_rsrc_t r = buf_rsrc(base, n * (uint32_t)sizeof(T));
  const uint32_t off = idx * (uint32_t)sizeof(T);
  if constexpr (sizeof(T) == 8) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, AUX));
  else if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, AUX));
  else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, AUX));
}

template <typename T, int AUX = BUF_CACHED>
__device__ __forceinline__ void buf_store(T* base, uint32_t n, uint32_t idx, T v)
{
  const __amdgpu_buffer_rsrc_t r = buf_rsrc(base, n * (uint32_t)sizeof(T));
  const uint32_t off = idx * (uint32_t)sizeof(T);
  if constexpr (sizeof(T) == 8) {
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, AUX);
  } else if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, AUX);
  } else {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, off, 0, AUX);
  }
}

// Load of a value that is read once and not again soon (the populations a
// collision consumes): a nontemporal load, which keeps the caches for the
// neighbour stencils of the node records.
template <typename T>
__device__ inline T stream_load(const T* p) { return __builtin_nontemporal_load(p); }

// Store of a value the next kernel reads once (the node records): a nontemporal
// store, which streams whole aligned runs to memory without displacing cached
// lines. Not for the streaming pushes, whose runs are shifted by one node: those
// rely on the cache to merge the stores of neighbouring wavefronts into lines.
template <typename T>
__device__ inline void stream_store(T* p, T v) { __builtin_nontemporal_store(v, p); }

// Compiler barrier between the lattices of a node: loads after it are not hoisted
// above it, which bounds the loads (and registers) a thread keeps in flight.
__device__ inline void lattice_barrier() { __asm__ __volatile__("" ::: "memory"); }

}  // namespace mclbm
