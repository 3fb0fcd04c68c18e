// device_ops.hpp -- gfx950 device primitives used by the node functions:
// stochastic-rounding conversions to 16-bit storage, streaming loads and stores, and a
// compiler barrier.
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
