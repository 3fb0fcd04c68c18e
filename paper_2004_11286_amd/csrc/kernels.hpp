// kernels.hpp -- kernel templates of libmclbm and the launch table ("Ops") that
// the C ABI dispatches through. Each precision is instantiated in its own
// translation unit (inst_*.hip) so the library builds in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include "node_ops.hpp"

namespace mclbm {
namespace kern {

constexpr int BLOCK = 256;
constexpr int RED_BLOCK = 256;
constexpr size_t ALIGN = 256;

inline size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
// Occupancy targets (waves per SIMD) that bound the register allocation: the
// kernels are memory bound and need several waves in flight per SIMD.
template <typename S, int M>
constexpr int collide_waves() { return (M == 2 && sizeof(S) < 8) ? 2 : 1; }
template <int M>
constexpr int moment_waves() { return M == 2 ? 2 : 1; }

template <typename S, typename Rec, int M>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(moment_waves<M>()))) void k_moments(const Params<double>* __restrict__ P, const S* __restrict__ pop,
                                                   Rec* __restrict__ rec)
{
  const int64_t node = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (node < P->n) state_node<S, Rec, M>(*P, pop, rec, node);
}

template <typename Rec, bool W>
__global__ __launch_bounds__(BLOCK) void k_gfield(const Params<double>* __restrict__ P,
                                                  const Rec* __restrict__ rec, Rec* __restrict__ G)
{
  const int64_t node = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (node < P->n) gfield_node<Rec, W>(*P, rec, G, node);
}

template <typename S, typename R, typename Rec, int M, bool W>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(collide_waves<S, M>()))) void k_collide(const Params<R>* __restrict__ P, const S* __restrict__ src,
                                                   S* __restrict__ dst, const Rec* __restrict__ rec,
                                                   const Rec* __restrict__ G, uint32_t step)
{
  const int64_t node = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (node < P->n) collide_node<S, R, Rec, M, W>(*P, src, dst, rec, G, node, step);
}

template <typename S, typename R, int M>
__global__ __launch_bounds__(BLOCK) void k_read(const Params<R>* __restrict__ P, const S* __restrict__ pop,
                                                double* X, double* rho, double* u, double* p, double* T)
{
  const int64_t node = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (node < P->n) read_node<S, R, M>(*P, pop, node, X, rho, u, p, T);
}

// Block sum of NV doubles per thread into out[blockIdx.x * NV + k] (fixed order).
template <int NV>
__device__ inline void block_sum(const double (&v)[NV], double* out)
{
  __shared__ double part[RED_BLOCK / 64][NV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = v[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) part[wave][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < RED_BLOCK / 64; ++w) s += part[w][threadIdx.x];
    out[(size_t)blockIdx.x * NV + threadIdx.x] = s;
  }
}

template <typename S, int M>
__global__ __launch_bounds__(RED_BLOCK) void k_conserved(const Params<double>* __restrict__ P,
                                                         const S* __restrict__ pop, double* __restrict__ partial)
{
  constexpr int NV = M + 6;
  double v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = 0.0;
  const int64_t node = (int64_t)blockIdx.x * RED_BLOCK + threadIdx.x;
  if (node < P->n) conserved_node<S, M>(*P, pop, node, v);
  block_sum<NV>(v, partial);
}

// Sums of the initial fields (X_a, p, T) for the reference state.
template <int M>
__global__ __launch_bounds__(RED_BLOCK) void k_field_sums(int64_t n, const double* __restrict__ X,
                                                          const double* __restrict__ p,
                                                          const double* __restrict__ T, double* __restrict__ partial)
{
  constexpr int NV = M + 2;
  double v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = 0.0;
  const int64_t node = (int64_t)blockIdx.x * RED_BLOCK + threadIdx.x;
  if (node < n) {
#pragma unroll
    for (int a = 0; a < M; ++a) v[a] = X[(size_t)a * n + node];
    v[M] = p[node];
    v[M + 1] = T[node];
  }
  block_sum<NV>(v, partial);
}

template <typename S, int M>
__global__ __launch_bounds__(BLOCK) void k_init(const Params<double>* __restrict__ P, const double* __restrict__ X,
                                                const double* __restrict__ p, const double* __restrict__ T,
                                                const double* __restrict__ u, S* __restrict__ pop,
                                                int* __restrict__ block_bad)
{
  const int64_t node = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  int bad = 0;
  if (node < P->n) bad = init_node<S, M>(*P, X, p, T, u, pop, node);
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) block_bad[blockIdx.x] = bad;
}

// ---------------------------------------------------------------------------
// Dispatch over (storage, arithmetic, species count, walls)
// ---------------------------------------------------------------------------
struct Ops {
  size_t s_bytes;   // bytes per stored population
  size_t r_bytes;   // bytes per record value
  int rec_fields;   // values per node in the record
  void (*moments)(const void* P, const void* pop, void* rec, unsigned grid, hipStream_t st);
  void (*gfield)(const void* P, const void* rec, void* G, unsigned grid, hipStream_t st);
  void (*collide)(const void* P, const void* src, void* dst, const void* rec, const void* G, uint32_t step,
                  unsigned grid, hipStream_t st);
  void (*read)(const void* P, const void* pop, double* X, double* rho, double* u, double* p, double* T,
               unsigned grid, hipStream_t st);
  void (*conserved)(const void* Pd, const void* pop, double* partial, unsigned grid, hipStream_t st);
  void (*init)(const void* Pd, const double* X, const double* p, const double* T, const double* u, void* pop,
               int* bad, unsigned grid, hipStream_t st);
  void (*field_sums)(int64_t n, const double* X, const double* p, const double* T, double* partial,
                     unsigned grid, hipStream_t st);
};

template <typename S, typename R, typename Rec, int M, bool W>
Ops make_ops()
{
  Ops o;
  o.s_bytes = sizeof(S);
  o.r_bytes = sizeof(Rec);
  o.rec_fields = RecLayout<M>::FIELDS;
  o.moments = [](const void* Pd, const void* pop, void* rec, unsigned grid, hipStream_t st) {
    hipLaunchKernelGGL((k_moments<S, Rec, M>), dim3(grid), dim3(BLOCK), 0, st, (const Params<double>*)Pd,
                       (const S*)pop, (Rec*)rec);
  };
  o.gfield = [](const void* Pd, const void* rec, void* G, unsigned grid, hipStream_t st) {
    hipLaunchKernelGGL((k_gfield<Rec, W>), dim3(grid), dim3(BLOCK), 0, st, (const Params<double>*)Pd,
                       (const Rec*)rec, (Rec*)G);
  };
  o.collide = [](const void* P, const void* src, void* dst, const void* rec, const void* G, uint32_t step,
                 unsigned grid, hipStream_t st) {
    hipLaunchKernelGGL((k_collide<S, R, Rec, M, W>), dim3(grid), dim3(BLOCK), 0, st, (const Params<R>*)P,
                       (const S*)src, (S*)dst, (const Rec*)rec, (const Rec*)G, step);
  };
  o.read = [](const void* P, const void* pop, double* X, double* rho, double* u, double* p, double* T,
              unsigned grid, hipStream_t st) {
    hipLaunchKernelGGL((k_read<S, R, M>), dim3(grid), dim3(BLOCK), 0, st, (const Params<R>*)P, (const S*)pop, X,
                       rho, u, p, T);
  };
  o.conserved = [](const void* Pd, const void* pop, double* partial, unsigned grid, hipStream_t st) {
    hipLaunchKernelGGL((k_conserved<S, M>), dim3(grid), dim3(RED_BLOCK), 0, st, (const Params<double>*)Pd,
                       (const S*)pop, partial);
  };
  o.init = [](const void* Pd, const double* X, const double* p, const double* T, const double* u, void* pop,
              int* bad, unsigned grid, hipStream_t st) {
    hipLaunchKernelGGL((k_init<S, M>), dim3(grid), dim3(BLOCK), 0, st, (const Params<double>*)Pd, X, p, T, u,
                       (S*)pop, bad);
  };
  o.field_sums = [](int64_t n, const double* X, const double* p, const double* T, double* partial, unsigned grid,
                    hipStream_t st) {
    hipLaunchKernelGGL((k_field_sums<M>), dim3(grid), dim3(RED_BLOCK), 0, st, n, X, p, T, partial);
  };
  return o;
}

template <typename S, typename R, typename Rec>
bool pick_m(int M, int walls, Ops& o)
{
  switch (M) {
    case 2: o = walls ? make_ops<S, R, Rec, 2, true>() : make_ops<S, R, Rec, 2, false>(); return true;
    case 3: o = walls ? make_ops<S, R, Rec, 3, true>() : make_ops<S, R, Rec, 3, false>(); return true;
    case 4: o = walls ? make_ops<S, R, Rec, 4, true>() : make_ops<S, R, Rec, 4, false>(); return true;
    default: return false;
  }
}


}  // namespace kern

// One entry point per instantiated (storage, arithmetic) pair.
bool pick_fp64(int M, int walls, kern::Ops& o);
bool pick_fp32_fp64(int M, int walls, kern::Ops& o);
bool pick_fp32(int M, int walls, kern::Ops& o);
bool pick_fp16(int M, int walls, kern::Ops& o);
bool pick_bf16(int M, int walls, kern::Ops& o);

}  // namespace mclbm
