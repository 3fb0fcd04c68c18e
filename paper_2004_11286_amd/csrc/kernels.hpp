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
// Tubes and launches
// ---------------------------------------------------------------------------
// A context holds one or more independent lattices ("tubes"). Tube t owns the
// node range [base, base + n_t) of every buffer, laid out exactly as a context
// of that single tube would be (pop[l][i][n_t], rec[k][n_t], ...), and its own
// parameter block P[t]. Launches are in blocks of BLOCK nodes; a block never
// straddles two tubes.
//
// Block shapes. In the linear numbering a block is BLOCK consecutive nodes of a
// tube (x fastest, rows wrapping). The step kernels can instead take a block as a
// tile of 2^sx x 2^sy x 2^sz nodes (sx + sy + sz = log2 BLOCK) at a tile origin of
// the tube's grid, so that the stencil neighbours in y and z of a block's nodes
// are mostly the block's own; threads of a tile that fall outside the grid (a
// ragged edge) do nothing. Every node computes the same values either way.
// The reductions and field transfers always use the linear numbering.
constexpr int LOG2_BLOCK = 8;
constexpr int NSHAPES = 6;
// (sx, sy) of each shape; shape 0 is the linear numbering
constexpr int SHAPE_SX[NSHAPES] = {0, 6, 5, 4, 6, 5};
constexpr int SHAPE_SY[NSHAPES] = {0, 2, 3, 4, 1, 2};

struct Tube {
  int64_t base;          // first node of the tube in the concatenated buffers
  int32_t first_block;   // first block of the tube in a linear launch over all tubes
  int32_t nblocks;
  int32_t nx, ny, nz;    // the tube's grid
  int32_t tiles_x, tiles_y;   // tiles per row and per plane of the current shape
  int32_t tfirst, tnblocks;   // first block and block count of the tube in a tiled launch
  int32_t pad;
};

struct Launch {
  const Tube* tubes;
  const int32_t* blk_tube;   // tube of every block (read when ntubes > 1)
  int32_t ntubes;
  int32_t block0;            // added to the block index: a launch over one tube
  int32_t swizzle;           // give each XCD a contiguous run of blocks
  int32_t shape;             // 0: linear numbering; else sx | sy << 4 of the tiles
};

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b mod 8). Renumbering so that XCD k takes blocks [k q, (k+1) q) keeps the
// neighbours a block's stencils read in the same XCD's L2.
__device__ inline uint32_t xcd_block(uint32_t b, uint32_t nb)
{
  constexpr uint32_t NXCD = 8;
  const uint32_t q = nb / NXCD;
  if (b >= q * NXCD) return b;
  return (b % NXCD) * q + b / NXCD;
}

struct Where {
  int t;
  int64_t base, node;
  uint32_t block;        // logical block in a launch over all tubes
};

// The tube, its first node and this thread's node (outside [0, n) for a tile
// thread beyond the grid: the kernels skip nodes >= n).
__device__ inline Where locate(const Launch& Ln)
{
  uint32_t b = blockIdx.x;
  if (Ln.swizzle) b = xcd_block(b, gridDim.x);
  b += (uint32_t)Ln.block0;
  const int t = Ln.ntubes > 1 ? Ln.blk_tube[b] : 0;
  const Tube tb = Ln.tubes[t];
  if (!Ln.shape) return {t, tb.base, (int64_t)(b - (uint32_t)tb.first_block) * BLOCK + threadIdx.x, b};
  const uint32_t sx = (uint32_t)Ln.shape & 15u, sy = (uint32_t)Ln.shape >> 4;
  uint32_t lb = b - (uint32_t)tb.tfirst;
  const uint32_t ix = lb % (uint32_t)tb.tiles_x;
  lb /= (uint32_t)tb.tiles_x;
  const uint32_t iy = lb % (uint32_t)tb.tiles_y, iz = lb / (uint32_t)tb.tiles_y;
  const uint32_t tid = threadIdx.x;
  const uint32_t x = (ix << sx) + (tid & ((1u << sx) - 1u));
  const uint32_t y = (iy << sy) + ((tid >> sx) & ((1u << sy) - 1u));
  const uint32_t z = (iz << (LOG2_BLOCK - sx - sy)) + (tid >> (sx + sy));
  const bool inside = x < (uint32_t)tb.nx && y < (uint32_t)tb.ny && z < (uint32_t)tb.nz;
  const int64_t node = inside ? (int64_t)x + (int64_t)tb.nx * ((int64_t)y + (int64_t)tb.ny * (int64_t)z)
                              : INT64_MAX;
  return {t, tb.base, node, b};
}

// Step number for the stochastic-rounding seeds: a constant in eager launches,
// a device counter plus the position inside a replayed graph.
struct StepNo {
  const uint32_t* ctr;
  uint32_t add;
};

__device__ inline uint32_t step_of(const StepNo& s) { return s.add + (s.ctr ? *s.ctr : 0u); }

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
// Occupancy targets (waves per SIMD) that bound the register allocation: the
// kernels are memory bound and need several waves in flight per SIMD. Variant
// 1 is the other choice (the autotuner measures both).
template <typename S, int M, int V>
constexpr int collide_waves() { return ((M == 2 && sizeof(S) < 8) ? 2 : 1) == 2 ? 2 - V : 1 + V; }
template <int M, int V>
constexpr int moment_waves() { return (M == 2 ? 2 : 1) == 2 ? 2 - V : 1 + V; }

template <int M, bool WEAK>
constexpr size_t pop_stride() { return (size_t)Lat<M, WEAK>::L * Q; }   // populations per node (stored lattices)

template <typename S, typename Rec, int M, int V, bool WEAK, bool CVT>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(moment_waves<M, V>()))) void k_moments(const Params<double>* __restrict__ P, Launch Ln, const S* __restrict__ pop,
                                                   Rec* __restrict__ rec)
{
  const Where w = locate(Ln);
  const Params<double>& Pt = P[w.t];
  if (w.node < Pt.n)
    state_node<S, Rec, M, WEAK, CVT>(Pt, pop + pop_stride<M, WEAK>() * w.base,
                                     rec + (size_t)RecLayout<M, WEAK, CVT>::FIELDS * w.base, w.node);
}

template <typename Rec, int W>
__global__ __launch_bounds__(BLOCK) void k_gfield(const Params<double>* __restrict__ P, Launch Ln,
                                                  const Rec* __restrict__ rec, Rec* __restrict__ G, int rec_fields)
{
  const Where w = locate(Ln);
  const Params<double>& Pt = P[w.t];
  if (w.node < Pt.n) gfield_node<Rec, W>(Pt, rec + (size_t)rec_fields * w.base, G + 3 * w.base, w.node);
}

// PART 0: all lattices; 1 and 2: the species lattices, then the momentum and
// energy lattices, as two launches with fewer registers each (a launch choice).
template <typename S, int M, int V, int PART>
constexpr int collide_part_waves() { return PART == 0 ? collide_waves<S, M, V>() : 2; }

template <typename S, typename R, typename Rec, int M, int W, int V, int PART, bool WEAK, bool CVT>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(collide_part_waves<S, M, V, PART>()))) void k_collide(const Params<R>* __restrict__ P, Launch Ln, const S* __restrict__ src,
                                                   S* __restrict__ dst, const Rec* __restrict__ rec,
                                                   const Rec* __restrict__ G, StepNo sn)
{
  const Where w = locate(Ln);
  const Params<R>& Pt = P[w.t];
  if (w.node < Pt.n) {
    const size_t po = pop_stride<M, WEAK>() * w.base;
    collide_node<S, R, Rec, M, W, PART, WEAK, CVT>(Pt, src + po, dst + po,
                                                   rec + (size_t)RecLayout<M, WEAK, CVT>::FIELDS * w.base,
                                                   G + 3 * w.base, w.node, step_of(sn));
  }
}

// The two-read step: the moments pass also collides and streams the species
// lattices (k_state_species); the second pass collides and streams the momentum
// and energy lattices (k_collide_fg). The two write disjoint lattices of dst.
template <typename S, typename R, typename Rec, int M, int W, int V, bool WEAK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(moment_waves<M, V>()))) void k_state_species(
    const Params<R>* __restrict__ P, Launch Ln, const S* __restrict__ src, S* __restrict__ dst, Rec* __restrict__ rec,
    StepNo sn)
{
  const Where w = locate(Ln);
  const Params<R>& Pt = P[w.t];
  static_assert(RecLayout<M, WEAK, false>::FIELDS >= REC2_FIELDS, "the two-read record fits the record buffer");
  if (w.node < Pt.n) {
    const size_t po = pop_stride<M, WEAK>() * w.base;
    state_species_node<S, R, Rec, M, W, WEAK>(Pt, src + po, dst + po,
                                              rec + (size_t)RecLayout<M, WEAK, false>::FIELDS * w.base, w.node,
                                              step_of(sn));
  }
}

// Occupancy targets of k_collide_fg: two waves per SIMD (variant 0; about 230
// registers), or no bound on the registers (variant 1: one wave per SIMD).
template <int V>
constexpr int collide_fg_waves() { return V == 0 ? 2 : 1; }

template <typename S, typename R, typename Rec, int M, int W, int V, bool WEAK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(collide_fg_waves<V>()))) void k_collide_fg(
    const Params<R>* __restrict__ P, Launch Ln, const S* __restrict__ src, S* __restrict__ dst,
    const Rec* __restrict__ rec, const Rec* __restrict__ G, StepNo sn)
{
  const Where w = locate(Ln);
  const Params<R>& Pt = P[w.t];
  if (w.node < Pt.n) {
    const size_t po = pop_stride<M, WEAK>() * w.base;
    fg_collide_node<S, R, Rec, M, W, WEAK>(Pt, src + po, dst + po,
                                           rec + (size_t)RecLayout<M, WEAK, false>::FIELDS * w.base,
                                           G + 3 * w.base, w.node, step_of(sn));
  }
}

// Open x ends: rewrite the populations entering the two boundary planes after
// the collision (a launch over all nodes; only x = 0 and x = nx - 1 write).
template <typename S, typename R, int M, bool WEAK>
__global__ __launch_bounds__(BLOCK) void k_open_fix(const Params<R>* __restrict__ P, Launch Ln, S* __restrict__ dst,
                                                    StepNo sn)
{
  const Where w = locate(Ln);
  const Params<R>& Pt = P[w.t];
  if (w.node < Pt.n) open_fix_node<S, R, Lat<M, WEAK>::L>(Pt, dst + pop_stride<M, WEAK>() * w.base, w.node, step_of(sn));
}

// Opposed jets: rewrite what enters the outlet rows and the nozzles after the
// collision (a launch over all nodes; only boundary rows and faces write).
template <typename S, typename R, int M, bool WEAK>
__global__ __launch_bounds__(BLOCK) void k_jets_fix(const Params<R>* __restrict__ P, Launch Ln, S* __restrict__ dst,
                                                    StepNo sn)
{
  const Where w = locate(Ln);
  const Params<R>& Pt = P[w.t];
  if (w.node < Pt.n) jets_fix_node<S, R, Lat<M, WEAK>::L>(Pt, dst + pop_stride<M, WEAK>() * w.base, w.node, step_of(sn));
}

template <typename T>
__device__ inline T* seg(T* p, int64_t off) { return p ? p + off : p; }

template <typename S, typename R, int M, bool WEAK, bool CVT>
__global__ __launch_bounds__(BLOCK) void k_read(const Params<R>* __restrict__ P, Launch Ln, const S* __restrict__ pop,
                                                double* X, double* rho, double* u, double* p, double* T)
{
  const Where w = locate(Ln);
  const Params<R>& Pt = P[w.t];
  if (w.node < Pt.n)
    read_node<S, R, M, WEAK, CVT>(Pt, pop + pop_stride<M, WEAK>() * w.base, w.node, seg(X, M * w.base),
                             seg(rho, w.base), seg(u, 3 * w.base), seg(p, w.base), seg(T, w.base));
}

// Block sum of NV doubles per thread into out[slot * NV + k] (fixed order).
template <int NV>
__device__ inline void block_sum(const double (&v)[NV], double* out, uint32_t slot)
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
    out[(size_t)slot * NV + threadIdx.x] = s;
  }
}

static_assert(RED_BLOCK == BLOCK, "reductions use the launch blocks of the tubes");

template <typename S, int M, bool WEAK>
__global__ __launch_bounds__(RED_BLOCK) void k_conserved(const Params<double>* __restrict__ P, Launch Ln,
                                                         const S* __restrict__ pop, double* __restrict__ partial)
{
  constexpr int NV = M + 6;
  double v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = 0.0;
  const Where w = locate(Ln);
  const Params<double>& Pt = P[w.t];
  if (w.node < Pt.n) conserved_node<S, M, WEAK>(Pt, pop + pop_stride<M, WEAK>() * w.base, w.node, v);
  block_sum<NV>(v, partial, w.block);
}

// Moles of every species in each x half of every tube (block partials [2 M]).
template <typename S, int M, bool WEAK>
__global__ __launch_bounds__(RED_BLOCK) void k_half_moles(const Params<double>* __restrict__ P, Launch Ln,
                                                          const S* __restrict__ pop, double* __restrict__ partial)
{
  constexpr int NV = 2 * M;
  double v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = 0.0;
  const Where w = locate(Ln);
  const Params<double>& Pt = P[w.t];
  if (w.node < Pt.n) half_moles_node<S, M, WEAK>(Pt, pop + pop_stride<M, WEAK>() * w.base, w.node, v);
  block_sum<NV>(v, partial, w.block);
}

// Sums of the initial fields (X_a, p, T) per tube, for the reference states
// (the parameter blocks are not filled yet: tube sizes come from tube_n).
template <int M>
__global__ __launch_bounds__(RED_BLOCK) void k_field_sums(const int64_t* __restrict__ tube_n, Launch Ln,
                                                          const double* __restrict__ X,
                                                          const double* __restrict__ p,
                                                          const double* __restrict__ T, double* __restrict__ partial)
{
  constexpr int NV = M + 2;
  double v[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = 0.0;
  const Where w = locate(Ln);
  const int64_t n = tube_n[w.t];
  if (w.node < n) {
#pragma unroll
    for (int a = 0; a < M; ++a) v[a] = X[(size_t)M * w.base + (size_t)a * n + w.node];
    v[M] = p[w.base + w.node];
    v[M + 1] = T[w.base + w.node];
  }
  block_sum<NV>(v, partial, w.block);
}

template <typename S, int M, bool WEAK, bool CVT>
__global__ __launch_bounds__(BLOCK) void k_init(const Params<double>* __restrict__ P, Launch Ln,
                                                const double* __restrict__ X, const double* __restrict__ p,
                                                const double* __restrict__ T, const double* __restrict__ u,
                                                S* __restrict__ pop, int* __restrict__ block_bad)
{
  const Where w = locate(Ln);
  const Params<double>& Pt = P[w.t];
  int bad = 0;
  if (w.node < Pt.n)
    bad = init_node<S, M, WEAK, CVT>(Pt, X + (size_t)M * w.base, p + w.base, T + w.base, u + 3 * w.base,
                                pop + pop_stride<M, WEAK>() * w.base, w.node);
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) block_bad[w.block] = bad;
}

// Fixed-point storage: the smallest and largest stored integer of every lattice
// and direction class of every tube, into out[((t MAXL + l) NCLS + k) 2 + {0, 1}]
// (the host sets the entries to 32767 and -32767 first). A launch over the
// linear numbering: every wavefront lies in one tube.
template <int M, bool WEAK>
__global__ __launch_bounds__(BLOCK) void k_range16(const Params<double>* __restrict__ P, Launch Ln,
                                                   const int16_t* __restrict__ pop, int32_t* __restrict__ out)
{
  constexpr int L = Lat<M, WEAK>::L;
  const Where w = locate(Ln);
  const Params<double>& Pt = P[w.t];
  int lo[L][NCLS], hi[L][NCLS];
#pragma unroll
  for (int l = 0; l < L; ++l)
#pragma unroll
    for (int k = 0; k < NCLS; ++k) {
      lo[l][k] = 32767;
      hi[l][k] = -32767;
    }
  if (w.node < Pt.n) {
    const int16_t* pb = pop + pop_stride<M, WEAK>() * w.base;
    const size_t n = (size_t)Pt.n;
#pragma unroll
    for (int l = 0; l < L; ++l)
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const int v = pb[(size_t)(l * Q + i) * n + w.node];
        lo[l][ccls(i)] = min(lo[l][ccls(i)], v);
        hi[l][ccls(i)] = max(hi[l][ccls(i)], v);
      }
  }
#pragma unroll
  for (int l = 0; l < L; ++l)
#pragma unroll
    for (int k = 0; k < NCLS; ++k) {
      int a = lo[l][k], b = hi[l][k];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        a = min(a, __shfl_xor(a, off, 64));
        b = max(b, __shfl_xor(b, off, 64));
      }
      if ((threadIdx.x & 63) == 0) {
        int32_t* o = out + ((size_t)(w.t * MAXL + l) * NCLS + k) * 2;
        atomicMin(o, a);
        atomicMax(o + 1, b);
      }
    }
}

// Fixed-point storage: re-encode every stored value with new tables,
// tab[((t MAXL + l) NCLS + k) 4 + {0, 1, 2, 3}] = old centre, old decoding
// factor, new centre, new encoding factor of tube t, lattice l, class k; the new
// integer is rounded stochastically (seeded by node, lattice and seed). A tube
// whose old decoding factors are zero keeps its values.
template <int M, bool WEAK>
__global__ __launch_bounds__(BLOCK) void k_rebase16(const Params<double>* __restrict__ P, Launch Ln,
                                                    int16_t* __restrict__ pop, const double* __restrict__ tab,
                                                    uint32_t seed)
{
  constexpr int L = Lat<M, WEAK>::L;
  const Where w = locate(Ln);
  const Params<double>& Pt = P[w.t];
  if (w.node >= Pt.n || tab[(size_t)w.t * MAXL * NCLS * 4 + 1] == 0.0) return;
  int16_t* pb = pop + pop_stride<M, WEAK>() * w.base;
  const size_t n = (size_t)Pt.n;
#pragma unroll
  for (int l = 0; l < L; ++l) {
    Rng rng(w.node, l + 32, seed);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double* tb = tab + ((size_t)(w.t * MAXL + l) * NCLS + ccls(i)) * 4;
      int16_t& v = pb[(size_t)(l * Q + i) * n + w.node];
      const double f = tb[0] + double(v) * tb[1];
      v = cvt_sr_i16(float((f - tb[2]) * tb[3]), rng.next());
    }
  }
}

// ---------------------------------------------------------------------------
// Dispatch over (storage, arithmetic, species count, walls, coupling, occupancy variant)
// ---------------------------------------------------------------------------
constexpr int NVARIANT = 2;

struct Ops {
  size_t s_bytes;   // bytes per stored population
  size_t r_bytes;   // bytes per record value
  int rec_fields;   // values per node in the record
  void (*moments[NVARIANT])(const void* P, const Launch& ln, const void* pop, void* rec, unsigned grid,
                            hipStream_t st);
  void (*gfield)(const void* P, const Launch& ln, const void* rec, void* G, int rec_fields, unsigned grid,
                 hipStream_t st);
  void (*collide[NVARIANT])(const void* P, const Launch& ln, const void* src, void* dst, const void* rec,
                            const void* G, StepNo sn, unsigned grid, hipStream_t st);
  // split collision: [0] species lattices, [1] momentum and energy lattices
  void (*collide_split[2])(const void* P, const Launch& ln, const void* src, void* dst, const void* rec,
                           const void* G, StepNo sn, unsigned grid, hipStream_t st);
  void (*read)(const void* P, const Launch& ln, const void* pop, double* X, double* rho, double* u, double* p,
               double* T, unsigned grid, hipStream_t st);
  void (*conserved)(const void* Pd, const Launch& ln, const void* pop, double* partial, unsigned grid,
                    hipStream_t st);
  void (*half_moles)(const void* Pd, const Launch& ln, const void* pop, double* partial, unsigned grid,
                     hipStream_t st);
  void (*init)(const void* Pd, const Launch& ln, const double* X, const double* p, const double* T,
               const double* u, void* pop, int* bad, unsigned grid, hipStream_t st);
  // the two-read step (null where not compiled: temperature-dependent properties)
  void (*state_species[NVARIANT])(const void* P, const Launch& ln, const void* src, void* dst, void* rec, StepNo sn,
                                  unsigned grid, hipStream_t st);
  void (*collide_fg[NVARIANT])(const void* P, const Launch& ln, const void* src, void* dst, const void* rec,
                               const void* G, StepNo sn, unsigned grid, hipStream_t st);
  // open x ends only (else null): after each collision, on its destination buffer
  void (*open_fix)(const void* P, const Launch& ln, void* dst, StepNo sn, unsigned grid, hipStream_t st);
  void (*field_sums)(const int64_t* tube_n, const Launch& ln, const double* X, const double* p, const double* T,
                     double* partial, unsigned grid, hipStream_t st);
  // fixed-point storage only (else null): range of the stored integers, re-encoding
  void (*range16)(const void* Pd, const Launch& ln, const void* pop, int32_t* out, unsigned grid, hipStream_t st);
  void (*rebase16)(const void* Pd, const Launch& ln, void* pop, const double* tab, uint32_t seed, unsigned grid,
                   hipStream_t st);
};

template <typename S, typename Rec, int M, int V, bool WEAK, bool CVT>
void launch_moments(const void* Pd, const Launch& ln, const void* pop, void* rec, unsigned grid, hipStream_t st)
{
  hipLaunchKernelGGL((k_moments<S, Rec, M, V, WEAK, CVT>), dim3(grid), dim3(BLOCK), 0, st, (const Params<double>*)Pd, ln,
                     (const S*)pop, (Rec*)rec);
}

template <typename S, typename R, typename Rec, int M, int W, int V, int PART, bool WEAK, bool CVT>
void launch_collide(const void* P, const Launch& ln, const void* src, void* dst, const void* rec, const void* G,
                    StepNo sn, unsigned grid, hipStream_t st)
{
  hipLaunchKernelGGL((k_collide<S, R, Rec, M, W, V, PART, WEAK, CVT>), dim3(grid), dim3(BLOCK), 0, st,
                     (const Params<R>*)P, ln, (const S*)src, (S*)dst, (const Rec*)rec, (const Rec*)G, sn);
}

template <typename S, typename R, typename Rec, int M, int W, int V, bool WEAK>
void launch_state_species(const void* P, const Launch& ln, const void* src, void* dst, void* rec, StepNo sn,
                          unsigned grid, hipStream_t st)
{
  hipLaunchKernelGGL((k_state_species<S, R, Rec, M, W, V, WEAK>), dim3(grid), dim3(BLOCK), 0, st,
                     (const Params<R>*)P, ln, (const S*)src, (S*)dst, (Rec*)rec, sn);
}

template <typename S, typename R, typename Rec, int M, int W, int V, bool WEAK>
void launch_collide_fg(const void* P, const Launch& ln, const void* src, void* dst, const void* rec, const void* G,
                       StepNo sn, unsigned grid, hipStream_t st)
{
  hipLaunchKernelGGL((k_collide_fg<S, R, Rec, M, W, V, WEAK>), dim3(grid), dim3(BLOCK), 0, st,
                     (const Params<R>*)P, ln, (const S*)src, (S*)dst, (const Rec*)rec, (const Rec*)G, sn);
}

template <typename S, typename R, typename Rec, int M, int W, bool WEAK, bool CVT>
Ops make_ops()
{
  Ops o;
  o.s_bytes = sizeof(S);
  o.r_bytes = sizeof(Rec);
  o.rec_fields = RecLayout<M, WEAK, CVT>::FIELDS;
  o.moments[0] = launch_moments<S, Rec, M, 0, WEAK, CVT>;
  o.moments[1] = launch_moments<S, Rec, M, 1, WEAK, CVT>;
  o.collide[0] = launch_collide<S, R, Rec, M, W, 0, 0, WEAK, CVT>;
  o.collide[1] = launch_collide<S, R, Rec, M, W, 1, 0, WEAK, CVT>;
  o.collide_split[0] = launch_collide<S, R, Rec, M, W, 0, 1, WEAK, CVT>;
  o.collide_split[1] = launch_collide<S, R, Rec, M, W, 0, 2, WEAK, CVT>;
  if constexpr (!CVT) {
    o.state_species[0] = launch_state_species<S, R, Rec, M, W, 0, WEAK>;
    o.state_species[1] = launch_state_species<S, R, Rec, M, W, 1, WEAK>;
    o.collide_fg[0] = launch_collide_fg<S, R, Rec, M, W, 0, WEAK>;
    o.collide_fg[1] = launch_collide_fg<S, R, Rec, M, W, 1, WEAK>;
  } else {
    o.state_species[0] = o.state_species[1] = nullptr;
    o.collide_fg[0] = o.collide_fg[1] = nullptr;
  }
  o.gfield = [](const void* Pd, const Launch& ln, const void* rec, void* G, int rec_fields, unsigned grid,
                hipStream_t st) {
    hipLaunchKernelGGL((k_gfield<Rec, W>), dim3(grid), dim3(BLOCK), 0, st, (const Params<double>*)Pd, ln,
                       (const Rec*)rec, (Rec*)G, rec_fields);
  };
  o.read = [](const void* P, const Launch& ln, const void* pop, double* X, double* rho, double* u, double* p,
              double* T, unsigned grid, hipStream_t st) {
    hipLaunchKernelGGL((k_read<S, R, M, WEAK, CVT>), dim3(grid), dim3(BLOCK), 0, st, (const Params<R>*)P, ln, (const S*)pop,
                       X, rho, u, p, T);
  };
  o.conserved = [](const void* Pd, const Launch& ln, const void* pop, double* partial, unsigned grid,
                   hipStream_t st) {
    hipLaunchKernelGGL((k_conserved<S, M, WEAK>), dim3(grid), dim3(RED_BLOCK), 0, st, (const Params<double>*)Pd, ln,
                       (const S*)pop, partial);
  };
  o.half_moles = [](const void* Pd, const Launch& ln, const void* pop, double* partial, unsigned grid,
                     hipStream_t st) {
    hipLaunchKernelGGL((k_half_moles<S, M, WEAK>), dim3(grid), dim3(RED_BLOCK), 0, st, (const Params<double>*)Pd, ln,
                       (const S*)pop, partial);
  };
  o.init = [](const void* Pd, const Launch& ln, const double* X, const double* p, const double* T,
              const double* u, void* pop, int* bad, unsigned grid, hipStream_t st) {
    hipLaunchKernelGGL((k_init<S, M, WEAK, CVT>), dim3(grid), dim3(BLOCK), 0, st, (const Params<double>*)Pd, ln, X, p, T, u,
                       (S*)pop, bad);
  };
  o.field_sums = [](const int64_t* tube_n, const Launch& ln, const double* X, const double* p, const double* T,
                    double* partial, unsigned grid, hipStream_t st) {
    hipLaunchKernelGGL((k_field_sums<M>), dim3(grid), dim3(RED_BLOCK), 0, st, tube_n, ln, X, p, T, partial);
  };
  o.range16 = nullptr;
  o.rebase16 = nullptr;
  if constexpr (is_fixed16<S>()) {
    o.range16 = [](const void* Pd, const Launch& ln, const void* pop, int32_t* out, unsigned grid, hipStream_t st) {
      hipLaunchKernelGGL((k_range16<M, WEAK>), dim3(grid), dim3(BLOCK), 0, st, (const Params<double>*)Pd, ln,
                         (const int16_t*)pop, out);
    };
    o.rebase16 = [](const void* Pd, const Launch& ln, void* pop, const double* tab, uint32_t seed, unsigned grid,
                    hipStream_t st) {
      hipLaunchKernelGGL((k_rebase16<M, WEAK>), dim3(grid), dim3(BLOCK), 0, st, (const Params<double>*)Pd, ln,
                         (int16_t*)pop, tab, seed);
    };
  }
  o.open_fix = nullptr;
  if constexpr (xbc(W) == BC_OPEN) {
    o.open_fix = [](const void* P, const Launch& ln, void* dst, StepNo sn, unsigned grid, hipStream_t st) {
      hipLaunchKernelGGL((k_open_fix<S, R, M, WEAK>), dim3(grid), dim3(BLOCK), 0, st, (const Params<R>*)P, ln, (S*)dst, sn);
    };
  } else if constexpr (xbc(W) == BC_JETS) {
    o.open_fix = [](const void* P, const Launch& ln, void* dst, StepNo sn, unsigned grid, hipStream_t st) {
      hipLaunchKernelGGL((k_jets_fix<S, R, M, WEAK>), dim3(grid), dim3(BLOCK), 0, st, (const Params<R>*)P, ln, (S*)dst, sn);
    };
  }
  return o;
}

// walls: 0 periodic x, 1 walls at both x ends (BC_PERIODIC, BC_WALLS)
template <typename S, typename R, typename Rec, bool WEAK, bool CVT = false>
bool pick_m(int M, int walls, Ops& o)
{
  switch (M) {
    case 2: o = walls ? make_ops<S, R, Rec, 2, BC_WALLS, WEAK, CVT>() : make_ops<S, R, Rec, 2, BC_PERIODIC, WEAK, CVT>(); return true;
    case 3: o = walls ? make_ops<S, R, Rec, 3, BC_WALLS, WEAK, CVT>() : make_ops<S, R, Rec, 3, BC_PERIODIC, WEAK, CVT>(); return true;
    case 4: o = walls ? make_ops<S, R, Rec, 4, BC_WALLS, WEAK, CVT>() : make_ops<S, R, Rec, 4, BC_PERIODIC, WEAK, CVT>(); return true;
    default: return false;
  }
}

// free-slip y walls with periodic (walls_x = 0) or walled (1) x ends
template <typename S, typename R, typename Rec, bool WEAK = false, bool CVT = false>
bool pick_m_yslip(int M, int walls_x, Ops& o)
{
  constexpr int P = BC_YSLIP | BC_PERIODIC, Wl = BC_YSLIP | BC_WALLS;
  switch (M) {
    case 2: o = walls_x ? make_ops<S, R, Rec, 2, Wl, WEAK, CVT>() : make_ops<S, R, Rec, 2, P, WEAK, CVT>(); return true;
    case 3: o = walls_x ? make_ops<S, R, Rec, 3, Wl, WEAK, CVT>() : make_ops<S, R, Rec, 3, P, WEAK, CVT>(); return true;
    case 4: o = walls_x ? make_ops<S, R, Rec, 4, Wl, WEAK, CVT>() : make_ops<S, R, Rec, 4, P, WEAK, CVT>(); return true;
    default: return false;
  }
}

// open x ends (periodic y)
template <typename S, typename R, typename Rec, bool WEAK = false, bool CVT = false>
bool pick_m_open(int M, Ops& o)
{
  switch (M) {
    case 2: o = make_ops<S, R, Rec, 2, BC_OPEN, WEAK, CVT>(); return true;
    case 3: o = make_ops<S, R, Rec, 3, BC_OPEN, WEAK, CVT>(); return true;
    case 4: o = make_ops<S, R, Rec, 4, BC_OPEN, WEAK, CVT>(); return true;
    default: return false;
  }
}

// the opposed jets (nozzle faces in x, outlets in y)
template <typename S, typename R, typename Rec, bool WEAK = false, bool CVT = false>
bool pick_m_jets(int M, Ops& o)
{
  constexpr int J = BC_JETS | BC_YOUT;
  switch (M) {
    case 2: o = make_ops<S, R, Rec, 2, J, WEAK, CVT>(); return true;
    case 3: o = make_ops<S, R, Rec, 3, J, WEAK, CVT>(); return true;
    case 4: o = make_ops<S, R, Rec, 4, J, WEAK, CVT>(); return true;
    default: return false;
  }
}

// every boundary set: walls = the x mode (0 periodic, 1 walls, 2 open) plus 4
// for free-slip y walls (not with open x ends)
template <typename S, typename R, typename Rec, bool WEAK, bool CVT>
bool pick_m_any(int M, int walls, Ops& o)
{
  const int wx = walls & 3;
  if (walls & 4) return wx != 2 && pick_m_yslip<S, R, Rec, WEAK, CVT>(M, wx, o);
  if (wx == 2) return pick_m_open<S, R, Rec, WEAK, CVT>(M, o);
  return pick_m<S, R, Rec, WEAK, CVT>(M, wx, o);
}

}  // namespace kern

// One entry point per instantiated (storage, arithmetic) pair. walls: the x
// boundary (0 periodic, 1 walls, 2 open, 3 opposed jets) plus 4 for free-slip y
// walls or 8 for outlets at the y ends (with the jets only); weak: 1
// for weak coupling; cvt: 1 for temperature-dependent specific heats and
// transport. Open ends, free-slip walls, weak coupling and the temperature-
// dependent kernels are compiled for FP64 and FP32 storage with FP64
// arithmetic only, in every combination (free-slip y walls not with open x ends).
bool pick_fp64(int M, int walls, int weak, int cvt, kern::Ops& o);
bool pick_fp32_fp64(int M, int walls, int weak, int cvt, kern::Ops& o);
bool pick_fp32(int M, int walls, int weak, int cvt, kern::Ops& o);
bool pick_fp16(int M, int walls, int weak, int cvt, kern::Ops& o);
bool pick_bf16(int M, int walls, int weak, int cvt, kern::Ops& o);
bool pick_i16(int M, int walls, int weak, int cvt, kern::Ops& o);

}  // namespace mclbm
