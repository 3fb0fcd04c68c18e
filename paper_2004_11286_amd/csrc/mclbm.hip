// mclbm.hip -- context management and the C ABI of libmclbm (include/mclbm.h).
//
// One time step = three launches over all nodes of all tubes, one thread per node:
//   k_moments  read the 27 L populations (L = M + 1 stored lattices under strong
//              coupling, M + 2 under weak) -> node record (FP64 state, Sec. 2.5.3,
//              3.2, 3.4: Phi, omega, C_p, rho, u, T, omega_1, q_neq, rho_a, V_a;
//              u_s under weak coupling, Y_a with temperature-dependent heat
//              capacities)
//   k_gfield   G_a = (1/omega - 1/2) d_a Phi_a from the records of the neighbours
//   k_collide  read the populations again, X_a = -d_a G_a and d C_p (or d Y_a)
//              from the neighbours, collide every lattice, push to the neighbours
//              of the other buffer (bounce-back at x walls); with open x ends a
//              fourth launch, k_open_fix, rewrites what enters the end planes
// The two reads of the populations are forced by the non-local terms of the
// momentum and energy collisions, which need the neighbours' moments at the same
// time level (eqs Xalpha and corrFourier). Populations are laid out as
// pop[l][i][z][y][x] per tube so that a wavefront's 64 lanes read and write 64
// consecutive values of one (lattice, direction) plane.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/mclbm.h"
#include "../../include/mclbm_nn.h"
#include "kernels.hpp"
#include "nn_internal.hpp"
#include "params_host.hpp"

using namespace mclbm;

namespace {

using kern::ALIGN;
using kern::align_up;
using kern::BLOCK;
using kern::Launch;
using kern::Ops;
using kern::RED_BLOCK;
using kern::StepNo;

// Deterministic second stage of the reductions: out[t][k] = sum over the blocks
// of tube t of partial[b][k], in a fixed order. One block per tube.
__global__ __launch_bounds__(RED_BLOCK) void k_reduce_tubes(const double* __restrict__ partial,
                                                            const kern::Tube* __restrict__ tubes, int nv,
                                                            double* __restrict__ out)
{
  __shared__ double buf[RED_BLOCK];
  const kern::Tube tb = tubes[blockIdx.x];
  for (int k = 0; k < nv; ++k) {
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < tb.nblocks; b += RED_BLOCK)
      s += partial[(size_t)(tb.first_block + b) * nv + k];
    buf[threadIdx.x] = s;
    __syncthreads();
    for (int w = RED_BLOCK / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) buf[threadIdx.x] += buf[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[(size_t)blockIdx.x * nv + k] = buf[0];
    __syncthreads();
  }
}

// Device step counter of graph replays (single thread, vector stores).
__global__ void k_counter_set(uint32_t* ctr, uint32_t v)
{
  if (threadIdx.x == 0 && blockIdx.x == 0) *ctr = v;
}
__global__ void k_counter_add(uint32_t* ctr, uint32_t v)
{
  if (threadIdx.x == 0 && blockIdx.x == 0) *ctr += v;
}

// FP32 trajectory fields from the double read-back: out[(M+5) base + k n_t + node],
// k = X_1..X_M, T, u_x, u_y, u_z, p.
__global__ __launch_bounds__(BLOCK) void k_pack_f32(Launch ln, const int64_t* __restrict__ tube_n, int M,
                                                   const double* __restrict__ X, const double* __restrict__ T,
                                                   const double* __restrict__ u, const double* __restrict__ p,
                                                   float* __restrict__ out)
{
  const kern::Where w = kern::locate(ln);
  const int64_t n = tube_n[w.t];
  if (w.node >= n) return;
  const int64_t b = w.base, i = w.node;
  float* o = out + (size_t)(M + 5) * b;
  for (int a = 0; a < M; ++a) o[(size_t)a * n + i] = (float)X[(size_t)M * b + (size_t)a * n + i];
  o[(size_t)M * n + i] = (float)T[b + i];
  for (int k = 0; k < 3; ++k) o[(size_t)(M + 1 + k) * n + i] = (float)u[3 * b + (size_t)k * n + i];
  o[(size_t)(M + 4) * n + i] = (float)p[b + i];
}

// Predicted fields (FP32 [M+5][n_t] per tube: X_1..X_M, T, u, p) -> FP64 fields
// for mclbm_init_fields: mole fractions clipped at zero and renormalised; a
// block flags a node whose state the equilibria cannot represent (T <= 0,
// p <= 0, R_a T + u^2 >= 1 for a species or the mixture, no species left) and
// writes the largest change of a mole fraction over its nodes, the installed
// X_a against the network's input fields `in` (same layout as pred).
__global__ __launch_bounds__(BLOCK) void k_pred_to_state(const Params<double>* __restrict__ P, Launch ln, int M,
                                                        const float* __restrict__ in, const float* __restrict__ pred,
                                                        double* __restrict__ X, double* __restrict__ p,
                                                        double* __restrict__ T, double* __restrict__ u,
                                                        int* __restrict__ block_bad, float* __restrict__ block_chg)
{
  __shared__ float wave_chg[BLOCK / 64];
  const kern::Where w = kern::locate(ln);
  const Params<double>& Pt = P[w.t];
  int bad = 0;
  float chg = 0.0f;
  if (w.node < Pt.n) {
    const int64_t n = Pt.n, b = w.base, i = w.node;
    const float* f = pred + (size_t)(M + 5) * b;
    const float* x0 = in + (size_t)(M + 5) * b;
    double xs[MAXM], sum = 0.0, mmix = 0.0;
    for (int a = 0; a < M; ++a) {
      xs[a] = fmax((double)f[(size_t)a * n + i], 0.0);
      sum += xs[a];
    }
    if (!(sum > 0.0)) bad = 1;
    const double Tn = (double)f[(size_t)M * n + i];
    double uu[3], usq = 0.0;
    for (int k = 0; k < 3; ++k) {
      uu[k] = (double)f[(size_t)(M + 1 + k) * n + i];
      usq += uu[k] * uu[k];
    }
    for (int a = 0; a < M; ++a) {
      xs[a] = sum > 0.0 ? xs[a] / sum : 0.0;
      mmix += xs[a] * Pt.m[a];
      if (!(Tn * Pt.inv_m[a] + usq < 1.0)) bad = 1;
      chg = fmaxf(chg, (float)fabs(xs[a] - (double)x0[(size_t)a * n + i]));
    }
    const double pn = (double)f[(size_t)(M + 4) * n + i];
    if (!(Tn > 0.0) || !(pn > 0.0) || !(mmix > 0.0) || !(Tn / mmix + usq < 1.0)) bad = 1;
    for (int a = 0; a < M; ++a) X[(size_t)M * b + (size_t)a * n + i] = xs[a];
    T[b + i] = Tn;
    p[b + i] = pn;
    for (int k = 0; k < 3; ++k) u[3 * b + (size_t)k * n + i] = uu[k];
  }
  for (int off = 32; off > 0; off >>= 1) chg = fmaxf(chg, __shfl_xor(chg, off, 64));
  if ((threadIdx.x & 63) == 0) wave_chg[threadIdx.x >> 6] = chg;
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) {
    float m = wave_chg[0];
    for (int k = 1; k < BLOCK / 64; ++k) m = fmaxf(m, wave_chg[k]);
    block_bad[w.block] = bad;
    block_chg[w.block] = m;
  }
}

// Conserved sums of the state mclbm_init_fields installs for FP64 fields (X, p, T,
// u per tube, as in k_pred_to_state's output): per node rho_1 .. rho_M and rho E
// of the local equilibrium (rho = p m / T, rho_a = rho Y_a, rho E = rho (U(T) +
// u^2/2) with U the mixture's internal energy from T_0 = 0); block partials
// [MAXM + 1] in the slots of kern::block_sum.
__global__ __launch_bounds__(BLOCK) void k_field_conserved(const Params<double>* __restrict__ P, Launch ln, int M,
                                                          const double* __restrict__ X, const double* __restrict__ p,
                                                          const double* __restrict__ T, const double* __restrict__ u,
                                                          double* __restrict__ partial)
{
  constexpr int NV = MAXM + 1;
  double v[NV];
  for (int k = 0; k < NV; ++k) v[k] = 0.0;
  const kern::Where w = kern::locate(ln);
  const Params<double>& Pt = P[w.t];
  if (w.node < Pt.n) {
    const int64_t n = Pt.n, b = w.base, i = w.node;
    double mmix = 0.0, Y[MAXM];
    for (int a = 0; a < M; ++a) mmix += X[(size_t)M * b + (size_t)a * n + i] * Pt.m[a];
    const double Tn = T[b + i];
    const double rho = p[b + i] * mmix / Tn;
    double usq = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double uk = u[3 * b + (size_t)k * n + i];
      usq += uk * uk;
    }
    double U = 0.0;                      // sum_a Y_a int_0^T C_{a,v}
    for (int a = 0; a < M; ++a) {
      Y[a] = X[(size_t)M * b + (size_t)a * n + i] * Pt.m[a] / mmix;
      v[a] = rho * Y[a];
      const double* c = Pt.cvc[a];
      U += Y[a] * Tn * (c[0] + Tn * (c[1] * 0.5 + Tn * (c[2] * (1.0 / 3.0) + Tn * (c[3] * 0.25))));
    }
    v[MAXM] = rho * (U + 0.5 * usq);
  }
  kern::block_sum<NV>(v, partial, w.block);
}

bool pick_ops(int precision, int M, int walls, int weak, int cvt, Ops& o)
{
  switch (precision) {
    case MCLBM_FP64: return pick_fp64(M, walls, weak, cvt, o);
    case MCLBM_FP32: return pick_fp32_fp64(M, walls, weak, cvt, o);
    case MCLBM_FP32_FP32: return pick_fp32(M, walls, weak, cvt, o);
    case MCLBM_FP16: return pick_fp16(M, walls, weak, cvt, o);
    case MCLBM_BF16: return pick_bf16(M, walls, weak, cvt, o);
    case MCLBM_I16: return pick_i16(M, walls, weak, cvt, o);
    default: return false;
  }
}

bool compute_is_fp64(int precision) { return precision == MCLBM_FP64 || precision == MCLBM_FP32; }

thread_local std::string g_last_error;

const char* kernel_names[3] = {"k_moments", "k_gfield", "k_collide"};
const char* kernel_names_two_read[3] = {"k_state_species", "k_gfield", "k_collide_fg"};

struct TubeHost {
  int nx = 0, ny = 0, nz = 0;
  int64_t n = 0, base = 0;
  HostSpecies hs{};
  RefTables tab{};
  double inlet[MAXM + 5] = {};   // open x ends and the jet at x = 0: X (M), p, T, u (3)
  double inlet2[MAXM + 5] = {};  // opposed jets: the jet at x = nx - 1
  int noz0 = 0, noz1 = 0;        // opposed jets: nozzle rows
};

}  // namespace

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
struct mclbm_ctx {
  int M = 0, wall_x = 0, wall_y = 0, precision = 0, weak = 0, cvt = 0, L = 0, ntubes = 0;
  int64_t n = 0;            // nodes over all tubes
  int64_t nblocks = 0;      // launch blocks over all tubes
  std::vector<TubeHost> tubes;
  Ops ops{};
  hipStream_t stream = nullptr;
  int device = 0;
  // workspace regions
  char* ws = nullptr;
  size_t ws_bytes = 0;
  void* dPd = nullptr;      // Params<double>[ntubes]
  void* dPr = nullptr;      // Params<float>[ntubes], or alias of dPd
  kern::Tube* dTubes = nullptr;
  int32_t* dBlkTube = nullptr;
  int32_t* dBlkTubeT = nullptr;   // tube of every block of a tiled launch (block shape > 0)
  int64_t nblocks_t = 0;          // blocks of a tiled launch over all tubes (current shape)
  int64_t* dTubeN = nullptr;
  uint32_t* dStepCtr = nullptr;
  void* pop[2] = {nullptr, nullptr};
  void* rec = nullptr;
  void* G = nullptr;
  double* staging = nullptr;
  double* partial = nullptr;
  double* reduced = nullptr;
  int* bad = nullptr;
  float* chg = nullptr;           // mclbm_nn_advance: largest mole-fraction change per block
  uint32_t* dFlag = nullptr;      // fixed point: range flag per tube (bit 0 re-range, bit 1 a value clamped)
  int32_t* dRange = nullptr;      // fixed point: k_range16 output [ntubes][MAXL][NCLS][2]
  double* dTab = nullptr;         // fixed point: k_rebase16 tables [ntubes][MAXL][NCLS][4]
  int64_t reranges = 0;           // fixed point: re-encodings since mclbm_init_fields or mclbm_load
  int32_t xperm[MAXM] = {};       // the caller's index of the library's species a (slaved: a = M - 1)
  bool xperm_identity = true;
  int cur = 0;
  int64_t steps = 0;
  bool initialised = false;
  // host copies (kept alive for asynchronous uploads)
  std::vector<Params<double>> hPd;
  std::vector<Params<float>> hPf;
  std::vector<kern::Tube> hTubes;
  std::vector<int32_t> hBlkTube;
  std::vector<int32_t> hBlkTubeT;
  std::vector<int64_t> hTubeN;
  // launch configuration
  mclbm_launch lc{};
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  int gsteps = 0;           // steps in the instantiated graph
  std::string err;
  // timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, int>> ev_pairs[3];   // indices into ev_pool per kernel
  size_t ev_used = 0;
  double acc_ms[3] = {0, 0, 0};
  int64_t acc_launches[3] = {0, 0, 0};
};

namespace {

struct Layout {
  size_t pd, pr, tubes, blk, blkT, tube_n, ctr, flag, range, tab, pop, rec, G, staging, partial, reduced, bad, chg, total;
  int64_t n, nblocks, nblocks_tmax;
};

// Tiles of block shape k (> 0) over an nx x ny x nz grid: per row, per plane, total.
void tile_counts(int k, int nx, int ny, int nz, int32_t& tx, int32_t& ty, int64_t& total)
{
  const int sx = kern::SHAPE_SX[k], sy = kern::SHAPE_SY[k], sz = kern::LOG2_BLOCK - sx - sy;
  tx = (int32_t)((nx + (1 << sx) - 1) >> sx);
  ty = (int32_t)((ny + (1 << sy) - 1) >> sy);
  total = (int64_t)tx * ty * ((nz + (1 << sz) - 1) >> sz);
}

size_t storage_bytes(int precision)
{
  switch (precision) {
    case MCLBM_FP64: return 8;
    case MCLBM_FP16: case MCLBM_BF16: case MCLBM_I16: return 2;
    default: return 4;
  }
}

size_t record_bytes(int precision) { return precision == MCLBM_FP64 ? 8 : 4; }

Layout layout_for(const mclbm_params* tp, int ntubes)
{
  const int M = tp[0].M, precision = tp[0].precision, weak = tp[0].weak;
  const int cvt = tp[0].cv_coef != nullptr || tp[0].transport_exp != nullptr;
  Layout l{};
  l.n = 0;
  l.nblocks = 0;
  for (int t = 0; t < ntubes; ++t) {
    const int64_t n = (int64_t)tp[t].nx * tp[t].ny * tp[t].nz;
    l.n += n;
    l.nblocks += (n + BLOCK - 1) / BLOCK;
  }
  l.nblocks_tmax = 0;
  for (int k = 1; k < kern::NSHAPES; ++k) {
    int64_t tot = 0;
    for (int t = 0; t < ntubes; ++t) {
      int32_t tx, ty;
      int64_t nt;
      tile_counts(k, tp[t].nx, tp[t].ny, tp[t].nz, tx, ty, nt);
      tot += nt;
    }
    l.nblocks_tmax = std::max(l.nblocks_tmax, tot);
  }
  const size_t s_bytes = storage_bytes(precision), r_bytes = record_bytes(precision);
  // stored lattices and record fields (RecLayout): M-1 stored species under
  // strong coupling, M under weak coupling (which also records u_s)
  const int ns = weak ? M : M - 1;
  const int L = ns + 2;
  const int rec_fields = REC_RHOA + ns + 3 * M + (weak ? 3 : 0) + (cvt ? M - 1 : 0);
  size_t off = 0;
  l.pd = off; off += align_up(sizeof(Params<double>) * ntubes);
  l.pr = off; off += align_up(sizeof(Params<float>) * ntubes);
  l.tubes = off; off += align_up(sizeof(kern::Tube) * ntubes);
  l.blk = off; off += align_up(sizeof(int32_t) * l.nblocks);
  l.blkT = off; off += align_up(sizeof(int32_t) * l.nblocks_tmax);
  l.tube_n = off; off += align_up(sizeof(int64_t) * ntubes);
  l.ctr = off; off += align_up(sizeof(uint32_t));
  l.flag = off; off += align_up(sizeof(uint32_t) * ntubes);
  l.range = off; off += align_up(sizeof(int32_t) * ntubes * MAXL * NCLS * 2);
  l.tab = off; off += align_up(sizeof(double) * ntubes * MAXL * NCLS * 4);
  l.pop = off; off += 2 * align_up((size_t)L * Q * l.n * s_bytes);
  l.rec = off; off += align_up((size_t)rec_fields * l.n * r_bytes);
  l.G = off; off += align_up((size_t)3 * l.n * r_bytes);
  // staging: fields of init_fields / read_moments ((M+6) n doubles), or the
  // doubles of read_fields_f32 followed by its packed floats ((M+5) n each)
  l.staging = off; off += align_up((size_t)(2 * M + 8) * l.n * sizeof(double));
  l.partial = off; off += align_up((size_t)l.nblocks * (MAXM + 6) * sizeof(double));
  l.reduced = off; off += align_up((size_t)ntubes * (MAXM + 6) * sizeof(double));
  l.bad = off; off += align_up((size_t)l.nblocks * sizeof(int));
  l.chg = off; off += align_up((size_t)l.nblocks * sizeof(float));
  l.total = off;
  return l;
}

int validate_one(const mclbm_params* p, std::string& err)
{
  if (!p) { err = "params is NULL"; return MCLBM_EARG; }
  if (p->M < 2 || p->M > MAXM) { err = "M must be in 2..8"; return MCLBM_EARG; }
  if (p->M > 4) { err = "the kernels are compiled for M = 2, 3, 4"; return MCLBM_EUNSUPPORTED; }
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) { err = "grid sizes must be positive"; return MCLBM_EARG; }
  const int64_t n = (int64_t)p->nx * p->ny * p->nz;
  if (n >= ((int64_t)1 << 31)) { err = "nx*ny*nz must be below 2^31"; return MCLBM_EARG; }
  // the kernels address one lattice direction (or record field) of a tube with a
  // 32-bit byte offset: n times the widest element (FP64 storage and records: 8
  // bytes, otherwise 4) must stay below 2^32
  const int64_t widest = p->precision == MCLBM_FP64 ? 8 : 4;
  if (n * widest >= ((int64_t)1 << 32)) {
    err = "nx*ny*nz times the element size must be below 2^32 bytes";
    return MCLBM_EARG;
  }
  if (p->wall_x < 0 || p->wall_x > 3) { err = "wall_x must be 0, 1, 2 or 3"; return MCLBM_EARG; }
  auto inlet_ok = [&](const double* in) {
    double xs = 0.0;
    bool ok = in[p->M] > 0 && in[p->M + 1] > 0;
    for (int k = 0; k < p->M + 5; ++k) ok = ok && std::isfinite(in[k]);
    for (int a = 0; a < p->M; ++a) {
      ok = ok && in[a] >= 0;
      xs += in[a];
    }
    return ok && std::fabs(xs - 1.0) <= 1e-12;
  };
  if (p->wall_x >= 2) {
    if (!p->inlet || (p->wall_x == 3 && !p->inlet_right)) {
      err = "open x ends need the inlet fields, the opposed jets both inlets";
      return MCLBM_EARG;
    }
    if (!inlet_ok(p->inlet) || (p->wall_x == 3 && !inlet_ok(p->inlet_right))) {
      err = "inlet: mole fractions must be non-negative and sum to 1, p and T positive";
      return MCLBM_EARG;
    }
    if (p->precision != MCLBM_FP64 && p->precision != MCLBM_FP32) {
      err = "open x ends and the opposed jets are compiled for MCLBM_FP64 and MCLBM_FP32 only";
      return MCLBM_EUNSUPPORTED;
    }
  }
  if ((p->wall_x == 3) != (p->wall_y == 2)) {
    err = "the opposed jets (wall_x = 3) and the y outlets (wall_y = 2) go together";
    return MCLBM_EARG;
  }
  if (p->wall_x == 3) {
    if (!(p->nozzle_y0 >= 1 && p->nozzle_y0 < p->nozzle_y1 && p->nozzle_y1 <= p->ny - 1)) {
      err = "the nozzle rows must satisfy 1 <= nozzle_y0 < nozzle_y1 <= ny - 1";
      return MCLBM_EARG;
    }
    if (p->weak || p->cv_coef || p->transport_exp) {
      err = "the opposed jets are compiled for strong coupling with constant properties";
      return MCLBM_EUNSUPPORTED;
    }
  }
  if (p->wall_x && p->nx < 2) { err = "walls need nx >= 2"; return MCLBM_EARG; }
  if (p->precision < MCLBM_FP64 || p->precision > MCLBM_I16) { err = "unknown precision"; return MCLBM_EARG; }
  if (p->weak != 0 && p->weak != 1) { err = "weak must be 0 or 1"; return MCLBM_EARG; }
  if (p->slaved < 0 || p->slaved > p->M) { err = "slaved must be 0 (species M) or 1..M"; return MCLBM_EARG; }
  if (p->weak && p->slaved != 0 && p->slaved != p->M) {
    err = "weak coupling slaves no species: slaved must be 0";
    return MCLBM_EARG;
  }
  if (p->wall_y < 0 || p->wall_y > 2) { err = "wall_y must be 0, 1 or 2"; return MCLBM_EARG; }
  if (p->wall_y == 1) {
    if (p->ny < 2) { err = "free-slip y walls need ny >= 2"; return MCLBM_EARG; }
    if (p->wall_x == 2 || (p->precision != MCLBM_FP64 && p->precision != MCLBM_FP32)) {
      err = "free-slip y walls are compiled for periodic or walled x ends, MCLBM_FP64 and MCLBM_FP32 only";
      return MCLBM_EUNSUPPORTED;
    }
  }
  if (p->weak && p->precision != MCLBM_FP64 && p->precision != MCLBM_FP32 && p->precision != MCLBM_FP16 &&
      p->precision != MCLBM_I16) {
    err = "weak coupling is compiled for MCLBM_FP64, MCLBM_FP32, MCLBM_FP16 and MCLBM_I16 only";
    return MCLBM_EUNSUPPORTED;
  }
  if (p->transport_exp) {
    bool ok = p->transport_exp[2 * p->M + 1] > 0;
    for (int k = 0; k < 2 * p->M + 2; ++k) ok = ok && std::isfinite(p->transport_exp[k]);
    if (!ok) {
      err = "transport_exp: exponents must be finite and T_ref positive";
      return MCLBM_EARG;
    }
    if (p->precision != MCLBM_FP64 && p->precision != MCLBM_FP32) {
      err = "temperature-dependent transport is compiled for MCLBM_FP64 and MCLBM_FP32 only";
      return MCLBM_EUNSUPPORTED;
    }
  }
  if (p->cv_coef) {
    for (int a = 0; a < p->M; ++a)
      for (int k = 0; k < 4; ++k) {
        const double c = p->cv_coef[a * 4 + k];
        if (!(k == 0 ? c > 0 : c >= 0) || !std::isfinite(c)) {
          err = "cv_coef: c_a0 must be positive and c_ak (k >= 1) non-negative";
          return MCLBM_EARG;
        }
      }
    if (p->precision != MCLBM_FP64 && p->precision != MCLBM_FP32) {
      err = "temperature-dependent specific heats are compiled for MCLBM_FP64 and MCLBM_FP32 only";
      return MCLBM_EUNSUPPORTED;
    }
  }
  if (!p->molar_mass || !p->cv || !p->D || !p->mu || !p->lambda) { err = "species arrays must be given"; return MCLBM_EARG; }
  for (int a = 0; a < p->M; ++a) {
    if (!(p->molar_mass[a] > 0) || !(p->cv[a] > 0) || !(p->mu[a] > 0) || !(p->lambda[a] > 0)) {
      err = "molar masses, heat capacities, viscosities and conductivities must be positive";
      return MCLBM_EARG;
    }
    for (int b = 0; b < p->M; ++b) {
      const double d = p->D[a * p->M + b];
      if (!(d > 0) || d != p->D[b * p->M + a]) { err = "D must be symmetric and positive"; return MCLBM_EARG; }
    }
  }
  return MCLBM_OK;
}

// The caller's (0-based) index of the slaved species: slaved = 0 means species M.
int slaved_of(const mclbm_params* p) { return p->slaved == 0 ? p->M - 1 : p->slaved - 1; }

int validate(const mclbm_params* tp, int ntubes, std::string& err)
{
  if (!tp) { err = "params is NULL"; return MCLBM_EARG; }
  if (ntubes < 1) { err = "ntubes must be positive"; return MCLBM_EARG; }
  int64_t total = 0, blocks = 0;
  for (int t = 0; t < ntubes; ++t) {
    int rc = validate_one(&tp[t], err);
    if (rc != MCLBM_OK) {
      if (ntubes > 1) err = "tube " + std::to_string(t) + ": " + err;
      return rc;
    }
    if (tp[t].M != tp[0].M || tp[t].wall_x != tp[0].wall_x || tp[t].precision != tp[0].precision ||
        tp[t].weak != tp[0].weak || tp[t].wall_y != tp[0].wall_y ||
        slaved_of(&tp[t]) != slaved_of(&tp[0]) ||
        (tp[t].cv_coef == nullptr) != (tp[0].cv_coef == nullptr) ||
        (tp[t].transport_exp == nullptr) != (tp[0].transport_exp == nullptr)) {
      err = "all tubes of a batch must share M, wall_x, precision, weak, the slaved species and whether cv_coef "
            "and transport_exp are given";
      return MCLBM_EARG;
    }
    const int64_t n = (int64_t)tp[t].nx * tp[t].ny * tp[t].nz;
    total += n;
    blocks += (n + BLOCK - 1) / BLOCK;
  }
  if (blocks >= ((int64_t)1 << 31) / BLOCK) { err = "too many nodes in the batch"; return MCLBM_EARG; }
  (void)total;
  return MCLBM_OK;
}

int fail(mclbm_ctx* c, int code, const std::string& msg)
{
  if (c) c->err = msg; else g_last_error = msg;
  return code;
}

#define HIP_TRY(ctx, call)                                                                        \
  do {                                                                                            \
    hipError_t e_ = (call);                                                                       \
    if (e_ != hipSuccess) return fail((ctx), MCLBM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

double absent_tol_for(int precision);

// Launch over every block of every tube (linear numbering).
Launch launch_all(const mclbm_ctx* c)
{
  return Launch{c->dTubes, c->dBlkTube, c->ntubes, 0, c->lc.swizzle, 0};
}

// The step kernels' launches take the block shape of the launch choice.
int32_t shape_code(const mclbm_ctx* c)
{
  const int k = c->lc.shape;
  return k ? kern::SHAPE_SX[k] | kern::SHAPE_SY[k] << 4 : 0;
}

Launch step_launch_all(const mclbm_ctx* c)
{
  if (!c->lc.shape) return launch_all(c);
  return Launch{c->dTubes, c->dBlkTubeT, c->ntubes, 0, c->lc.swizzle, shape_code(c)};
}

unsigned step_grid_all(const mclbm_ctx* c) { return (unsigned)(c->lc.shape ? c->nblocks_t : c->nblocks); }

// Step launch over the blocks of tube t only.
Launch step_launch_one(const mclbm_ctx* c, int t)
{
  if (!c->lc.shape)
    return Launch{c->dTubes, c->dBlkTube, c->ntubes, c->hTubes[t].first_block, c->lc.swizzle, 0};
  return Launch{c->dTubes, c->dBlkTubeT, c->ntubes, c->hTubes[t].tfirst, c->lc.swizzle, shape_code(c)};
}

unsigned step_grid_one(const mclbm_ctx* c, int t)
{
  return (unsigned)(c->lc.shape ? c->hTubes[t].tnblocks : c->hTubes[t].nblocks);
}

// The equilibrium of the inlet fields in every stored lattice of a context's
// coupling and heat-capacity mode (one node, n = 1).
template <int M>
int inlet_node(int weak, int cvt, const Params<double>& P1, const double* in, double* dev)
{
  const double *X = in, *p = in + M, *T = in + M + 1, *u = in + M + 2;
  if (weak && cvt) return init_node<double, M, true, true>(P1, X, p, T, u, dev, 0);
  if (weak) return init_node<double, M, true, false>(P1, X, p, T, u, dev, 0);
  if (cvt) return init_node<double, M, false, true>(P1, X, p, T, u, dev, 0);
  return init_node<double, M>(P1, X, p, T, u, dev, 0);
}

int push_params(mclbm_ctx* c)
{
  HIP_TRY(c, hipStreamSynchronize(c->stream));   // previous uploads from the host blocks are done
  const double tol = absent_tol_for(c->precision);
  for (int t = 0; t < c->ntubes; ++t) {
    const TubeHost& th = c->tubes[t];
    // the kernels read the reference of a direction at its class's representative
    for (int l = 0; l < c->L; ++l)
      for (int i = 0; i < Q; ++i)
        if (!(th.tab.ref[l][i] == th.tab.ref[l][crep(i)]))
          return fail(c, MCLBM_ESTATE, "reference tables differ within a direction class");
    fill_params<double>(c->hPd[t], th.hs, th.nx, th.ny, th.nz, c->wall_x, c->L, th.tab, tol, c->dFlag + t, c->xperm,
                        th.noz0, th.noz1);
    fill_params<float>(c->hPf[t], th.hs, th.nx, th.ny, th.nz, c->wall_x, c->L, th.tab, tol, c->dFlag + t, c->xperm,
                       th.noz0, th.noz1);
    // the inlet equilibria of every stored lattice, as deviations from f_ref: the
    // initialisation of one node (n = 1, unit scale) at the inlet fields (open x
    // ends: one inlet; opposed jets: one per x face)
    const int sides = c->wall_x == 3 ? 2 : (c->wall_x == 2 ? 1 : 0);
    for (int side = 0; side < sides; ++side) {
      Params<double> P1 = c->hPd[t];
      P1.n = 1;
      for (int l = 0; l < MAXL; ++l) P1.scale[l] = 1.0;
      double dev[MAXL * Q] = {};
      const int M = c->M;
      const double* in = side ? th.inlet2 : th.inlet;
      int bad = 1;
      switch (M) {
        case 2: bad = inlet_node<2>(c->weak, c->cvt, P1, in, dev); break;
        case 3: bad = inlet_node<3>(c->weak, c->cvt, P1, in, dev); break;
        case 4: bad = inlet_node<4>(c->weak, c->cvt, P1, in, dev); break;
        default: break;
      }
      if (bad) return fail(c, MCLBM_ESTATE, "infeasible inlet state (R_a T + u^2 >= 1)");
      for (int l = 0; l < c->L; ++l)
        for (int i = 0; i < Q; ++i) {
          (side ? c->hPd[t].inl2 : c->hPd[t].inl)[l][i] = dev[l * Q + i];
          (side ? c->hPf[t].inl2 : c->hPf[t].inl)[l][i] = (float)dev[l * Q + i];
        }
    }
  }
  HIP_TRY(c, hipMemcpyAsync(c->dPd, c->hPd.data(), sizeof(Params<double>) * c->ntubes, hipMemcpyHostToDevice,
                            c->stream));
  if (!compute_is_fp64(c->precision))
    HIP_TRY(c, hipMemcpyAsync(c->dPr, c->hPf.data(), sizeof(Params<float>) * c->ntubes, hipMemcpyHostToDevice,
                              c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return MCLBM_OK;
}

// Block numbering of the tubes: blocks of the tubes follow each other in the
// launch order (given, or longest first); the memory layout does not change.
int push_block_map(mclbm_ctx* c)
{
  std::vector<int> order(c->ntubes);
  std::iota(order.begin(), order.end(), 0);
  if (c->lc.order == 1)
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return c->tubes[a].n > c->tubes[b].n; });
  int32_t blk = 0, blkT = 0;
  const int k = c->lc.shape;
  for (int t : order) {
    const TubeHost& th = c->tubes[t];
    kern::Tube& tb = c->hTubes[t];
    const int32_t nb = (int32_t)((th.n + BLOCK - 1) / BLOCK);
    tb.base = th.base;
    tb.first_block = blk;
    tb.nblocks = nb;
    tb.nx = th.nx;
    tb.ny = th.ny;
    tb.nz = th.nz;
    for (int32_t b = 0; b < nb; ++b) c->hBlkTube[blk + b] = t;
    blk += nb;
    tb.tiles_x = tb.tiles_y = tb.tfirst = tb.tnblocks = 0;
    if (k) {
      int64_t nt = 0;
      tile_counts(k, th.nx, th.ny, th.nz, tb.tiles_x, tb.tiles_y, nt);
      tb.tfirst = blkT;
      tb.tnblocks = (int32_t)nt;
      for (int32_t b = 0; b < (int32_t)nt; ++b) c->hBlkTubeT[blkT + b] = t;
      blkT += (int32_t)nt;
    }
  }
  c->nblocks_t = blkT;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->dTubes, c->hTubes.data(), sizeof(kern::Tube) * c->ntubes, hipMemcpyHostToDevice,
                            c->stream));
  HIP_TRY(c, hipMemcpyAsync(c->dBlkTube, c->hBlkTube.data(), sizeof(int32_t) * c->nblocks, hipMemcpyHostToDevice,
                            c->stream));
  if (blkT)
    HIP_TRY(c, hipMemcpyAsync(c->dBlkTubeT, c->hBlkTubeT.data(), sizeof(int32_t) * blkT, hipMemcpyHostToDevice,
                              c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return MCLBM_OK;
}

// Power-of-two scale that maps the reference populations of a lattice to
// magnitudes around 2^10 (16-bit storage only), so that scaling is exact.
double scale_for(int precision, const double* ref_l)
{
  if (precision != MCLBM_FP16 && precision != MCLBM_BF16) return 1.0;
  double mx = 0.0;
  for (int i = 0; i < Q; ++i) mx = std::max(mx, std::fabs(ref_l[i]));
  if (!(mx > 0.0)) return 1.0;
  return std::ldexp(1.0, (int)std::floor(std::log2(1024.0 / mx)));
}

// Round a scaled reference value to the nearest value the storage type holds,
// so that a population equal to zero (an absent species) is stored exactly.
double round_to_storage(int precision, double v)
{
  switch (precision) {
    case MCLBM_FP32:
    case MCLBM_FP32_FP32: return (double)(float)v;
    case MCLBM_FP16: return (double)(float)(_Float16)(float)v;
    case MCLBM_BF16: {
      float f = (float)v;
      uint32_t u;
      std::memcpy(&u, &f, 4);
      u += 0x7fffu + ((u >> 16) & 1u);      // round to nearest even on the upper 16 bits
      u &= 0xffff0000u;
      std::memcpy(&f, &u, 4);
      return (double)f;
    }
    default: return v;
  }
}

// Relative density below which a species counts as absent (eq transform12 then
// has a zero row for it, V_a = 0): the resolution of the stored populations.
// With FP64 and FP32 storage an absent species is stored exactly (the reference
// values are representable and the moments are summed in FP64), so the
// threshold only guards against round-off. With 16-bit storage, stochastic
// rounding leaves noise of about one unit in the last place on the populations
// of a nearly absent species; treating such a species as present would give it
// an arbitrarily large diffusion velocity, whose quadratic Stefan--Maxwell
// source makes the step unstable.
double absent_tol_for(int precision)
{
  switch (precision) {
    case MCLBM_FP16: case MCLBM_I16: return 1e-4;
    case MCLBM_BF16: return 1e-3;
    default: return 1e-12;
  }
}

// Reference tables of every tube from its mean state, rounded to storage.
// 16-bit fixed-point storage (MCLBM_I16). Each class k of directions (equal
// |c_x|, |c_y|, |c_z|) of each stored lattice l has a centre f_ref and a
// half-width h: a population f is stored as the integer nearest (stochastically)
// to (f - f_ref) 32767 / h. The first tables of mclbm_init_fields centre every
// class on the mean state's equilibrium at rest with a half-width of
// FIX_FIRST_RANGE times that value; k_range16 then measures what the state takes
// and fit_class sets the half-width to FIX_MARGIN times the measured one (at
// least the centre's magnitude). During
// the steps a value past 3/4 of its range (the margin partly used) makes the
// host fit the tables again to the state and re-encode it (rerange).
constexpr double FIX_FIRST_RANGE = 64.0;
int check_launch(mclbm_ctx* c, const char* what);
constexpr double FIX_MARGIN = 2.0;
constexpr int FIX_CHECK_STEPS = 8;    // steps between reads of the range flag
constexpr double FIX_REL = 1.0;       // least half-width, relative to the class's centre
// Steps the initialisation takes (and discards) with its first, wide tables to see
// the range of the transient that follows the initial state. The classes of small
// weight (edges and corners at a low lattice temperature R_a T) hold equilibrium
// values far below the non-equilibrium parts that a sharp front adds to them (a
// diffusion or heat flux enters at a lower power of the weight): in the ternary
// tube's second step a species' corner populations leave a range fitted to the
// initial equilibria fifteen times over, and the energy lattice's x faces four
// times; the excursion is largest in the first steps and decays after.
constexpr int FIX_PROBE_STEPS = 4;
int eager_step(mclbm_ctx* c);

// Tables of class k of lattice l: centre and decoding factor rounded to FP32 (the
// FP32 and FP64 kernels then decode a value alike), encoding factor its inverse.
void set_class(RefTables& tb, int l, int k, double centre, double half)
{
  const double ce = (double)(float)centre;
  const double inv = (double)(float)(half / 32767.0);
  for (int i = 0; i < Q; ++i)
    if (ccls(i) == k) tb.ref[l][i] = ce;
  tb.inv_qs[l][k] = inv;
  tb.qs[l][k] = (double)(float)(1.0 / inv);
}

// Floor of a class's half-width: a millionth of the lattice's largest reference
// magnitude (a class that holds one value everywhere still gets a range).
double class_floor(const RefTables& tb, int l)
{
  double mx = 0.0;
  for (int i = 0; i < Q; ++i) mx = std::max(mx, std::fabs(tb.ref[l][i]));
  return mx > 0.0 ? 1e-6 * mx : 1e-20;
}

// Fit class k of lattice l to the stored integers lo..hi (current tables): centre
// the middle of the values, half-width FIX_MARGIN times their half-spread plus
// one storage unit, and at least FIX_REL times the centre's magnitude (a
// population may double). The floor matters where the values of a class barely
// differ over the grid (the moving populations of a gas at rest at uniform
// pressure): a flow that starts later moves such a population by about
// (c_i . u / theta) of itself. In the ternary tube the diffusion-driven flow
// moves the momentum lattice's x faces by up to 56% of themselves within 30
// steps (up to 30% in one step) and the energy lattice's rest population by 1.4
// times its initial spread; a floor of an eighth of the centre, or none, lets
// them reach the end of the range between two checks.
void fit_class(RefTables& tb, int l, int k, int32_t lo, int32_t hi)
{
  int i0 = 0;
  while (ccls(i0) != k) ++i0;
  const double c0 = tb.ref[l][i0], inv0 = tb.inv_qs[l][k];
  const double flo = c0 + lo * inv0, fhi = c0 + hi * inv0;
  const double centre = 0.5 * (flo + fhi);
  const double half = FIX_MARGIN * (0.5 * (fhi - flo) + inv0);
  set_class(tb, l, k, centre, std::max({half, FIX_REL * std::fabs(centre), class_floor(tb, l)}));
}

// Reference tables of every tube from its mean state, rounded to storage (for
// fixed point: the first, wide tables).
int upload_params(mclbm_ctx* c, const std::vector<RefState>& rs)
{
  for (int t = 0; t < c->ntubes; ++t) {
    TubeHost& th = c->tubes[t];
    RefTables& tb = th.tab;
    reference_tables(th.hs, c->L - 2, rs[t], tb);
    for (int l = 0; l < MAXL; ++l) {
      tb.scale[l] = 1.0;
      for (int k = 0; k < NCLS; ++k) tb.qs[l][k] = tb.inv_qs[l][k] = 0.0;
    }
    for (int l = 0; l < c->L; ++l) {
      tb.scale[l] = scale_for(c->precision, tb.ref[l]);
      // FP32 storage of FP64 arithmetic keeps the species populations themselves
      // (reference zero): the stochastic rounding of a store is then relative to
      // the population, so a nearly absent species is not buried in rounding
      // noise of the size of the mean state's population (which would give it a
      // diffusion velocity from noise)
      const bool absolute = c->precision == MCLBM_FP32 && l < c->L - 2;
      for (int i = 0; i < Q; ++i) {
        if (absolute) tb.ref[l][i] = 0.0;
        tb.ref[l][i] = round_to_storage(c->precision, tb.ref[l][i] * tb.scale[l]) / tb.scale[l];
      }
      if (c->precision == MCLBM_I16) {
        const double fl = class_floor(tb, l);
        for (int k = 0; k < NCLS; ++k) {
          int i0 = 0;
          while (ccls(i0) != k) ++i0;
          const double r = tb.ref[l][i0];
          set_class(tb, l, k, r, FIX_FIRST_RANGE * std::max(std::fabs(r), fl));
        }
      }
    }
    reference_moments(tb, c->L);
  }
  return push_params(c);
}

// Fixed point: the smallest and largest stored integer of every tube, lattice and
// class of the current state, mm[((t MAXL + l) NCLS + k) 2 + {0, 1}].
int measure_ranges(mclbm_ctx* c, std::vector<int32_t>& mm)
{
  const size_t cnt = (size_t)c->ntubes * MAXL * NCLS * 2;
  mm.assign(cnt, 0);
  for (size_t j = 0; j < cnt; j += 2) {
    mm[j] = 32767;
    mm[j + 1] = -32767;
  }
  HIP_TRY(c, hipMemcpyAsync(c->dRange, mm.data(), sizeof(int32_t) * cnt, hipMemcpyHostToDevice, c->stream));
  c->ops.range16(c->dPd, launch_all(c), c->pop[c->cur], c->dRange, (unsigned)c->nblocks, c->stream);
  int rc = check_launch(c, "k_range16");
  if (rc) return rc;
  HIP_TRY(c, hipMemcpyAsync(mm.data(), c->dRange, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return MCLBM_OK;
}

int clear_range_flags(mclbm_ctx* c)
{
  HIP_TRY(c, hipMemsetAsync(c->dFlag, 0, sizeof(uint32_t) * c->ntubes, c->stream));
  return MCLBM_OK;
}

// Fixed point: fit every class of the tubes whose flag asks for it to the current
// state and re-encode their state with the new tables (k_rebase16; the other
// tubes keep theirs: a zero old decoding factor marks them), then upload the
// tables and clear the flags.
int rerange(mclbm_ctx* c, const std::vector<uint32_t>& flags)
{
  std::vector<int32_t> mm;
  int rc = measure_ranges(c, mm);
  if (rc) return rc;
  std::vector<double> tab((size_t)c->ntubes * MAXL * NCLS * 4, 0.0);
  for (int t = 0; t < c->ntubes; ++t) {
    if (!(flags[t] & 1u)) continue;
    c->reranges += 1;
    RefTables& tb = c->tubes[t].tab;
    for (int l = 0; l < c->L; ++l)
      for (int k = 0; k < NCLS; ++k) {
        const size_t j = ((size_t)t * MAXL + l) * NCLS + k;
        const int32_t lo = mm[2 * j], hi = mm[2 * j + 1];
        if (lo <= -32767 || hi >= 32767)
          return fail(c, MCLBM_ESTATE, "fixed-point storage: a stored value reached the end of its range");
        int i0 = 0;
        while (ccls(i0) != k) ++i0;
        tab[4 * j + 0] = tb.ref[l][i0];
        tab[4 * j + 1] = tb.inv_qs[l][k];
        fit_class(tb, l, k, lo, hi);
        tab[4 * j + 2] = tb.ref[l][i0];
        tab[4 * j + 3] = tb.qs[l][k];
      }
    reference_moments(tb, c->L);
  }
  HIP_TRY(c, hipMemcpyAsync(c->dTab, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice, c->stream));
  c->ops.rebase16(c->dPd, launch_all(c), c->pop[c->cur], c->dTab, (uint32_t)c->steps * 0x9E3779B1u + 0x5bd1e995u,
                  (unsigned)c->nblocks, c->stream);
  rc = check_launch(c, "k_rebase16");
  if (rc) return rc;
  rc = push_params(c);   // synchronises the stream first: the tables are read by k_rebase16
  if (rc) return rc;
  return clear_range_flags(c);
}

int record_event(mclbm_ctx* c, int& idx)
{
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t e;
    HIP_TRY(c, hipEventCreate(&e));
    c->ev_pool.push_back(e);
  }
  idx = (int)c->ev_used++;
  HIP_TRY(c, hipEventRecord(c->ev_pool[idx], c->stream));
  return MCLBM_OK;
}

int harvest_timing(mclbm_ctx* c)
{
  if (c->ev_used == 0) return MCLBM_OK;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < 3; ++k) {
    for (auto& pr : c->ev_pairs[k]) {
      float ms = 0.f;
      HIP_TRY(c, hipEventElapsedTime(&ms, c->ev_pool[pr.first], c->ev_pool[pr.second]));
      c->acc_ms[k] += ms;
      c->acc_launches[k] += 1;
    }
    c->ev_pairs[k].clear();
  }
  c->ev_used = 0;
  return MCLBM_OK;
}

int check_launch(mclbm_ctx* c, const char* what)
{
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, MCLBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return MCLBM_OK;
}

void drop_graph(mclbm_ctx* c)
{
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  c->gexec = nullptr;
  c->gsteps = 0;
}

// Collision and streaming from buffer `from`: one launch, or the species
// lattices and the momentum and energy lattices in two (they write disjoint
// lattices of the other buffer).
void collide(mclbm_ctx* c, const Launch& ln, int from, StepNo sn, unsigned grid, hipStream_t st)
{
  if (c->lc.split) {
    c->ops.collide_split[0](c->dPr, ln, c->pop[from], c->pop[1 - from], c->rec, c->G, sn, grid, st);
    c->ops.collide_split[1](c->dPr, ln, c->pop[from], c->pop[1 - from], c->rec, c->G, sn, grid, st);
  } else {
    c->ops.collide[c->lc.variant](c->dPr, ln, c->pop[from], c->pop[1 - from], c->rec, c->G, sn, grid, st);
  }
  if (c->ops.open_fix) c->ops.open_fix(c->dPr, ln, c->pop[1 - from], sn, grid, st);
}

// Whether steps take the two-read path (compiled for constant properties).
bool two_read(const mclbm_ctx* c) { return !c->lc.three_pass && c->ops.state_species[0] != nullptr; }

// First pass of a step from buffer `from`: moments -> record (three-pass), or
// moments -> record plus the species collisions into the other buffer (two-read).
void first_pass(mclbm_ctx* c, const Launch& ln, int from, StepNo sn, unsigned grid, hipStream_t st)
{
  const int v = c->lc.variant;
  if (two_read(c)) c->ops.state_species[v](c->dPr, ln, c->pop[from], c->pop[1 - from], c->rec, sn, grid, st);
  else c->ops.moments[v](c->dPd, ln, c->pop[from], c->rec, grid, st);
}

// Last pass: the collision of every lattice (three-pass), or of the momentum and
// energy lattices (two-read), then the open-end fix-up.
void last_pass(mclbm_ctx* c, const Launch& ln, int from, StepNo sn, unsigned grid, hipStream_t st)
{
  if (two_read(c)) {
    c->ops.collide_fg[c->lc.variant](c->dPr, ln, c->pop[from], c->pop[1 - from], c->rec, c->G, sn, grid, st);
    if (c->ops.open_fix) c->ops.open_fix(c->dPr, ln, c->pop[1 - from], sn, grid, st);
  } else {
    collide(c, ln, from, sn, grid, st);
  }
}

// The launches of one step from buffer `from` on stream st.
void enqueue_step(mclbm_ctx* c, int from, StepNo sn, hipStream_t st)
{
  const int rf = c->ops.rec_fields;
  auto one = [&](const Launch& ln, unsigned grid) {
    first_pass(c, ln, from, sn, grid, st);
    c->ops.gfield(c->dPd, ln, c->rec, c->G, rf, grid, st);
    last_pass(c, ln, from, sn, grid, st);
  };
  if (!c->lc.sequential) {
    one(step_launch_all(c), step_grid_all(c));
    return;
  }
  for (int t = 0; t < c->ntubes; ++t) one(step_launch_one(c, t), step_grid_one(c, t));
}

// One eager step, with per-kernel events when timing is enabled (batched only).
int eager_step(mclbm_ctx* c)
{
  const StepNo sn{nullptr, (uint32_t)c->steps};
  int rc = 0;
  if (c->timing && !c->lc.sequential) {
    const Launch ln = step_launch_all(c);
    const unsigned grid = step_grid_all(c);
    int e0 = 0, e1 = 0, e2 = 0, e3 = 0;
    if ((rc = record_event(c, e0))) return rc;
    first_pass(c, ln, c->cur, sn, grid, c->stream);
    if ((rc = record_event(c, e1))) return rc;
    c->ops.gfield(c->dPd, ln, c->rec, c->G, c->ops.rec_fields, grid, c->stream);
    if ((rc = record_event(c, e2))) return rc;
    last_pass(c, ln, c->cur, sn, grid, c->stream);
    if ((rc = record_event(c, e3))) return rc;
    c->ev_pairs[0].push_back({e0, e1});
    c->ev_pairs[1].push_back({e1, e2});
    c->ev_pairs[2].push_back({e2, e3});
  } else {
    enqueue_step(c, c->cur, sn, c->stream);
  }
  rc = check_launch(c, "mclbm_step");
  if (rc) return rc;
  c->cur = 1 - c->cur;
  c->steps += 1;
  if (c->timing && c->ev_used > 3000 && (rc = harvest_timing(c))) return rc;
  return MCLBM_OK;
}

// Capture K steps starting from buffer 0 into a graph on a private stream
// (kernel nodes only; the step counter is advanced by a kernel, not a memset).
int build_graph(mclbm_ctx* c, int K)
{
  drop_graph(c);
  if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  for (int j = 0; j < K; ++j) enqueue_step(c, j & 1, StepNo{c->dStepCtr, (uint32_t)j}, c->cap_stream);
  hipLaunchKernelGGL(k_counter_add, dim3(1), dim3(64), 0, c->cap_stream, c->dStepCtr, (uint32_t)K);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
  if (e != hipSuccess) return fail(c, MCLBM_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    c->gexec = nullptr;
    return fail(c, MCLBM_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  c->gsteps = K;
  return MCLBM_OK;
}

int graph_steps(mclbm_ctx* c, int64_t& nsteps)
{
  const int K = c->lc.graph_steps;
  if (nsteps > 0 && c->cur == 1) {             // replays start from buffer 0
    int rc = eager_step(c);
    if (rc) return rc;
    --nsteps;
  }
  const int64_t chunks = nsteps / K;
  if (chunks == 0) return MCLBM_OK;
  if (c->gsteps != K) {
    int rc = build_graph(c, K);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_counter_set, dim3(1), dim3(64), 0, c->stream, c->dStepCtr, (uint32_t)c->steps);
  int rc = check_launch(c, "k_counter_set");
  if (rc) return rc;
  for (int64_t k = 0; k < chunks; ++k) {
    HIP_TRY(c, hipGraphLaunch(c->gexec, c->stream));
    c->steps += K;
  }
  nsteps -= chunks * K;
  return MCLBM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" size_t mclbm_batch_workspace_bytes(const mclbm_params* tubes, int32_t ntubes)
{
  std::string err;
  if (validate(tubes, ntubes, err) != MCLBM_OK) {
    g_last_error = err;
    return 0;
  }
  return layout_for(tubes, ntubes).total;
}

extern "C" size_t mclbm_workspace_bytes(const mclbm_params* p) { return mclbm_batch_workspace_bytes(p, 1); }

extern "C" int mclbm_batch_create(const mclbm_params* tp, int32_t ntubes, void* dev_workspace, size_t bytes,
                                  void* hip_stream, mclbm_ctx** out)
{
  if (!out) return fail(nullptr, MCLBM_EARG, "out is NULL");
  *out = nullptr;
  std::string err;
  int rc = validate(tp, ntubes, err);
  if (rc != MCLBM_OK) return fail(nullptr, rc, err);
  const Layout lay = layout_for(tp, ntubes);
  if (!dev_workspace) return fail(nullptr, MCLBM_EARG, "workspace is NULL");
  if (((uintptr_t)dev_workspace) % ALIGN) return fail(nullptr, MCLBM_EARG, "workspace must be 256-byte aligned");
  if (bytes < lay.total) return fail(nullptr, MCLBM_EARG, "workspace too small");
  mclbm_ctx* c = new (std::nothrow) mclbm_ctx();
  if (!c) return fail(nullptr, MCLBM_EARG, "out of host memory");
  c->M = tp[0].M;
  c->wall_x = tp[0].wall_x;
  c->precision = tp[0].precision;
  c->weak = tp[0].weak;
  c->cvt = tp[0].cv_coef != nullptr || tp[0].transport_exp != nullptr;
  c->wall_y = tp[0].wall_y;
  c->L = (c->weak ? c->M : c->M - 1) + 2;
  if (c->cvt) {
    // the three-pass step (temperature-dependent properties): the fused collision
    // spills at two waves per SIMD (binary shear layer 256^3, FP32: collide 4.06
    // ms); the split collision, two launches with fewer registers each, does not.
    // With four or more stored lattices (weak coupling) the higher-occupancy
    // moments kernel is the faster choice too (5.74 -> 5.4 ms per step)
    c->lc.split = 1;
    if (c->weak) c->lc.variant = 1;
  }
  c->ntubes = ntubes;
  c->n = lay.n;
  c->nblocks = lay.nblocks;
  c->tubes.resize(ntubes);
  {
    const int sl = slaved_of(&tp[0]);
    int k = 0;
    for (int a = 0; a < c->M; ++a)
      if (a != sl) c->xperm[k++] = a;
    c->xperm[c->M - 1] = sl;
    for (int a = 0; a < c->M; ++a) c->xperm_identity = c->xperm_identity && c->xperm[a] == a;
  }
  int64_t base = 0;
  for (int t = 0; t < ntubes; ++t) {
    const mclbm_params* p = &tp[t];
    TubeHost& th = c->tubes[t];
    th.nx = p->nx; th.ny = p->ny; th.nz = p->nz;
    th.n = (int64_t)p->nx * p->ny * p->nz;
    th.base = base;
    base += th.n;
    th.hs.M = p->M;
    // species in the library's order: the caller's, with the slaved species moved last
    const int* xp = c->xperm;
    for (int a = 0; a < p->M; ++a) {
      const int ua = xp[a];
      th.hs.m[a] = p->molar_mass[ua];
      th.hs.cv[a] = p->cv[ua];
      th.hs.mu[a] = p->mu[ua];
      th.hs.lam[a] = p->lambda[ua];
      for (int b = 0; b < p->M; ++b) th.hs.D[a][b] = p->D[ua * p->M + xp[b]];
      for (int k = 0; k < 4; ++k) th.hs.cvc[a][k] = p->cv_coef ? p->cv_coef[ua * 4 + k] : (k == 0 ? p->cv[ua] : 0.0);
    }
    th.hs.cvt = p->cv_coef != nullptr;
    for (int a = 0; a < p->M; ++a) {
      th.hs.s_mu[a] = p->transport_exp ? p->transport_exp[xp[a]] : 0.0;
      th.hs.s_lam[a] = p->transport_exp ? p->transport_exp[p->M + xp[a]] : 0.0;
    }
    th.hs.s_D = p->transport_exp ? p->transport_exp[2 * p->M] : 0.0;
    th.hs.T_ref = p->transport_exp ? p->transport_exp[2 * p->M + 1] : 1.0;
    th.hs.trn = p->transport_exp != nullptr;
    if (p->wall_x >= 2)
      for (int k = 0; k < p->M + 5; ++k) th.inlet[k] = p->inlet[k];
    if (p->wall_x == 3) {
      for (int k = 0; k < p->M + 5; ++k) th.inlet2[k] = p->inlet_right[k];
      th.noz0 = p->nozzle_y0;
      th.noz1 = p->nozzle_y1;
    }
  }
  if (!pick_ops(c->precision, c->M, c->wall_x | (c->wall_y << 2), c->weak, c->cvt, c->ops)) {
    delete c;
    return fail(nullptr, MCLBM_EUNSUPPORTED, "no kernels compiled for this configuration");
  }
  c->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(nullptr, MCLBM_EDEVICE, "hipGetDevice failed");
  }
  char* ws = (char*)dev_workspace;
  c->ws = ws;
  c->ws_bytes = bytes;
  c->dPd = ws + lay.pd;
  c->dPr = compute_is_fp64(c->precision) ? c->dPd : (void*)(ws + lay.pr);
  c->dTubes = (kern::Tube*)(ws + lay.tubes);
  c->dBlkTube = (int32_t*)(ws + lay.blk);
  c->dBlkTubeT = (int32_t*)(ws + lay.blkT);
  c->dTubeN = (int64_t*)(ws + lay.tube_n);
  c->dStepCtr = (uint32_t*)(ws + lay.ctr);
  c->dFlag = (uint32_t*)(ws + lay.flag);
  c->dRange = (int32_t*)(ws + lay.range);
  c->dTab = (double*)(ws + lay.tab);
  const size_t popb = align_up((size_t)c->L * Q * c->n * c->ops.s_bytes);
  c->pop[0] = ws + lay.pop;
  c->pop[1] = ws + lay.pop + popb;
  c->rec = ws + lay.rec;
  c->G = ws + lay.G;
  c->staging = (double*)(ws + lay.staging);
  c->partial = (double*)(ws + lay.partial);
  c->reduced = (double*)(ws + lay.reduced);
  c->bad = (int*)(ws + lay.bad);
  c->chg = (float*)(ws + lay.chg);
  c->hPd.resize(ntubes);
  c->hPf.resize(ntubes);
  c->hTubes.resize(ntubes);
  c->hBlkTube.resize(c->nblocks);
  c->hBlkTubeT.resize(lay.nblocks_tmax);
  c->hTubeN.resize(ntubes);
  for (int t = 0; t < ntubes; ++t) c->hTubeN[t] = c->tubes[t].n;
  rc = push_block_map(c);
  if (rc == MCLBM_OK) {
    hipError_t e = hipMemcpyAsync(c->dTubeN, c->hTubeN.data(), sizeof(int64_t) * ntubes, hipMemcpyHostToDevice,
                                  c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) rc = fail(c, MCLBM_EDEVICE, hipGetErrorString(e));
  }
  if (rc != MCLBM_OK) {
    g_last_error = c->err;
    delete c;
    return rc;
  }
  *out = c;
  return MCLBM_OK;
}

extern "C" int mclbm_create(const mclbm_params* p, void* dev_workspace, size_t bytes, void* hip_stream,
                            mclbm_ctx** out)
{
  return mclbm_batch_create(p, 1, dev_workspace, bytes, hip_stream, out);
}

// ---------------------------------------------------------------------------
// Static workspace: mclbm_create_static. For callers that cannot allocate device
// memory, a context whose workspace is an array in the library's code object,
// one copy per device, of MCLBM_STATIC_WORKSPACE_BYTES. Its device address is
// looked up once per device (hipGetSymbolAddress) with that device current; the
// array's name is never used as a device address in host code. One context per
// device may hold the array at a time.
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[MCLBM_STATIC_WORKSPACE_BYTES];

namespace {
constexpr int STATIC_MAX_DEVICES = 64;
std::mutex g_static_mu;
void* g_static_ptr[STATIC_MAX_DEVICES] = {};
const mclbm_ctx* g_static_owner[STATIC_MAX_DEVICES] = {};

// Release the device's static workspace if c holds it (called by mclbm_destroy).
void release_static(const mclbm_ctx* c)
{
  std::lock_guard<std::mutex> lock(g_static_mu);
  for (int d = 0; d < STATIC_MAX_DEVICES; ++d)
    if (g_static_owner[d] == c) g_static_owner[d] = nullptr;
}
}  // namespace

extern "C" int mclbm_create_static(const mclbm_params* p, void* hip_stream, mclbm_ctx** out)
{
  if (!out) return fail(nullptr, MCLBM_EARG, "out is NULL");
  *out = nullptr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(nullptr, MCLBM_EDEVICE, "hipGetDevice failed");
  if (dev < 0 || dev >= STATIC_MAX_DEVICES) return fail(nullptr, MCLBM_EARG, "device index beyond the static table");
  std::string err;
  const int vrc = validate(p, 1, err);
  if (vrc != MCLBM_OK) return fail(nullptr, vrc, err);
  const size_t need = layout_for(p, 1).total;
  if (need > (size_t)MCLBM_STATIC_WORKSPACE_BYTES)
    return fail(nullptr, MCLBM_EARG,
                "the context needs " + std::to_string(need) + " workspace bytes; the static workspace holds " +
                    std::to_string((size_t)MCLBM_STATIC_WORKSPACE_BYTES) + " (use mclbm_create)");
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(nullptr, MCLBM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_static_ptr[dev] = ptr;
  }
  if (g_static_owner[dev])
    return fail(nullptr, MCLBM_EARG, "the static workspace of this device is held by another context");
  const int rc = mclbm_batch_create(p, 1, g_static_ptr[dev], (size_t)MCLBM_STATIC_WORKSPACE_BYTES, hip_stream, out);
  if (rc == MCLBM_OK) g_static_owner[dev] = *out;
  return rc;
}

extern "C" void mclbm_destroy(mclbm_ctx* c)
{
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  release_static(c);
  drop_graph(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  delete c;
}

extern "C" const char* mclbm_last_error(const mclbm_ctx* c)
{
  return c ? c->err.c_str() : g_last_error.c_str();
}

extern "C" int32_t mclbm_tube_count(const mclbm_ctx* c) { return c ? c->ntubes : -1; }

extern "C" int64_t mclbm_node_count(const mclbm_ctx* c) { return c ? c->n : -1; }

namespace {

// Reduce NV values per tube from the per-block partials to host out[ntubes][nv].
int reduce_to_host(mclbm_ctx* c, int nv, double* out)
{
  hipLaunchKernelGGL(k_reduce_tubes, dim3(c->ntubes), dim3(RED_BLOCK), 0, c->stream, c->partial, c->dTubes, nv,
                     c->reduced);
  int rc = check_launch(c, "k_reduce_tubes");
  if (rc) return rc;
  HIP_TRY(c, hipMemcpyAsync(out, c->reduced, sizeof(double) * nv * c->ntubes, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return MCLBM_OK;
}

}  // namespace

extern "C" int mclbm_init_fields(mclbm_ctx* c, const double* X, const double* p, const double* T, const double* u,
                                 int on_device)
{
  if (!c) return MCLBM_EARG;
  if (!X || !p || !T || !u) return fail(c, MCLBM_EARG, "field pointers must be given");
  const int M = c->M;
  const int64_t N = c->n;
  const double *dX = X, *dp = p, *dT = T, *du = u;
  std::vector<RefState> rs(c->ntubes);
  if (!on_device) {
    // host fields: validate, compute each tube's reference state here, stage to the device
    for (int t = 0; t < c->ntubes; ++t) {
      const TubeHost& th = c->tubes[t];
      const int64_t n = th.n;
      const double* Xt = X + (size_t)M * th.base;
      double sum[MAXM + 2] = {};
      for (int64_t i = 0; i < n; ++i) {
        double xs = 0.0;
        for (int a = 0; a < M; ++a) {
          const double v = Xt[(size_t)a * n + i];
          if (!(v >= 0.0)) return fail(c, MCLBM_EARG, "mole fractions must be non-negative");
          xs += v;
          sum[a] += v;
        }
        if (std::fabs(xs - 1.0) > 1e-9) return fail(c, MCLBM_EARG, "mole fractions must sum to 1");
        sum[M] += p[th.base + i];
        sum[M + 1] += T[th.base + i];
      }
      for (int a = 0; a < M; ++a) rs[t].X[a] = sum[c->xperm[a]] / n;
      rs[t].p = sum[M] / n;
      rs[t].T = sum[M + 1] / n;
    }
    double* st = c->staging;
    HIP_TRY(c, hipMemcpyAsync(st, X, sizeof(double) * M * N, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(st + (size_t)M * N, p, sizeof(double) * N, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(st + (size_t)(M + 1) * N, T, sizeof(double) * N, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(st + (size_t)(M + 2) * N, u, sizeof(double) * 3 * N, hipMemcpyHostToDevice, c->stream));
    dX = st;
    dp = st + (size_t)M * N;
    dT = st + (size_t)(M + 1) * N;
    du = st + (size_t)(M + 2) * N;
  } else {
    c->ops.field_sums(c->dTubeN, launch_all(c), dX, dp, dT, c->partial, (unsigned)c->nblocks, c->stream);
    int rc = check_launch(c, "k_field_sums");
    if (rc) return rc;
    std::vector<double> sum((size_t)c->ntubes * (M + 2));
    rc = reduce_to_host(c, M + 2, sum.data());
    if (rc) return rc;
    for (int t = 0; t < c->ntubes; ++t) {
      const double n = (double)c->tubes[t].n;
      const double* s = &sum[(size_t)t * (M + 2)];
      double xs = 0.0;
      for (int a = 0; a < M; ++a) {
        rs[t].X[a] = s[c->xperm[a]] / n;
        xs += rs[t].X[a];
      }
      rs[t].p = s[M] / n;
      rs[t].T = s[M + 1] / n;
      if (!(std::fabs(xs - 1.0) < 1e-6) || !(rs[t].p > 0) || !(rs[t].T > 0))
        return fail(c, MCLBM_EARG, "fields are not a valid state (mean mole fractions, p, T)");
    }
  }
  // the tube sizes of k_init come from the parameter blocks
  int rc = upload_params(c, rs);
  if (rc) return rc;
  c->cur = 0;
  // fixed point: initialise with the first (wide) tables, measure the range the
  // state and the FIX_PROBE_STEPS steps after it take, fit the tables to it and
  // initialise again; a class found at the end of its range is widened and
  // measured again. Each tube goes through these passes on its own (a tube's
  // tables do not depend on the other tubes).
  std::vector<char> fitted(c->ntubes, 0), done(c->ntubes, 0);
  for (int pass = 0;; ++pass) {
    c->cur = 0;
    c->steps = 0;
    c->ops.init(c->dPd, launch_all(c), dX, dp, dT, du, c->pop[0], c->bad, (unsigned)c->nblocks, c->stream);
    rc = check_launch(c, "k_init");
    if (rc) return rc;
    std::vector<int> bad(c->nblocks);
    HIP_TRY(c, hipMemcpyAsync(bad.data(), c->bad, sizeof(int) * c->nblocks, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int64_t b = 0; b < c->nblocks; ++b)
      if (bad[b]) return fail(c, MCLBM_ESTATE, "infeasible initial state: need T > 0, p > 0, R_a T + u^2 < 1");
    if (c->precision != MCLBM_I16) break;
    if (pass >= 8) return fail(c, MCLBM_ESTATE, "fixed-point storage: no range found that holds the initial state");
    std::vector<int32_t> m0, mu;
    if ((rc = measure_ranges(c, m0))) return rc;
    mu = m0;
    bool probe = false;
    for (int t = 0; t < c->ntubes; ++t) probe = probe || !fitted[t];
    if (probe) {                          // the transient, with the wide tables
      const bool timing = c->timing;
      c->timing = false;
      for (int k = 0; k < FIX_PROBE_STEPS && !rc; ++k) {
        std::vector<int32_t> mk;
        if (!(rc = eager_step(c)) && !(rc = measure_ranges(c, mk)))
          for (size_t j = 0; j < mu.size(); j += 2) {
            mu[j] = std::min(mu[j], mk[j]);
            mu[j + 1] = std::max(mu[j + 1], mk[j + 1]);
          }
      }
      c->timing = timing;
      if (rc) return rc;
    }
    bool all_done = true;
    for (int t = 0; t < c->ntubes; ++t) {
      if (done[t]) continue;
      RefTables& tb = c->tubes[t].tab;
      const std::vector<int32_t>& mm = fitted[t] ? m0 : mu;
      bool clamped = false;
      for (int l = 0; l < c->L; ++l)
        for (int k = 0; k < NCLS; ++k) {
          const size_t j = ((size_t)t * MAXL + l) * NCLS + k;
          if (mm[2 * j] > -32767 && mm[2 * j + 1] < 32767) continue;
          int i0 = 0;
          while (ccls(i0) != k) ++i0;
          set_class(tb, l, k, tb.ref[l][i0], FIX_FIRST_RANGE * 32767.0 * tb.inv_qs[l][k]);
          clamped = true;
        }
      if (!clamped && fitted[t]) {
        done[t] = 1;
        continue;
      }
      all_done = false;
      fitted[t] = !clamped;
      if (fitted[t])
        for (int l = 0; l < c->L; ++l)
          for (int k = 0; k < NCLS; ++k) {
            const size_t j = ((size_t)t * MAXL + l) * NCLS + k;
            fit_class(tb, l, k, mu[2 * j], mu[2 * j + 1]);
          }
      reference_moments(tb, c->L);
    }
    if (all_done) break;
    if ((rc = push_params(c))) return rc;
  }
  if (c->precision == MCLBM_I16 && (rc = clear_range_flags(c))) return rc;
  c->reranges = 0;
  c->steps = 0;
  c->initialised = true;
  return MCLBM_OK;
}

namespace {
// nsteps steps: graph replays where chosen, the rest eager.
int plain_steps(mclbm_ctx* c, int64_t nsteps)
{
  if (c->lc.graph_steps > 0 && !c->timing) {
    int rc = graph_steps(c, nsteps);
    if (rc) return rc;
  }
  for (int64_t t = 0; t < nsteps; ++t) {
    int rc = eager_step(c);
    if (rc) return rc;
  }
  return MCLBM_OK;
}

// Fixed point: the step counts after which the host reads the range flags, the
// powers of two below FIX_CHECK_STEPS (the transient of a sharp initial state)
// and the multiples of FIX_CHECK_STEPS. They depend on the step count only, not
// on how the steps are split into calls or launched (a checkpoint keeps the
// flags), so every split and launch choice gives the same trajectory.
int64_t next_check(int64_t steps)
{
  if (steps < FIX_CHECK_STEPS) {
    int64_t p = 1;
    while (p <= steps) p *= 2;
    return p;
  }
  return (steps / FIX_CHECK_STEPS + 1) * FIX_CHECK_STEPS;
}

// Fixed point: steps up to each check; there a value clamped or not finite is an
// error, and the tubes with a value past 3/4 of its range are re-ranged.
int fixed16_steps(mclbm_ctx* c, int64_t nsteps)
{
  while (nsteps > 0) {
    const int64_t m = std::min(nsteps, next_check(c->steps) - c->steps);
    nsteps -= m;
    int rc = plain_steps(c, m);
    if (rc) return rc;
    if (next_check(c->steps - 1) != c->steps) continue;
    std::vector<uint32_t> flags(c->ntubes);
    HIP_TRY(c, hipMemcpyAsync(flags.data(), c->dFlag, sizeof(uint32_t) * c->ntubes, hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    uint32_t any = 0;
    for (int t = 0; t < c->ntubes; ++t) {
      if (flags[t] & 2u)
        return fail(c, MCLBM_ESTATE, "fixed-point storage: a value of tube " + std::to_string(t) +
                                         " left its range or was not finite (step " + std::to_string(c->steps) + ")");
      any |= flags[t];
    }
    if (any && (rc = rerange(c, flags))) return rc;
  }
  return MCLBM_OK;
}
}  // namespace

extern "C" int mclbm_step(mclbm_ctx* c, int64_t nsteps)
{
  if (!c) return MCLBM_EARG;
  if (!c->initialised) return fail(c, MCLBM_EARG, "mclbm_init_fields or mclbm_load first");
  if (nsteps < 0) return fail(c, MCLBM_EARG, "nsteps must be non-negative");
  if (c->precision == MCLBM_I16) return fixed16_steps(c, nsteps);
  return plain_steps(c, nsteps);
}

extern "C" int64_t mclbm_range_refits(const mclbm_ctx* c) { return c ? c->reranges : -1; }

extern "C" int mclbm_read_moments(mclbm_ctx* c, double* X, double* rho, double* u, double* p, double* T,
                                  int on_device)
{
  if (!c) return MCLBM_EARG;
  if (!c->initialised) return fail(c, MCLBM_EARG, "no state yet");
  const int64_t N = c->n;
  const int M = c->M;
  const unsigned grid = (unsigned)c->nblocks;
  if (on_device) {
    c->ops.read(c->dPr, launch_all(c), c->pop[c->cur], X, rho, u, p, T, grid, c->stream);
    int rc = check_launch(c, "k_read");
    if (rc) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MCLBM_OK;
  }
  double* st = c->staging;
  double* sX = st;
  double* srho = st + (size_t)M * N;
  double* su = st + (size_t)(M + 1) * N;
  double* sp = st + (size_t)(M + 4) * N;
  double* sT = st + (size_t)(M + 5) * N;
  c->ops.read(c->dPr, launch_all(c), c->pop[c->cur], X ? sX : nullptr, rho ? srho : nullptr, u ? su : nullptr,
              p ? sp : nullptr, T ? sT : nullptr, grid, c->stream);
  int rc = check_launch(c, "k_read");
  if (rc) return rc;
  if (X) HIP_TRY(c, hipMemcpyAsync(X, sX, sizeof(double) * M * N, hipMemcpyDeviceToHost, c->stream));
  if (rho) HIP_TRY(c, hipMemcpyAsync(rho, srho, sizeof(double) * N, hipMemcpyDeviceToHost, c->stream));
  if (u) HIP_TRY(c, hipMemcpyAsync(u, su, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, c->stream));
  if (p) HIP_TRY(c, hipMemcpyAsync(p, sp, sizeof(double) * N, hipMemcpyDeviceToHost, c->stream));
  if (T) HIP_TRY(c, hipMemcpyAsync(T, sT, sizeof(double) * N, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return MCLBM_OK;
}

extern "C" int mclbm_read_fields_f32(mclbm_ctx* c, float* out, int on_device)
{
  if (!c) return MCLBM_EARG;
  if (!out) return fail(c, MCLBM_EARG, "out is NULL");
  if (!c->initialised) return fail(c, MCLBM_EARG, "no state yet");
  const int64_t N = c->n;
  const int M = c->M;
  double* st = c->staging;
  double* sX = st;
  double* su = st + (size_t)M * N;
  double* sT = st + (size_t)(M + 3) * N;
  double* sp = st + (size_t)(M + 4) * N;
  // the packed FP32 fields reuse the staging area behind the doubles:
  // 1.5 (M + 5) n doubles <= (2 M + 8) n for M >= 1
  float* sF = (float*)(st + (size_t)(M + 5) * N);
  static_assert(sizeof(float) * 2 == sizeof(double), "staging holds (M+5) floats in (M+5)/2 doubles");
  const unsigned grid = (unsigned)c->nblocks;
  c->ops.read(c->dPr, launch_all(c), c->pop[c->cur], sX, nullptr, su, sp, sT, grid, c->stream);
  int rc = check_launch(c, "k_read");
  if (rc) return rc;
  float* dst = on_device ? out : sF;
  hipLaunchKernelGGL(k_pack_f32, dim3(grid), dim3(BLOCK), 0, c->stream, launch_all(c), c->dTubeN, M, sX, sT, su, sp,
                     dst);
  rc = check_launch(c, "k_pack_f32");
  if (rc) return rc;
  if (!on_device)
    HIP_TRY(c, hipMemcpyAsync(out, sF, sizeof(float) * (M + 5) * N, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return MCLBM_OK;
}

extern "C" int mclbm_conservation(mclbm_ctx* c, double* out)
{
  if (!c || !out) return c ? fail(c, MCLBM_EARG, "out is NULL") : MCLBM_EARG;
  if (!c->initialised) return fail(c, MCLBM_EARG, "no state yet");
  const int nv = c->M + 6;
  c->ops.conserved(c->dPd, launch_all(c), c->pop[c->cur], c->partial, (unsigned)c->nblocks, c->stream);
  int rc = check_launch(c, "k_conserved");
  if (rc) return rc;
  std::vector<double> tmp((size_t)c->ntubes * nv);
  rc = reduce_to_host(c, nv, tmp.data());
  if (rc) return rc;
  bool flagged = false;
  for (int t = 0; t < c->ntubes; ++t) {
    for (int k = 0; k < c->M + 5; ++k)
      out[(size_t)t * (c->M + 5) + (k < c->M ? c->xperm[k] : k)] = tmp[(size_t)t * nv + k];
    flagged = flagged || tmp[(size_t)t * nv + c->M + 5] != 0.0;
  }
  if (flagged) return fail(c, MCLBM_ENAN, "non-finite value or negative slaved density in the state");
  return MCLBM_OK;
}

extern "C" int mclbm_half_tube_moles(mclbm_ctx* c, double* out)
{
  if (!c || !out) return c ? fail(c, MCLBM_EARG, "out is NULL") : MCLBM_EARG;
  if (!c->initialised) return fail(c, MCLBM_EARG, "no state yet");
  const int nv = 2 * c->M;
  c->ops.half_moles(c->dPd, launch_all(c), c->pop[c->cur], c->partial, (unsigned)c->nblocks, c->stream);
  int rc = check_launch(c, "k_half_moles");
  if (rc) return rc;
  std::vector<double> tmp((size_t)c->ntubes * nv);
  rc = reduce_to_host(c, nv, tmp.data());
  if (rc) return rc;
  for (int t = 0; t < c->ntubes; ++t)
    for (int h = 0; h < 2; ++h)
      for (int a = 0; a < c->M; ++a)
        out[(size_t)t * nv + h * c->M + c->xperm[a]] = tmp[(size_t)t * nv + h * c->M + a];
  return MCLBM_OK;
}

extern "C" int64_t mclbm_step_count(const mclbm_ctx* c) { return c ? c->steps : -1; }

namespace {
struct CkptHeader {
  char magic[8];
  int32_t M, wall_x, precision, ntubes;
  int32_t weak, cvt;
  int64_t steps;
  int32_t slaved, pad;   // the caller's index of the slaved species
};
struct CkptTube {
  int32_t nx, ny, nz;
  uint32_t range_flag;   // fixed point: the tube's range flag between two checks
  RefTables tab;
};
const char kMagic[8] = "MCLBMv5";

size_t header_bytes(const mclbm_ctx* c) { return sizeof(CkptHeader) + sizeof(CkptTube) * c->ntubes; }
}  // namespace

extern "C" size_t mclbm_state_bytes(const mclbm_ctx* c)
{
  if (!c) return 0;
  return header_bytes(c) + (size_t)c->L * Q * c->n * c->ops.s_bytes;
}

extern "C" int mclbm_save(mclbm_ctx* c, void* host_buf, size_t bytes)
{
  if (!c || !host_buf) return c ? fail(c, MCLBM_EARG, "buffer is NULL") : MCLBM_EARG;
  if (!c->initialised) return fail(c, MCLBM_EARG, "no state yet");
  if (bytes < mclbm_state_bytes(c)) return fail(c, MCLBM_EARG, "buffer too small");
  CkptHeader h{};
  std::memcpy(h.magic, kMagic, 8);
  h.M = c->M; h.wall_x = c->wall_x | (c->wall_y << 2);   // the x and y boundary kinds
  h.precision = c->precision; h.ntubes = c->ntubes; h.weak = c->weak; h.cvt = c->cvt;
  h.steps = c->steps;
  h.slaved = c->xperm[c->M - 1];
  std::vector<uint32_t> flags(c->ntubes, 0);
  if (c->precision == MCLBM_I16) {
    HIP_TRY(c, hipMemcpyAsync(flags.data(), c->dFlag, sizeof(uint32_t) * c->ntubes, hipMemcpyDeviceToHost,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  char* dst = (char*)host_buf;
  std::memcpy(dst, &h, sizeof(h));
  for (int t = 0; t < c->ntubes; ++t) {
    const TubeHost& th = c->tubes[t];
    CkptTube ct{};
    ct.nx = th.nx; ct.ny = th.ny; ct.nz = th.nz;
    ct.range_flag = flags[t];
    ct.tab = th.tab;
    std::memcpy(dst + sizeof(h) + sizeof(CkptTube) * t, &ct, sizeof(ct));
  }
  HIP_TRY(c, hipMemcpyAsync(dst + header_bytes(c), c->pop[c->cur], (size_t)c->L * Q * c->n * c->ops.s_bytes,
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return MCLBM_OK;
}

extern "C" int mclbm_load(mclbm_ctx* c, const void* host_buf, size_t bytes)
{
  if (!c || !host_buf) return c ? fail(c, MCLBM_EARG, "buffer is NULL") : MCLBM_EARG;
  if (bytes < mclbm_state_bytes(c)) return fail(c, MCLBM_EARG, "buffer too small");
  const char* src = (const char*)host_buf;
  CkptHeader h;
  std::memcpy(&h, src, sizeof(h));
  if (std::memcmp(h.magic, kMagic, 8) != 0 || h.M != c->M || h.wall_x != (c->wall_x | (c->wall_y << 2)) ||
      h.precision != c->precision ||
      h.ntubes != c->ntubes || h.weak != c->weak || h.cvt != c->cvt || h.slaved != c->xperm[c->M - 1])
    return fail(c, MCLBM_EARG, "checkpoint does not match this context");
  std::vector<CkptTube> ct(c->ntubes);
  for (int t = 0; t < c->ntubes; ++t) {
    std::memcpy(&ct[t], src + sizeof(h) + sizeof(CkptTube) * t, sizeof(CkptTube));
    if (ct[t].nx != c->tubes[t].nx || ct[t].ny != c->tubes[t].ny || ct[t].nz != c->tubes[t].nz)
      return fail(c, MCLBM_EARG, "checkpoint does not match this context");
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int t = 0; t < c->ntubes; ++t) {
    TubeHost& th = c->tubes[t];
    th.tab = ct[t].tab;
  }
  int rc = push_params(c);
  if (rc) return rc;
  HIP_TRY(c, hipMemcpyAsync(c->pop[0], src + header_bytes(c), (size_t)c->L * Q * c->n * c->ops.s_bytes,
                            hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->cur = 0;
  c->steps = h.steps;
  c->reranges = 0;
  if (c->precision == MCLBM_I16) {
    std::vector<uint32_t> flags(c->ntubes);
    for (int t = 0; t < c->ntubes; ++t) flags[t] = ct[t].range_flag;
    HIP_TRY(c, hipMemcpyAsync(c->dFlag, flags.data(), sizeof(uint32_t) * c->ntubes, hipMemcpyHostToDevice,
                              c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  c->initialised = true;
  return MCLBM_OK;
}

extern "C" int mclbm_set_timing(mclbm_ctx* c, int enable)
{
  if (!c) return MCLBM_EARG;
  int rc = harvest_timing(c);
  if (rc) return rc;
  c->timing = enable != 0;
  for (int k = 0; k < 3; ++k) {
    c->acc_ms[k] = 0.0;
    c->acc_launches[k] = 0;
  }
  return MCLBM_OK;
}

extern "C" int mclbm_kernel_stats(mclbm_ctx* c, int32_t kernel, double* total_ms, int64_t* launches,
                                  const char** name)
{
  if (!c) return MCLBM_EARG;
  if (kernel < 0 || kernel > 2) return fail(c, MCLBM_EARG, "unknown kernel id");
  int rc = harvest_timing(c);
  if (rc) return rc;
  if (total_ms) *total_ms = c->acc_ms[kernel];
  if (launches) *launches = c->acc_launches[kernel];
  if (name) *name = two_read(c) ? kernel_names_two_read[kernel] : kernel_names[kernel];
  return MCLBM_OK;
}

extern "C" int mclbm_get_launch(const mclbm_ctx* c, mclbm_launch* out)
{
  if (!c || !out) return MCLBM_EARG;
  *out = c->lc;
  return MCLBM_OK;
}

extern "C" int mclbm_set_launch(mclbm_ctx* c, const mclbm_launch* in)
{
  if (!c) return MCLBM_EARG;
  if (!in) return fail(c, MCLBM_EARG, "launch is NULL");
  if (in->variant < 0 || in->variant >= kern::NVARIANT) return fail(c, MCLBM_EARG, "variant must be 0 or 1");
  if ((in->swizzle | in->sequential | in->split | in->three_pass) & ~1)
    return fail(c, MCLBM_EARG, "swizzle, sequential, split and three_pass are 0 or 1");
  if (in->order != 0 && in->order != 1) return fail(c, MCLBM_EARG, "order must be 0 or 1");
  if (in->graph_steps < 0 || (in->graph_steps & 1) || in->graph_steps > 100000)
    return fail(c, MCLBM_EARG, "graph_steps must be an even number in 0..100000");
  if (in->shape < 0 || in->shape >= kern::NSHAPES) return fail(c, MCLBM_EARG, "shape must be in 0..5");
  const bool remap = in->order != c->lc.order || in->shape != c->lc.shape;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  drop_graph(c);
  c->lc = *in;
  if (remap) return push_block_map(c);
  return MCLBM_OK;
}

extern "C" int mclbm_autotune(mclbm_ctx* c, int32_t trial_steps, char* report, size_t report_len)
{
  if (!c) return MCLBM_EARG;
  if (!c->initialised) return fail(c, MCLBM_EARG, "mclbm_init_fields or mclbm_load first");
  if (trial_steps < 2) return fail(c, MCLBM_EARG, "trial_steps must be at least 2");
  if (c->timing) return fail(c, MCLBM_EARG, "disable timing before autotuning");
  const int G = trial_steps & ~1;
  std::vector<mclbm_launch> cands;
  // (three_pass, variant, split): the two-read step where compiled, then the three-pass step
  const int paths[6][3] = {{0, 0, 0}, {0, 1, 0}, {1, 0, 0}, {1, 1, 0}, {1, 0, 1}, {1, 1, 1}};
  const bool has_two_read = c->ops.state_species[0] != nullptr;
  for (int order = 0; order < (c->ntubes > 1 ? 2 : 1); ++order)
    for (const auto& pv : paths) {
      if (!pv[0] && !has_two_read) continue;
      for (int sw = 0; sw < 2; ++sw)
        for (int g = 0; g < 2; ++g) {
          mclbm_launch l{};
          l.three_pass = pv[0];
          l.variant = pv[1];
          l.split = pv[2];
          l.swizzle = sw;
          l.order = order;
          l.graph_steps = g ? G : 0;
          cands.push_back(l);
        }
    }
  hipEvent_t e0, e1;
  HIP_TRY(c, hipEventCreate(&e0));
  HIP_TRY(c, hipEventCreate(&e1));
  std::string rep = "three_pass variant split swizzle order graph_steps shape ms_per_step\n";
  double best = 1e300;
  mclbm_launch best_l = c->lc;
  int rc = MCLBM_OK;
  auto trial = [&](const mclbm_launch& l) -> int {
    int r = mclbm_set_launch(c, &l);
    if (r) return r;
    // first launches of this choice (graph build, caches), then start from buffer 0
    if ((r = mclbm_step(c, l.graph_steps ? G : 2))) return r;
    if (c->cur == 1 && (r = mclbm_step(c, 1))) return r;
    if (hipEventRecord(e0, c->stream) != hipSuccess) return fail(c, MCLBM_EDEVICE, "hipEventRecord");
    if ((r = mclbm_step(c, G))) return r;
    if (hipEventRecord(e1, c->stream) != hipSuccess) return fail(c, MCLBM_EDEVICE, "hipEventRecord");
    if (hipEventSynchronize(e1) != hipSuccess) return fail(c, MCLBM_EDEVICE, "hipEventSynchronize");
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return fail(c, MCLBM_EDEVICE, "hipEventElapsedTime");
    const double per = ms / G;
    char line[128];
    std::snprintf(line, sizeof line, "%d %d %d %d %d %d %d %.6f\n", l.three_pass, l.variant, l.split, l.swizzle,
                  l.order, l.graph_steps, l.shape, per);
    rep += line;
    if (per < best) {
      best = per;
      best_l = l;
    }
    return MCLBM_OK;
  };
  for (const mclbm_launch& l : cands)
    if ((rc = trial(l))) break;
  // the block shapes, with the fastest path, swizzle, order and graph choice
  const mclbm_launch base = best_l;
  for (int k = 1; k < kern::NSHAPES && !rc; ++k) {
    mclbm_launch l = base;
    l.shape = k;
    rc = trial(l);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  rc = mclbm_set_launch(c, &best_l);
  if (rc) return rc;
  char line[128];
  std::snprintf(line, sizeof line, "chosen %d %d %d %d %d %d %d %.6f\n", best_l.three_pass, best_l.variant,
                best_l.split, best_l.swizzle, best_l.order, best_l.graph_steps, best_l.shape, best);
  rep += line;
  if (report && report_len > 0) {
    const size_t k = std::min(report_len - 1, rep.size());
    std::memcpy(report, rep.data(), k);
    report[k] = '\0';
  }
  return MCLBM_OK;
}

extern "C" int mclbm_nn_advance(mclbm_ctx* c, mclbm_nn* net, int32_t K, double resid_tol, double change_tol,
                                int32_t* used_fallback, double* max_residual, double* max_change)
{
  if (!c) return MCLBM_EARG;
  if (!net) return fail(c, MCLBM_EARG, "network is NULL");
  if (!c->initialised) return fail(c, MCLBM_EARG, "no state yet");
  if (K < 1) return fail(c, MCLBM_EARG, "K must be positive");
  if (std::isnan(resid_tol) || std::isnan(change_tol)) return fail(c, MCLBM_EARG, "tolerances must not be NaN");
  if (!c->xperm_identity)
    return fail(c, MCLBM_EUNSUPPORTED, "the surrogate takes contexts whose slaved species is the last (slaved = 0)");
  const int M = c->M;
  int channels = 0, species = 0;
  std::vector<int> dims;
  mclbm::nn::geometry(net, &channels, &species, &dims);
  if (channels != M + 5) return fail(c, MCLBM_EARG, "the network must have M + 5 channels (X, T, u, p)");
  if (species != 0 && species != M) return fail(c, MCLBM_EARG, "the network's species differ from the context's");
  if ((int)dims.size() != 3 * c->ntubes) return fail(c, MCLBM_EARG, "network and context have different tubes");
  for (int t = 0; t < c->ntubes; ++t)
    if (dims[3 * t] != c->tubes[t].nx || dims[3 * t + 1] != c->tubes[t].ny || dims[3 * t + 2] != c->tubes[t].nz)
      return fail(c, MCLBM_EARG, "network and context have different tubes");
  // conserved sums of the current state: masses of the species and energy per tube
  std::vector<double> before((size_t)c->ntubes * (M + 5));
  int rc = mclbm_conservation(c, before.data());
  if (rc) return rc;
  float *fin = nullptr, *fout = nullptr;
  mclbm_nn_io(net, &fin, &fout);
  rc = mclbm_read_fields_f32(c, fin, 1);
  if (rc) return rc;
  rc = mclbm_nn_forward(net);
  if (rc) return fail(c, rc, std::string("surrogate: ") + mclbm_nn_last_error(net));
  // the fields to install: mole fractions clipped at zero and renormalised
  const int64_t N = c->n;
  double* st = c->staging;
  double *X = st, *p = st + (size_t)M * N, *T = st + (size_t)(M + 1) * N, *u = st + (size_t)(M + 2) * N;
  const unsigned grid = (unsigned)c->nblocks;
  hipLaunchKernelGGL(k_pred_to_state, dim3(grid), dim3(BLOCK), 0, c->stream, (const Params<double>*)c->dPd,
                     launch_all(c), M, fin, fout, X, p, T, u, c->bad, c->chg);
  rc = check_launch(c, "k_pred_to_state");
  if (rc) return rc;
  std::vector<int> bad(c->nblocks);
  std::vector<float> chg(c->nblocks);
  HIP_TRY(c, hipMemcpyAsync(bad.data(), c->bad, sizeof(int) * c->nblocks, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(chg.data(), c->chg, sizeof(float) * c->nblocks, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  bool ok = true;
  for (int64_t b = 0; b < c->nblocks && ok; ++b) ok = bad[b] == 0;
  // the size of the hop: the largest change of a mole fraction at any node
  double change = HUGE_VAL;
  if (ok) {
    change = 0.0;
    for (int64_t b = 0; b < c->nblocks; ++b) change = std::max(change, (double)chg[b]);
  }
  // residual of the installed state: the largest relative change of a species'
  // mass or of the energy over any tube, which the walled or periodic lattice
  // keeps (to its rounding) and the network, predicting T and u directly, does not
  double mx = HUGE_VAL;
  if (ok) {
    hipLaunchKernelGGL(k_field_conserved, dim3(grid), dim3(BLOCK), 0, c->stream, (const Params<double>*)c->dPd,
                       launch_all(c), M, X, p, T, u, c->partial);
    rc = check_launch(c, "k_field_conserved");
    if (rc) return rc;
    std::vector<double> after((size_t)c->ntubes * (MAXM + 1));
    rc = reduce_to_host(c, MAXM + 1, after.data());
    if (rc) return rc;
    mx = 0.0;
    for (int t = 0; t < c->ntubes; ++t) {
      const double* b0 = &before[(size_t)t * (M + 5)];
      const double* a1 = &after[(size_t)t * (MAXM + 1)];
      double mass = 0.0;
      for (int a = 0; a < M; ++a) mass += b0[a];
      for (int a = 0; a < M; ++a)
        if (b0[a] > 1e-12 * mass) mx = std::max(mx, std::fabs(a1[a] - b0[a]) / b0[a]);
      mx = std::max(mx, std::fabs(a1[MAXM] - b0[M + 4]) / std::fabs(b0[M + 4]));
    }
    if (!std::isfinite(mx)) mx = HUGE_VAL;
    ok = mx <= resid_tol && change <= change_tol;
  }
  if (max_residual) *max_residual = mx;
  if (max_change) *max_change = change;
  if (ok) {
    const int64_t steps = c->steps;
    rc = mclbm_init_fields(c, X, p, T, u, 1);
    if (rc) return rc;
    c->steps = steps + K;
  } else {
    rc = mclbm_step(c, K);
    if (rc) return rc;
  }
  if (used_fallback) *used_fallback = ok ? 0 : 1;
  return MCLBM_OK;
}

// --------------------------------------------------------------------------
// Streaming copy (the read + write ceiling of the memory system)
// --------------------------------------------------------------------------
namespace {
typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_stream_copy(const f32x4* __restrict__ src, f32x4* __restrict__ dst,
                                                     size_t n16)
{
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    stream_store(dst + i, stream_load(src + i));
}
}  // namespace

extern "C" int mclbm_stream_copy(void* dst, const void* src, size_t bytes, void* hip_stream)
{
  if (!dst || !src || bytes % 16 || ((uintptr_t)dst | (uintptr_t)src) % 16) return MCLBM_EARG;
  const char *d = (const char*)dst, *s = (const char*)src;
  if (d < s + bytes && s < d + bytes) return MCLBM_EARG;
  if (bytes == 0) return MCLBM_OK;
  // a grid-stride loop over 8 blocks per compute unit: 2048 blocks of 256 threads
  hipLaunchKernelGGL(k_stream_copy, dim3(2048), dim3(256), 0, (hipStream_t)hip_stream, (const f32x4*)src,
                     (f32x4*)dst, bytes / 16);
  return hipGetLastError() == hipSuccess ? MCLBM_OK : MCLBM_EDEVICE;
}
