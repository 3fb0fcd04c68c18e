// mclbm.hip -- HIP kernels for gfx950 and the C ABI of libmclbm (include/mclbm.h).
//
// One time step = three launches over all nodes, one thread per node:
//   k_moments  read 27 (M+1) populations -> record {Phi_x, Phi_y, Phi_z, omega, C_p}
//   k_gfield   G_a = (1/omega - 1/2) d_a Phi_a from the record of the 18 neighbours
//   k_collide  read the populations again, X_a = -d_a G_a and d C_p from the
//              neighbours, collide every lattice, push to the neighbours of the
//              other buffer (bounce-back at x walls)
// The two reads of the populations are forced by the non-local terms of the
// momentum and energy collisions, which need the neighbours' moments at the same
// time level (eqs Xalpha and corrFourier). Populations are laid out as
// pop[l][i][z][y][x] so that a wavefront's 64 lanes read and write 64 consecutive
// values of one (lattice, direction) plane.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/mclbm.h"
#include "kernels.hpp"
#include "params_host.hpp"

using namespace mclbm;

namespace {

using kern::Ops;

int push_params(mclbm_ctx* c);
using kern::BLOCK;
using kern::RED_BLOCK;
using kern::ALIGN;
using kern::align_up;

// Deterministic second stage: out[k] = sum over blocks of partial[b][k].
__global__ __launch_bounds__(RED_BLOCK) void k_reduce_partials(const double* __restrict__ partial, int64_t nblocks,
                                                               int nv, double* __restrict__ out)
{
  __shared__ double buf[RED_BLOCK];
  for (int k = 0; k < nv; ++k) {
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < nblocks; b += RED_BLOCK) s += partial[(size_t)b * nv + k];
    buf[threadIdx.x] = s;
    __syncthreads();
    for (int w = RED_BLOCK / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) buf[threadIdx.x] += buf[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = buf[0];
    __syncthreads();
  }
}

bool pick_ops(int precision, int M, int walls, Ops& o)
{
  switch (precision) {
    case MCLBM_FP64: return pick_fp64(M, walls, o);
    case MCLBM_FP32: return pick_fp32_fp64(M, walls, o);
    case MCLBM_FP32_FP32: return pick_fp32(M, walls, o);
    case MCLBM_FP16: return pick_fp16(M, walls, o);
    case MCLBM_BF16: return pick_bf16(M, walls, o);
    default: return false;
  }
}

bool compute_is_fp64(int precision) { return precision == MCLBM_FP64 || precision == MCLBM_FP32; }

thread_local std::string g_last_error;

const char* kernel_names[3] = {"k_moments", "k_gfield", "k_collide"};

}  // namespace

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
struct mclbm_ctx {
  int M = 0, nx = 0, ny = 0, nz = 0, wall_x = 0, precision = 0, L = 0;
  int64_t n = 0;
  HostSpecies hs{};
  Ops ops{};
  hipStream_t stream = nullptr;
  int device = 0;
  // workspace regions
  char* ws = nullptr;
  size_t ws_bytes = 0;
  void* dPd = nullptr;      // Params<double>
  void* dPr = nullptr;      // Params<R> (R = float) or alias of dPd
  void* pop[2] = {nullptr, nullptr};
  void* rec = nullptr;
  void* G = nullptr;
  double* staging = nullptr;
  double* partial = nullptr;
  double* reduced = nullptr;
  int* bad = nullptr;
  int cur = 0;
  int64_t steps = 0;
  bool initialised = false;
  // host copies of the parameter blocks (kept alive for asynchronous uploads)
  Params<double> hPd{};
  Params<float> hPf{};
  double ref[MAXL][Q] = {};
  double ref0[MAXL] = {}, ref2[MAXL] = {}, scale[MAXL] = {};
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
  size_t pd, pr, pop, rec, G, staging, partial, reduced, bad, total;
};

Layout layout_for(int M, int64_t n, int precision)
{
  size_t s_bytes = 8, r_bytes = 8;
  switch (precision) {
    case MCLBM_FP64: s_bytes = 8; r_bytes = 8; break;
    case MCLBM_FP32: s_bytes = 4; r_bytes = 4; break;
    case MCLBM_FP32_FP32: s_bytes = 4; r_bytes = 4; break;
    case MCLBM_FP16: case MCLBM_BF16: s_bytes = 2; r_bytes = 4; break;
  }
  const int L = M + 1;
  const int64_t nblocks = (n + RED_BLOCK - 1) / RED_BLOCK;
  Layout l{};
  size_t off = 0;
  l.pd = off; off += align_up(sizeof(Params<double>));
  l.pr = off; off += align_up(sizeof(Params<float>));
  l.pop = off; off += 2 * align_up((size_t)L * Q * n * s_bytes);
  const int rec_fields = REC_RHOA + (M - 1) + 3 * M;
  l.rec = off; off += align_up((size_t)rec_fields * n * r_bytes);
  l.G = off; off += align_up((size_t)3 * n * r_bytes);
  l.staging = off; off += align_up((size_t)(M + 6) * n * sizeof(double));
  l.partial = off; off += align_up((size_t)nblocks * (MAXM + 6) * sizeof(double));
  l.reduced = off; off += align_up((MAXM + 6) * sizeof(double));
  l.bad = off; off += align_up((size_t)((n + BLOCK - 1) / BLOCK) * sizeof(int));
  l.total = off;
  return l;
}

int validate(const mclbm_params* p, std::string& err)
{
  if (!p) { err = "params is NULL"; return MCLBM_EARG; }
  if (p->M < 2 || p->M > MAXM) { err = "M must be in 2..8"; return MCLBM_EARG; }
  if (p->M > 4) { err = "this build compiles M = 2, 3, 4"; return MCLBM_EUNSUPPORTED; }
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) { err = "grid sizes must be positive"; return MCLBM_EARG; }
  const int64_t n = (int64_t)p->nx * p->ny * p->nz;
  if (n >= ((int64_t)1 << 31)) { err = "nx*ny*nz must be below 2^31"; return MCLBM_EARG; }
  if (p->wall_x != 0 && p->wall_x != 1) { err = "wall_x must be 0 or 1"; return MCLBM_EARG; }
  if (p->wall_x && p->nx < 2) { err = "walls need nx >= 2"; return MCLBM_EARG; }
  if (p->precision < MCLBM_FP64 || p->precision > MCLBM_BF16) { err = "unknown precision"; return MCLBM_EARG; }
  if (p->reserved0 || p->reserved1) { err = "reserved fields must be 0"; return MCLBM_EARG; }
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

unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

double absent_tol_for(int precision);

int push_params(mclbm_ctx* c)
{
  HIP_TRY(c, hipStreamSynchronize(c->stream));   // previous uploads from the host blocks are done
  const double tol = absent_tol_for(c->precision);
  fill_params<double>(c->hPd, c->hs, c->nx, c->ny, c->nz, c->wall_x, c->ref, c->ref0, c->ref2, c->scale, tol);
  fill_params<float>(c->hPf, c->hs, c->nx, c->ny, c->nz, c->wall_x, c->ref, c->ref0, c->ref2, c->scale, tol);
  HIP_TRY(c, hipMemcpyAsync(c->dPd, &c->hPd, sizeof(c->hPd), hipMemcpyHostToDevice, c->stream));
  if (!compute_is_fp64(c->precision))
    HIP_TRY(c, hipMemcpyAsync(c->dPr, &c->hPf, sizeof(c->hPf), hipMemcpyHostToDevice, c->stream));
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
    case MCLBM_FP16: return 1e-4;
    case MCLBM_BF16: return 1e-3;
    default: return 1e-12;
  }
}

int upload_params(mclbm_ctx* c, const RefState& rs)
{
  reference_tables(c->hs, rs, c->ref, c->ref0, c->ref2);
  for (int l = 0; l < MAXL; ++l) c->scale[l] = 1.0;
  for (int l = 0; l < c->L; ++l) {
    c->scale[l] = scale_for(c->precision, c->ref[l]);
    c->ref0[l] = 0.0;
    c->ref2[l] = 0.0;
    for (int i = 0; i < Q; ++i) {
      c->ref[l][i] = round_to_storage(c->precision, c->ref[l][i] * c->scale[l]) / c->scale[l];
      c->ref0[l] += c->ref[l][i];
      c->ref2[l] += c->ref[l][i] * cx(i) * cx(i);
    }
  }
  return push_params(c);
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

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" size_t mclbm_workspace_bytes(const mclbm_params* p)
{
  std::string err;
  if (validate(p, err) != MCLBM_OK) {
    g_last_error = err;
    return 0;
  }
  return layout_for(p->M, (int64_t)p->nx * p->ny * p->nz, p->precision).total;
}

extern "C" int mclbm_create(const mclbm_params* p, void* dev_workspace, size_t bytes, void* hip_stream,
                            mclbm_ctx** out)
{
  if (!out) return fail(nullptr, MCLBM_EARG, "out is NULL");
  *out = nullptr;
  std::string err;
  int rc = validate(p, err);
  if (rc != MCLBM_OK) return fail(nullptr, rc, err);
  const int64_t n = (int64_t)p->nx * p->ny * p->nz;
  Layout lay = layout_for(p->M, n, p->precision);
  if (!dev_workspace) return fail(nullptr, MCLBM_EARG, "workspace is NULL");
  if (((uintptr_t)dev_workspace) % ALIGN) return fail(nullptr, MCLBM_EARG, "workspace must be 256-byte aligned");
  if (bytes < lay.total) return fail(nullptr, MCLBM_EARG, "workspace too small");
  mclbm_ctx* c = new (std::nothrow) mclbm_ctx();
  if (!c) return fail(nullptr, MCLBM_EARG, "out of host memory");
  c->M = p->M; c->nx = p->nx; c->ny = p->ny; c->nz = p->nz; c->wall_x = p->wall_x;
  c->precision = p->precision; c->L = p->M + 1; c->n = n;
  c->hs.M = p->M;
  for (int a = 0; a < p->M; ++a) {
    c->hs.m[a] = p->molar_mass[a];
    c->hs.cv[a] = p->cv[a];
    c->hs.mu[a] = p->mu[a];
    c->hs.lam[a] = p->lambda[a];
    for (int b = 0; b < p->M; ++b) c->hs.D[a][b] = p->D[a * p->M + b];
  }
  if (!pick_ops(p->precision, p->M, p->wall_x, c->ops)) {
    delete c;
    return fail(nullptr, MCLBM_EUNSUPPORTED, "no kernels compiled for this configuration");
  }
  c->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(nullptr, MCLBM_EDEVICE, "hipGetDevice failed");
  }
  char* ws = (char*)dev_workspace;
  c->ws = ws; c->ws_bytes = bytes;
  c->dPd = ws + lay.pd;
  c->dPr = compute_is_fp64(p->precision) ? c->dPd : (void*)(ws + lay.pr);
  const size_t popb = align_up((size_t)c->L * Q * n * c->ops.s_bytes);
  c->pop[0] = ws + lay.pop;
  c->pop[1] = ws + lay.pop + popb;
  c->rec = ws + lay.rec;
  c->G = ws + lay.G;
  c->staging = (double*)(ws + lay.staging);
  c->partial = (double*)(ws + lay.partial);
  c->reduced = (double*)(ws + lay.reduced);
  c->bad = (int*)(ws + lay.bad);
  *out = c;
  return MCLBM_OK;
}

extern "C" void mclbm_destroy(mclbm_ctx* c)
{
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  for (auto e : c->ev_pool) (void)hipEventDestroy(e);
  delete c;
}

extern "C" const char* mclbm_last_error(const mclbm_ctx* c)
{
  return c ? c->err.c_str() : g_last_error.c_str();
}

namespace {

// Reduce NV values from per-block partials to host out[NV].
int reduce_to_host(mclbm_ctx* c, int64_t nblocks, int nv, double* out)
{
  hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(RED_BLOCK), 0, c->stream, c->partial, nblocks, nv, c->reduced);
  int rc = check_launch(c, "k_reduce_partials");
  if (rc) return rc;
  HIP_TRY(c, hipMemcpyAsync(out, c->reduced, sizeof(double) * nv, hipMemcpyDeviceToHost, c->stream));
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
  const int64_t n = c->n;
  const double *dX = X, *dp = p, *dT = T, *du = u;
  RefState rs{};
  if (!on_device) {
    // host fields: validate, compute the reference state here, stage to the device
    double sum[MAXM + 2] = {};
    for (int64_t i = 0; i < n; ++i) {
      double xs = 0.0;
      for (int a = 0; a < M; ++a) {
        const double v = X[(size_t)a * n + i];
        if (!(v >= 0.0)) return fail(c, MCLBM_EARG, "mole fractions must be non-negative");
        xs += v;
        sum[a] += v;
      }
      if (std::fabs(xs - 1.0) > 1e-9) return fail(c, MCLBM_EARG, "mole fractions must sum to 1");
      sum[M] += p[i];
      sum[M + 1] += T[i];
    }
    for (int a = 0; a < M; ++a) rs.X[a] = sum[a] / n;
    rs.p = sum[M] / n;
    rs.T = sum[M + 1] / n;
    double* st = c->staging;
    HIP_TRY(c, hipMemcpyAsync(st, X, sizeof(double) * M * n, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(st + (size_t)M * n, p, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(st + (size_t)(M + 1) * n, T, sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(st + (size_t)(M + 2) * n, u, sizeof(double) * 3 * n, hipMemcpyHostToDevice, c->stream));
    dX = st;
    dp = st + (size_t)M * n;
    dT = st + (size_t)(M + 1) * n;
    du = st + (size_t)(M + 2) * n;
  } else {
    const int64_t nb = grid_for(n, RED_BLOCK);
    c->ops.field_sums(n, dX, dp, dT, c->partial, (unsigned)nb, c->stream);
    int rc = check_launch(c, "k_field_sums");
    if (rc) return rc;
    double sum[MAXM + 2] = {};
    rc = reduce_to_host(c, nb, M + 2, sum);
    if (rc) return rc;
    for (int a = 0; a < M; ++a) rs.X[a] = sum[a] / n;
    rs.p = sum[M] / n;
    rs.T = sum[M + 1] / n;
    double xs = 0.0;
    for (int a = 0; a < M; ++a) xs += rs.X[a];
    if (!(std::fabs(xs - 1.0) < 1e-6) || !(rs.p > 0) || !(rs.T > 0))
      return fail(c, MCLBM_EARG, "fields are not a valid state (mean mole fractions, p, T)");
  }
  int rc = upload_params(c, rs);
  if (rc) return rc;
  const unsigned grid = grid_for(n, BLOCK);
  c->ops.init(c->dPd, dX, dp, dT, du, c->pop[0], c->bad, grid, c->stream);
  rc = check_launch(c, "k_init");
  if (rc) return rc;
  std::vector<int> bad(grid);
  HIP_TRY(c, hipMemcpyAsync(bad.data(), c->bad, sizeof(int) * grid, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (unsigned b = 0; b < grid; ++b)
    if (bad[b]) return fail(c, MCLBM_ESTATE, "infeasible initial state: need T > 0, p > 0, R_a T + u^2 < 1");
  c->cur = 0;
  c->steps = 0;
  c->initialised = true;
  return MCLBM_OK;
}

extern "C" int mclbm_step(mclbm_ctx* c, int64_t nsteps)
{
  if (!c) return MCLBM_EARG;
  if (!c->initialised) return fail(c, MCLBM_EARG, "mclbm_init_fields or mclbm_load first");
  if (nsteps < 0) return fail(c, MCLBM_EARG, "nsteps must be non-negative");
  const unsigned grid = grid_for(c->n, BLOCK);
  for (int64_t t = 0; t < nsteps; ++t) {
    int e0 = 0, e1 = 0, e2 = 0, e3 = 0, rc = 0;
    if (c->timing && (rc = record_event(c, e0))) return rc;
    c->ops.moments(c->dPd, c->pop[c->cur], c->rec, grid, c->stream);
    if (c->timing && (rc = record_event(c, e1))) return rc;
    c->ops.gfield(c->dPd, c->rec, c->G, grid, c->stream);
    if (c->timing && (rc = record_event(c, e2))) return rc;
    c->ops.collide(c->dPr, c->pop[c->cur], c->pop[1 - c->cur], c->rec, c->G, (uint32_t)c->steps, grid,
                   c->stream);
    if (c->timing) {
      if ((rc = record_event(c, e3))) return rc;
      c->ev_pairs[0].push_back({e0, e1});
      c->ev_pairs[1].push_back({e1, e2});
      c->ev_pairs[2].push_back({e2, e3});
    }
    rc = check_launch(c, "mclbm_step");
    if (rc) return rc;
    c->cur = 1 - c->cur;
    c->steps += 1;
    if (c->timing && c->ev_used > 3000 && (rc = harvest_timing(c))) return rc;
  }
  return MCLBM_OK;
}

extern "C" int mclbm_read_moments(mclbm_ctx* c, double* X, double* rho, double* u, double* p, double* T,
                                  int on_device)
{
  if (!c) return MCLBM_EARG;
  if (!c->initialised) return fail(c, MCLBM_EARG, "no state yet");
  const int64_t n = c->n;
  const int M = c->M;
  const unsigned grid = grid_for(n, BLOCK);
  if (on_device) {
    c->ops.read(c->dPr, c->pop[c->cur], X, rho, u, p, T, grid, c->stream);
    int rc = check_launch(c, "k_read");
    if (rc) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return MCLBM_OK;
  }
  double* st = c->staging;
  double* sX = st;
  double* srho = st + (size_t)M * n;
  double* su = st + (size_t)(M + 1) * n;
  double* sp = st + (size_t)(M + 4) * n;
  double* sT = st + (size_t)(M + 5) * n;
  c->ops.read(c->dPr, c->pop[c->cur], X ? sX : nullptr, rho ? srho : nullptr, u ? su : nullptr, p ? sp : nullptr,
              T ? sT : nullptr, grid, c->stream);
  int rc = check_launch(c, "k_read");
  if (rc) return rc;
  if (X) HIP_TRY(c, hipMemcpyAsync(X, sX, sizeof(double) * M * n, hipMemcpyDeviceToHost, c->stream));
  if (rho) HIP_TRY(c, hipMemcpyAsync(rho, srho, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  if (u) HIP_TRY(c, hipMemcpyAsync(u, su, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, c->stream));
  if (p) HIP_TRY(c, hipMemcpyAsync(p, sp, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  if (T) HIP_TRY(c, hipMemcpyAsync(T, sT, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return MCLBM_OK;
}

extern "C" int mclbm_conservation(mclbm_ctx* c, double* out)
{
  if (!c || !out) return c ? fail(c, MCLBM_EARG, "out is NULL") : MCLBM_EARG;
  if (!c->initialised) return fail(c, MCLBM_EARG, "no state yet");
  const int nv = c->M + 6;
  const int64_t nb = grid_for(c->n, RED_BLOCK);
  c->ops.conserved(c->dPd, c->pop[c->cur], c->partial, (unsigned)nb, c->stream);
  int rc = check_launch(c, "k_conserved");
  if (rc) return rc;
  double tmp[MAXM + 6];
  rc = reduce_to_host(c, nb, nv, tmp);
  if (rc) return rc;
  for (int k = 0; k < c->M + 5; ++k) out[k] = tmp[k];
  if (tmp[c->M + 5] != 0.0) return fail(c, MCLBM_ENAN, "non-finite value or negative slaved density in the state");
  return MCLBM_OK;
}

extern "C" int64_t mclbm_step_count(const mclbm_ctx* c) { return c ? c->steps : -1; }

namespace {
struct CkptHeader {
  char magic[8];
  int32_t M, nx, ny, nz, wall_x, precision;
  int64_t steps;
  double ref[MAXL][Q], ref0[MAXL], ref2[MAXL], scale[MAXL];
};
}  // namespace

extern "C" size_t mclbm_state_bytes(const mclbm_ctx* c)
{
  if (!c) return 0;
  return sizeof(CkptHeader) + (size_t)c->L * Q * c->n * c->ops.s_bytes;
}

extern "C" int mclbm_save(mclbm_ctx* c, void* host_buf, size_t bytes)
{
  if (!c || !host_buf) return c ? fail(c, MCLBM_EARG, "buffer is NULL") : MCLBM_EARG;
  if (!c->initialised) return fail(c, MCLBM_EARG, "no state yet");
  if (bytes < mclbm_state_bytes(c)) return fail(c, MCLBM_EARG, "buffer too small");
  CkptHeader h{};
  std::memcpy(h.magic, "MCLBMv1", 8);
  h.M = c->M; h.nx = c->nx; h.ny = c->ny; h.nz = c->nz; h.wall_x = c->wall_x; h.precision = c->precision;
  h.steps = c->steps;
  std::memcpy(h.ref, c->ref, sizeof(h.ref));
  std::memcpy(h.ref0, c->ref0, sizeof(h.ref0));
  std::memcpy(h.ref2, c->ref2, sizeof(h.ref2));
  std::memcpy(h.scale, c->scale, sizeof(h.scale));
  std::memcpy(host_buf, &h, sizeof(h));
  HIP_TRY(c, hipMemcpyAsync((char*)host_buf + sizeof(h), c->pop[c->cur], (size_t)c->L * Q * c->n * c->ops.s_bytes,
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return MCLBM_OK;
}

extern "C" int mclbm_load(mclbm_ctx* c, const void* host_buf, size_t bytes)
{
  if (!c || !host_buf) return c ? fail(c, MCLBM_EARG, "buffer is NULL") : MCLBM_EARG;
  if (bytes < mclbm_state_bytes(c)) return fail(c, MCLBM_EARG, "buffer too small");
  CkptHeader h;
  std::memcpy(&h, host_buf, sizeof(h));
  if (std::memcmp(h.magic, "MCLBMv1", 8) != 0 || h.M != c->M || h.nx != c->nx || h.ny != c->ny || h.nz != c->nz ||
      h.wall_x != c->wall_x || h.precision != c->precision)
    return fail(c, MCLBM_EARG, "checkpoint does not match this context");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  std::memcpy(c->ref, h.ref, sizeof(h.ref));
  std::memcpy(c->ref0, h.ref0, sizeof(h.ref0));
  std::memcpy(c->ref2, h.ref2, sizeof(h.ref2));
  std::memcpy(c->scale, h.scale, sizeof(h.scale));
  int rc = push_params(c);
  if (rc) return rc;
  HIP_TRY(c, hipMemcpyAsync(c->pop[0], (const char*)host_buf + sizeof(h), (size_t)c->L * Q * c->n * c->ops.s_bytes,
                            hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->cur = 0;
  c->steps = h.steps;
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
  if (name) *name = kernel_names[kernel];
  return MCLBM_OK;
}
