// node_ops.hpp -- per-node work of one time step of the M+2-lattice mixture
// lattice Boltzmann model (Sawant, Dorschner, Karlin, arXiv 2004.11286),
// written as inlined functions that the HIP kernels call once per lattice node.
//
// Storage: pop[l][i][n] with l = 0..NS-1 the stored species, l = NS the
// momentum lattice f, l = NS+1 the energy lattice g; n = x + nx (y + ny z).
// Under strong coupling (Sec. 3.5.2) NS = M-1: species M is slaved to the
// momentum lattice and no quantity ever reads its populations. Under weak
// coupling (Sec. 3.5.1) NS = M: the species subsystem of Sec. 2 keeps its own
// density and velocity (eqs rhoSPEC, uSPEC) and takes T from the energy lattice.
// Stored values are d = s_l (f - f_ref,l,i).
//
// A step is three passes:
//   state_node    reads every population of a node, forms the moments in FP64,
//                 the macroscopic state, the transport coefficients, the
//                 Stefan--Maxwell diffusion velocities (eq transform12) and the
//                 non-equilibrium energy flux, and writes them as a node record;
//   gfield_node   G_a = (1/omega - 1/2) d_a Phi_a from the neighbours' records;
//   collide_node  collides one lattice at a time from the record (reading each
//                 population once), restores the exact incoming mass, momentum
//                 and energy of the lattice, and pushes the post-collision values
//                 to the neighbours (streaming), bouncing them back at x walls.
#pragma once

#include <type_traits>


#include <device_ops.hpp>   // device primitives (include path: csrc/)

#include "lattice.hpp"

namespace mclbm {

// Node record (structure of arrays, rec[k * n + node]).
enum {
  REC_PHIX = 0, REC_PHIY = 1, REC_PHIZ = 2,   // Phi_a = rho u_a (1 - 3 R T) - rho u_a^3 (eq Xalpha)
  REC_OMEGA = 3, REC_CP = 4,                   // omega (eq omega), mixture C_p
  REC_RHO = 5, REC_UX = 6, REC_UY = 7, REC_UZ = 8, REC_T = 9, REC_OMEGA1 = 10,
  REC_QNX = 11, REC_QNY = 12, REC_QNZ = 13,    // q - q^eq - u.(P - P^eq)
  REC_RHOA = 14                                // then rho_a (stored species), V_a (3 M),
};                                             // and under weak coupling u_s (3)
template <int M, bool WEAK = false, bool CVT = false>
struct RecLayout {
  static constexpr int V = REC_RHOA + Lat<M, WEAK>::NS;
  static constexpr int US = V + 3 * M;
  static constexpr int YF = US + (WEAK ? 3 : 0);         // with C_v(T): Y_a, a < M-1
  static constexpr int FIELDS = YF + (CVT ? M - 1 : 0);
};

// Temperature-dependent specific heats (Sec. 3.1): the mixture's C_v(T) =
// sum_k c_k T^k with c_k = sum_a Y_a c_ak (eq Cvmix), and its integral from
// T_0 = 0, U(T) = sum_a Y_a U_a(T) (eqs specUa, Umix).
template <typename R, int M>
__host__ __device__ __forceinline__ void mix_cv_poly(const Params<R>& P, const R Y[M], R c[4])
{
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    c[k] = R(0);
#pragma unroll
    for (int a = 0; a < M; ++a) c[k] += Y[a] * P.cvc[a][k];
  }
}

template <typename R>
__host__ __device__ __forceinline__ R poly_cv(const R c[4], R T)
{
  return c[0] + T * (c[1] + T * (c[2] + T * c[3]));
}

template <typename R>
__host__ __device__ __forceinline__ R poly_U(const R c[4], R T)
{
  return T * (c[0] + T * (c[1] * R(0.5) + T * (c[2] * R(1.0 / 3.0) + T * (c[3] * R(0.25)))));
}

// T from U(T) = e (eq temperature) by Newton's method. With c_0 > 0 and c_k >= 0,
// U is increasing and convex and e / c_0 bounds the root from above, so the
// iterates fall monotonically; the loop ends when the step is below 1e-15 T
// (a few iterations), or after 40.
template <typename R>
__host__ __device__ __forceinline__ R solve_temperature(const R c[4], R e)
{
  R T = e / c[0];
  for (int it = 0; it < 40; ++it) {
    const R dT = (poly_U(c, T) - e) / poly_cv(c, T);
    T -= dT;
    if (!(dT > R(1e-15) * T || dT < -R(1e-15) * T)) break;
  }
  return T;
}

// Macroscopic state of a node (Secs. 2.1, 3.1, 3.2; strong coupling Sec. 3.5.2).
template <typename R, int M>
struct Mix {
  R rho, inv_rho, u[3], usq, rhoE;
  R rho_a[M], Y[M], X[M];
  R mmix, Rg, Cv, Cp, T, P;
};

// rho_s: species densities. Strong coupling: rho_s[0..M-2] stored, the slaved
// species takes the deficit and Y_a = rho_a / rho. Weak coupling: all M stored,
// Y_a = rho_a / sum_b rho_b (the species subsystem's own density, eq rhoSPEC).
template <typename R, int M, bool WEAK = false, bool CVT = false>
__host__ __device__ __forceinline__ void mixture_state(const Params<R>& P, R rho, const R j[3], R rhoE,
                                              const R rho_s[M], Mix<R, M>& s)
{
  s.rho = rho;
  s.inv_rho = R(1) / rho;
  s.rhoE = rhoE;
  s.usq = R(0);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    s.u[k] = j[k] * s.inv_rho;
    s.usq += s.u[k] * s.u[k];
  }
  R inv_rs = s.inv_rho;
  if constexpr (WEAK) {
    R rs = R(0);
#pragma unroll
    for (int a = 0; a < M; ++a) {
      s.rho_a[a] = rho_s[a];
      rs += rho_s[a];
    }
    inv_rs = R(1) / rs;
  } else {
    R deficit = rho;
#pragma unroll
    for (int a = 0; a < M - 1; ++a) {
      s.rho_a[a] = rho_s[a];
      deficit -= rho_s[a];
    }
    s.rho_a[M - 1] = deficit;
  }
  R inv_m = R(0), Cv = R(0), Cp = R(0);
#pragma unroll
  for (int a = 0; a < M; ++a) {
    s.Y[a] = s.rho_a[a] * inv_rs;
    inv_m += s.Y[a] * P.inv_m[a];
    Cv += s.Y[a] * P.cv[a];
    Cp += s.Y[a] * P.cp[a];
  }
  s.Rg = inv_m;                      // R = R_U / m with R_U = 1
  s.mmix = R(1) / inv_m;
#pragma unroll
  for (int a = 0; a < M; ++a) s.X[a] = s.Y[a] * s.mmix * P.inv_m[a];
  if constexpr (CVT) {
    R c[4];
    mix_cv_poly<R, M>(P, s.Y, c);
    s.T = solve_temperature<R>(c, rhoE * s.inv_rho - R(0.5) * s.usq);
    s.Cv = poly_cv<R>(c, s.T);
    s.Cp = s.Cv + s.Rg;                                // Mayer
  } else {
    s.Cv = Cv;
    s.Cp = Cp;
    s.T = (rhoE * s.inv_rho - R(0.5) * s.usq) / Cv;  // constant specific heats, T_0 = 0
  }
  s.P = rho * s.Rg * s.T;
}

// Wilke's mixture viscosity and Mathur's mixture conductivity (Sec. 3.3).
template <typename R, int M>
__host__ __device__ __forceinline__ R mixture_viscosity(const Params<R>& P, const R X[M])
{
  R mu = R(0);
#pragma unroll
  for (int a = 0; a < M; ++a) {
    R den = R(0);
#pragma unroll
    for (int b = 0; b < M; ++b) den += P.phi[a][b] * X[b];
    mu += P.mu[a] * X[a] / den;
  }
  return mu;
}

template <typename R, int M>
__host__ __device__ __forceinline__ R mixture_conductivity(const Params<R>& P, const R X[M])
{
  R lin = R(0), harm = R(0);
#pragma unroll
  for (int a = 0; a < M; ++a) {
    lin += X[a] * P.lam[a];
    harm += X[a] * P.inv_lam[a];
  }
  return R(0.5) * (lin + R(1) / harm);
}

// The same at temperature T with temperature-dependent transport (R19):
// mu_a (T/T_ref)^s_mu,a in Wilke's rule, with phi_ab (eq wilkePhi) from those
// viscosities, and lambda_a (T/T_ref)^s_lam,a in Mathur's rule.
template <typename R, int M>
__host__ __device__ __forceinline__ void mixture_transport_T(const Params<R>& P, const R X[M], R T, R& mu, R& lam)
{
  if (!P.trn) {                        // constant transport: the precomputed Wilke factors
    mu = mixture_viscosity<R, M>(P, X);
    lam = mixture_conductivity<R, M>(P, X);
    return;
  }
  const R lt = log(T / P.T_ref);
  R mua[M], lin = R(0), harm = R(0);
#pragma unroll
  for (int a = 0; a < M; ++a) {
    mua[a] = P.mu[a] * exp(P.s_mu[a] * lt);
    const R la = P.lam[a] * exp(P.s_lam[a] * lt);
    lin += X[a] * la;
    harm += X[a] / la;
  }
  mu = R(0);
#pragma unroll
  for (int a = 0; a < M; ++a) {
    R den = R(0);
#pragma unroll
    for (int b = 0; b < M; ++b) {
      const R num = R(1) + sqrt((mua[a] / mua[b]) * sqrt(P.m[b] / P.m[a]));
      den += num * num / (sqrt(R(8)) * sqrt(R(1) + P.m[a] / P.m[b])) * X[b];
    }
    mu += mua[a] * X[a] / den;
  }
  lam = R(0.5) * (lin + R(1) / harm);
}

// 1 / D_ab(T) = (1 / D_ab) (T_ref / T)^s_D: the factor (T_ref / T)^s_D.
template <typename R>
__host__ __device__ __forceinline__ R inv_diffusivity_factor(const Params<R>& P, R T)
{
  return P.trn ? exp(-P.s_D * log(T / P.T_ref)) : R(1);
}

// A stored population (read once per pass: a nontemporal load) as a scaled deviation.
template <typename S, typename R>
__host__ __device__ __forceinline__ R load_dev(const S* __restrict__ p, size_t idx, R inv_scale)
{
  return R(stream_load(p + idx)) * inv_scale;
}

// Element idx of the array that starts at base. The base is the same for every
// lane of a wavefront (an array of one lattice direction, or of one record field,
// of one tube) and the byte offset fits in 32 bits (a tube's node count times the
// widest element is below 2^32, checked at context creation), so the access is a
// scalar base plus a 32-bit vector offset instead of 64-bit address arithmetic.
template <typename T>
__host__ __device__ __forceinline__ T* at32(T* base, uint32_t idx)
{
  return (T*)((char*)base + idx * (uint32_t)sizeof(T));
}

// Neighbour offsets of a node: x positions, y and z strides, wrapped periodically.
struct Nbr {
  uint32_t x[3], y[3], z[3];  // index contributions for c = -1, 0, +1
  bool lo, hi;                // node touches the x = 0 / x = nx-1 wall
  bool ylo, yhi;              // node touches the y = 0 / y = ny-1 wall
  uint32_t yy;                // the node's y
};

template <typename R>
__host__ __device__ __forceinline__ Nbr neighbours(const Params<R>& P, int64_t node)
{
  Nbr b;
  // node counts fit in 32 bits (checked at context creation): 32-bit division
  const uint32_t nx = (uint32_t)P.nx, ny = (uint32_t)P.ny, nz = (uint32_t)P.nz;
  const uint32_t nd = (uint32_t)node;
  const uint32_t x = nd % nx;
  const uint32_t t = nd / nx;
  const uint32_t y = t % ny;
  const uint32_t z = t / ny;
  const uint32_t sy = nx, sz = nx * ny;
  b.x[0] = x == 0 ? nx - 1 : x - 1;
  b.x[1] = x;
  b.x[2] = x == nx - 1 ? 0 : x + 1;
  b.y[0] = (y == 0 ? ny - 1 : y - 1) * sy;
  b.y[1] = y * sy;
  b.y[2] = (y == ny - 1 ? 0 : y + 1) * sy;
  b.z[0] = (z == 0 ? nz - 1 : z - 1) * sz;
  b.z[1] = z * sz;
  b.z[2] = (z == nz - 1 ? 0 : z + 1) * sz;
  b.lo = x == 0;
  b.hi = x == nx - 1;
  b.ylo = y == 0;
  b.yhi = y == ny - 1;
  b.yy = y;
  return b;
}

// Boundary kinds, one integer: the x ends (BC & 3) are periodic, half-way
// bounce-back walls (Sec. 4.2), open (equilibrium inlet at x = 0, zero-gradient
// outlet at x = nx - 1), or the opposed jets of Sec. 4.3 (on both x faces the
// nozzle rows are equilibrium inlets and the other rows free-slip walls);
// BC_YSLIP adds free-slip walls at both y ends (specular reflection) and BC_YOUT
// zero-gradient outlets at both y ends (the jets' outlets); otherwise y is periodic.
enum { BC_PERIODIC = 0, BC_WALLS = 1, BC_OPEN = 2, BC_JETS = 3, BC_YSLIP = 4, BC_YOUT = 8 };
__host__ __device__ constexpr int xbc(int BC) { return BC & 3; }

// A nozzle row of the opposed jets.
template <typename R>
__host__ __device__ __forceinline__ bool nozzle_row(const Params<R>& P, int y)
{
  return y >= P.noz0 && y < P.noz1;
}

// Stencil neighbour index: beyond an x wall the ghost node mirrors the boundary
// node; beyond an open end or a nozzle it holds the boundary node's values (zero
// gradient); beyond a free-slip y wall it mirrors the boundary node, beyond an
// outlet it holds its values. Mirror and zero gradient read the same node; they
// differ in the sign of the field's normal component (is_ghost, is_ghost_y).
template <int BC>
__host__ __device__ __forceinline__ uint32_t stencil_index(const Nbr& b, int ci, int cj, int ck)
{
  uint32_t xi = b.x[ci + 1];
  if (xbc(BC) != BC_PERIODIC) {
    if (ci < 0 && b.lo) xi = b.x[1];
    if (ci > 0 && b.hi) xi = b.x[1];
  }
  uint32_t yi = b.y[cj + 1];
  if (BC & (BC_YSLIP | BC_YOUT)) {
    if (cj < 0 && b.ylo) yi = b.y[1];
    if (cj > 0 && b.yhi) yi = b.y[1];
  }
  return xi + yi + b.z[ck + 1];
}

// A mirrored wall ghost in x (odd fields change sign there; not at open ends or
// nozzles). With the jets, the ghost of direction (ci, cj) lies in row y + cj
// (the boundary row beyond an outlet): a wall row beside the nozzles mirrors.
template <int BC, typename R>
__host__ __device__ __forceinline__ bool is_ghost(const Params<R>& P, const Nbr& b, int ci, int cj)
{
  if (xbc(BC) == BC_JETS) {
    if (!((ci < 0 && b.lo) || (ci > 0 && b.hi))) return false;
    int yg = (int)b.yy + cj;
    if (yg < 0) yg = 0;
    if (yg >= P.ny) yg = P.ny - 1;
    return !nozzle_row(P, yg);
  }
  return xbc(BC) == BC_WALLS && ((ci < 0 && b.lo) || (ci > 0 && b.hi));
}

// A mirrored free-slip ghost in y (Phi_y changes sign there).
template <int BC>
__host__ __device__ __forceinline__ bool is_ghost_y(const Nbr& b, int cj)
{
  return (BC & BC_YSLIP) && ((cj < 0 && b.ylo) || (cj > 0 && b.yhi));
}

// --------------------------------------------------------------------------
// Diffusion velocities: rho_a V_a + 1/2 sum_b K_ab (V_a - V_b) = j_a - rho_a u
// (eq transform12), with K_ab = P X_a X_b / D_ab; u and P are those of the
// species subsystem (the mixture's under strong coupling; under weak coupling
// u_s = sum_a j_a / sum_a rho_a and the Dalton pressure sum_a rho_a R_a T). A
// species whose density is at or below the detection threshold has a zero row
// and column: V_a = 0.
// --------------------------------------------------------------------------
template <typename R, int M>
__host__ __device__ __forceinline__ void species_present(const Params<R>& P, const R rho_a[M], R rho, bool present[M])
{
#pragma unroll
  for (int a = 0; a < M; ++a) present[a] = rho_a[a] > P.absent_tol * rho || rho_a[a] < -P.absent_tol * rho;
}

template <typename R, int M>
__host__ __device__ __forceinline__ void friction_matrix(const Params<R>& P, const Mix<R, M>& s, R Pk,
                                                const bool present[M], R K[M][M])
{
#pragma unroll
  for (int a = 0; a < M; ++a)
#pragma unroll
    for (int c = 0; c < M; ++c)
      K[a][c] = (present[a] && present[c]) ? Pk * s.X[a] * s.X[c] * P.invD[a][c] : R(0);
}

template <typename R, int M>
__host__ __device__ __forceinline__ void diffusion_velocities(const Mix<R, M>& s, const bool present[M], const R K[M][M],
                                                     const R js[M][3], const R uref[3], R V[M][3])
{
  R A[M][M], rhs[M][3];
#pragma unroll
  for (int a = 0; a < M; ++a) {
    R diag = present[a] ? s.rho_a[a] : R(1);
#pragma unroll
    for (int c = 0; c < M; ++c) {
      if (c == a) continue;
      diag += R(0.5) * K[a][c];
      A[a][c] = -R(0.5) * K[a][c];
    }
    A[a][a] = diag;
#pragma unroll
    for (int k = 0; k < 3; ++k) rhs[a][k] = present[a] ? js[a][k] - s.rho_a[a] * uref[k] : R(0);
  }
  // Gaussian elimination without pivoting: the matrix is column diagonally dominant
#pragma unroll
  for (int c = 0; c < M; ++c) {
    const R inv = R(1) / A[c][c];
#pragma unroll
    for (int r = c + 1; r < M; ++r) {
      const R f = A[r][c] * inv;
#pragma unroll
      for (int c2 = c + 1; c2 < M; ++c2) A[r][c2] -= f * A[c][c2];
#pragma unroll
      for (int k = 0; k < 3; ++k) rhs[r][k] -= f * rhs[c][k];
    }
  }
#pragma unroll
  for (int r = M - 1; r >= 0; --r) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      R acc = rhs[r][k];
#pragma unroll
      for (int c = r + 1; c < M; ++c) acc -= A[r][c] * V[c][k];
      V[r][k] = acc / A[r][r];
    }
  }
}

// Sign-selected accumulation: acc += c v for c in {-1, 0, 1} known at compile time.
template <typename R>
__host__ __device__ __forceinline__ void acc_c(R& acc, int c, R v)
{
  if (c > 0) acc += v;
  if (c < 0) acc -= v;
}

// --------------------------------------------------------------------------
// Pass 1: node state -> record (FP64 arithmetic, record stored as Rec)
// --------------------------------------------------------------------------
template <typename S, typename Rec, int M, bool WEAK = false, bool CVT = false>
__host__ __device__ __forceinline__ void state_node(const Params<double>& P, const S* __restrict__ pop,
                                           Rec* __restrict__ rec, int64_t node)
{
  using D = double;
  const size_t n = (size_t)P.n;
  const uint32_t nd = (uint32_t)node;
  constexpr int NS = Lat<M, WEAK>::NS, LF = Lat<M, WEAK>::LF, LG = Lat<M, WEAK>::LG;
  D rho_s[M], js[M][3];
#pragma unroll
  for (int a = 0; a < NS; ++a) {
    D r = 0.0, ja[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const D d = load_dev<S, D>(at32(pop + (size_t)(a * Q + i) * n, nd), 0, dec_scale<S>(P, a, i));
      r += d;
      acc_c(ja[0], cx(i), d);
      acc_c(ja[1], cy(i), d);
      acc_c(ja[2], cz(i), d);
    }
    rho_s[a] = P.ref0[a] + r;
#pragma unroll
    for (int k = 0; k < 3; ++k) js[a][k] = ja[k];
    lattice_barrier();
  }
  if constexpr (!WEAK) rho_s[M - 1] = 0.0;
  D rho = 0.0, j[3] = {0.0, 0.0, 0.0}, Pd[3] = {0.0, 0.0, 0.0}, Pxy = 0.0, Pxz = 0.0, Pyz = 0.0;
  D rhoE = 0.0, q[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const D d = load_dev<S, D>(at32(pop + (size_t)(LF * Q + i) * n, nd), 0, dec_scale<S>(P, LF, i));
    rho += d;
    acc_c(j[0], cx(i), d);
    acc_c(j[1], cy(i), d);
    acc_c(j[2], cz(i), d);
    if (cx(i)) Pd[0] += d;
    if (cy(i)) Pd[1] += d;
    if (cz(i)) Pd[2] += d;
    acc_c(Pxy, cx(i) * cy(i), d);
    acc_c(Pxz, cx(i) * cz(i), d);
    acc_c(Pyz, cy(i) * cz(i), d);
    const D e = load_dev<S, D>(at32(pop + (size_t)(LG * Q + i) * n, nd), 0, dec_scale<S>(P, LG, i));
    rhoE += e;
    acc_c(q[0], cx(i), e);
    acc_c(q[1], cy(i), e);
    acc_c(q[2], cz(i), e);
  }
  rho += P.ref0[LF];
  rhoE += P.ref0[LG];
#pragma unroll
  for (int k = 0; k < 3; ++k) Pd[k] += P.ref2[LF][k];
  Mix<D, M> s;
  mixture_state<D, M, WEAK, CVT>(P, rho, j, rhoE, rho_s, s);
  D us[3], Pk = s.P;                     // velocity and pressure of the species subsystem
  if constexpr (WEAK) {
    D rs = 0.0;
#pragma unroll
    for (int a = 0; a < M; ++a) rs += s.rho_a[a];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      D jt = 0.0;
#pragma unroll
      for (int a = 0; a < M; ++a) jt += js[a][k];
      us[k] = jt / rs;                   // eq uSPEC
    }
    Pk = rs * s.Rg * s.T;                // Dalton: sum_a rho_a R_a T
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) {        // slaved species momentum: the deficit (eq uMATCH)
      D jm = j[k];
#pragma unroll
      for (int a = 0; a < M - 1; ++a) jm -= js[a][k];
      js[M - 1][k] = jm;
      us[k] = s.u[k];
    }
  }
  bool present[M];
  species_present<D, M>(P, s.rho_a, s.rho, present);
  D K[M][M], V[M][3];
  if constexpr (CVT) Pk *= inv_diffusivity_factor<D>(P, s.T);   // K_ab = P X_a X_b / D_ab(T)
  friction_matrix<D, M>(P, s, Pk, present, K);
  diffusion_velocities<D, M>(s, present, K, js, us, V);
  const D theta = s.Rg * s.T;
  D mu_mix, lam_mix;
  if constexpr (CVT) {
    mixture_transport_T<D, M>(P, s.X, s.T, mu_mix, lam_mix);
  } else {
    mu_mix = mixture_viscosity<D, M>(P, s.X);
    lam_mix = mixture_conductivity<D, M>(P, s.X);
  }
  const D omega = 2.0 * s.P / (s.P + 2.0 * mu_mix);
  const D omega1 = 2.0 * s.P * s.Cp / (s.P * s.Cp + 2.0 * lam_mix);
  // non-equilibrium energy flux q - q^eq - u.(P - P^eq), used by the energy collision
  D H = s.Cp * s.T;                      // mixture enthalpy (eq specH)
  if constexpr (CVT) {
    D c[4];
    mix_cv_poly<D, M>(P, s.Y, c);
    H = poly_U<D>(c, s.T) + s.Rg * s.T;
  }
  const D hyd = H + 0.5 * s.usq;
  const D Pn[3][3] = {{Pd[0], Pxy, Pxz}, {Pxy, Pd[1], Pyz}, {Pxz, Pyz, Pd[2]}};
  D qn[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    D up = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) up += s.u[c] * (Pn[c][k] - (c == k ? s.P : 0.0) - rho * s.u[c] * s.u[k]);
    qn[k] = q[k] - hyd * rho * s.u[k] - up;
  }
  auto put = [&](int f, D v) { buf_store<Rec, BUF_NT>(rec + (size_t)f * n, (uint32_t)n, nd, Rec(v)); };
#pragma unroll
  for (int k = 0; k < 3; ++k) put(REC_PHIX + k, j[k] * (1.0 - 3.0 * theta) - j[k] * s.u[k] * s.u[k]);
  put(REC_OMEGA, omega);
  put(REC_CP, s.Cp);
  put(REC_RHO, rho);
#pragma unroll
  for (int k = 0; k < 3; ++k) put(REC_UX + k, s.u[k]);
  put(REC_T, s.T);
  put(REC_OMEGA1, omega1);
#pragma unroll
  for (int k = 0; k < 3; ++k) put(REC_QNX + k, qn[k]);
#pragma unroll
  for (int a = 0; a < NS; ++a) put(REC_RHOA + a, s.rho_a[a]);
#pragma unroll
  for (int a = 0; a < M; ++a)
#pragma unroll
    for (int k = 0; k < 3; ++k) put(RecLayout<M, WEAK>::V + 3 * a + k, V[a][k]);
  if constexpr (WEAK) {
#pragma unroll
    for (int k = 0; k < 3; ++k) put(RecLayout<M, WEAK>::US + k, us[k]);
  }
  if constexpr (CVT) {
#pragma unroll
    for (int a = 0; a < M - 1; ++a) put(RecLayout<M, WEAK, CVT>::YF + a, s.Y[a]);
  }
}

// --------------------------------------------------------------------------
// Pass 2: G_a = (1/omega - 1/2) d_a Phi_a, with d_a = 3 sum_i w_i c_ia (.)(x + c_i)
// --------------------------------------------------------------------------
template <typename R, int BC>
__host__ __device__ __forceinline__ void gfield_node(const Params<double>& P, const R* __restrict__ rec,
                                            R* __restrict__ G, int64_t node)
{
  const size_t n = (size_t)P.n;
  const uint32_t nd = (uint32_t)node;
  Nbr b = neighbours(P, node);
  R dphi[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (csq(i) == 0) continue;
    const uint32_t nb = stencil_index<BC>(b, cx(i), cy(i), cz(i));
    const R w3 = R(3.0 * w13(i));
    if (cx(i)) {
      R v = *at32(rec + (size_t)REC_PHIX * n, nb);
      if (is_ghost<BC>(P, b, cx(i), cy(i))) v = -v; // Phi_x is odd under the wall mirror
      dphi[0] += cx(i) > 0 ? w3 * v : -(w3 * v);
    }
    if (cy(i)) {
      R v = *at32(rec + (size_t)REC_PHIY * n, nb);
      if (is_ghost_y<BC>(b, cy(i))) v = -v;         // Phi_y is odd under the y mirror
      dphi[1] += cy(i) > 0 ? w3 * v : -(w3 * v);
    }
    if (cz(i)) {
      R v = *at32(rec + (size_t)REC_PHIZ * n, nb);
      dphi[2] += cz(i) > 0 ? w3 * v : -(w3 * v);
    }
  }
  R om = *at32(rec + (size_t)REC_OMEGA * n, nd);
  R f = R(1) / om - R(0.5);
#pragma unroll
  for (int k = 0; k < 3; ++k) buf_store<R, BUF_NT>(G + (size_t)k * n, (uint32_t)n, nd, R(f * dphi[k]));
}

// --------------------------------------------------------------------------
// Pass 3: collide every lattice and push (stream) to the other buffer
// --------------------------------------------------------------------------
// Counter-based hash (a 32-bit integer mixer) for stochastic rounding.
__host__ __device__ __forceinline__ uint32_t mix32(uint32_t x)
{
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

// Conversion of a scaled deviation to the storage type. FP64 storage is exact and
// FP32 arithmetic with FP32 storage rounds to nearest; FP32 storage of FP64
// arithmetic and 16-bit storage round stochastically, which removes the bias
// that round-to-nearest accumulates where a value changes by less than its
// last place per step (the change is quantised to whole units of the last
// place; in the 20000-step ternary tube, round to nearest leaves the mole
// fractions 3.5e-5 off).
template <typename S, typename R>
struct Store {
  __host__ __device__ static S cvt(R v, uint32_t) { return S(v); }
};

template <>
struct Store<float, double> {
  __host__ __device__ static float cvt(double x, uint32_t rnd) { return cvt_sr_f32(x, rnd); }
};

template <>
struct Store<_Float16, float> {
  __host__ __device__ static _Float16 cvt(float x, uint32_t rnd) { return cvt_sr_f16(x, rnd); }
};

template <>
struct Store<__bf16, float> {
  __host__ __device__ static __bf16 cvt(float x, uint32_t rnd) { return cvt_sr_bf16(x, rnd); }
};

template <typename S>
constexpr bool is_fixed16() { return std::is_same<S, int16_t>::value; }

// Encoding and decoding factors of lattice l, direction i: one per lattice for
// the floating-point storage types, one per lattice and direction class for
// fixed point.
template <typename S, typename R>
__host__ __device__ __forceinline__ R enc_scale(const Params<R>& P, int l, int i)
{
  if constexpr (is_fixed16<S>()) return P.qs[l][ccls(i)];
  else return P.scale[l];
}

template <typename S, typename R>
__host__ __device__ __forceinline__ R dec_scale(const Params<R>& P, int l, int i)
{
  if constexpr (is_fixed16<S>()) return P.inv_qs[l][ccls(i)];
  else return P.inv_scale[l];
}

// Storage of an initial deviation (FP64 arithmetic): fixed point rounds to
// nearest and clamps (the initial range is chosen to hold every value).
template <typename S>
__host__ __device__ __forceinline__ S init_store(const Params<double>& P, int l, int i, double dev)
{
  if constexpr (is_fixed16<S>()) {
    const double x = rint(dev * P.qs[l][ccls(i)]);
    return (int16_t)(x > 32767.0 ? 32767.0 : (x < -32767.0 ? -32767.0 : x));
  } else {
    return S(dev * P.scale[l]);
  }
}

// Random words for stochastic rounding: one hash per (node, lattice, step), then
// a linear congruential sequence (only its upper bits are used). An additive
// (Weyl) sequence would save the multiply, but its fixed increment correlates the
// rounding of a node's directions (opposite directions nearly anti-correlated for
// some pairs), which leaves each rounding unbiased but raises the noise of the
// first moments: FP16 storage of the ternary tube drifted 1.7 times further from
// the FP64 result over 1000 steps.
// Fixed-point storage draws 8 bits per store, the two upper bytes of one word
// for two stores (next8; the lower bytes of a power-of-two LCG have short
// periods), and keeps the range of the rounded values (32768 plus the value in
// storage units) for range_check.
struct Rng {
  uint32_t s;
  uint32_t held = 0;
  bool have = false;
  float ymax = 32768.0f, ymin = 32768.0f;
  __host__ __device__ Rng(int64_t node, int l, uint32_t step)
      : s(mix32((uint32_t)node ^ mix32((uint32_t)l * 0x632BE5ABu + step * 0x9E3779B1u))) {}
  __host__ __device__ uint32_t next()
  {
    s = s * 1664525u + 1013904223u;
    return s;
  }
  __host__ __device__ uint32_t next8()
  {
    if (have) {
      have = false;
      return (held >> 16) & 0xFFu;
    }
    held = next();
    have = true;
    return held >> 24;
  }
};

// Round a post-collision deviation of lattice l, direction i to storage.
template <typename S, typename R>
__host__ __device__ __forceinline__ S to_store(const Params<R>& P, int l, int i, R dev, Rng& rng)
{
  if constexpr (is_fixed16<S>()) {
    float y;
    const int16_t v = fma_sr_i16(float(dev), float(P.qs[l][ccls(i)]), rng.next8(), y);
    rng.ymax = __builtin_elementwise_maximum(rng.ymax, y);   // NaN propagates
    rng.ymin = __builtin_elementwise_minimum(rng.ymin, y);
    return v;
  } else {
    return Store<S, R>::cvt(dev * P.scale[l], rng.next());
  }
}

template <typename S, typename R>
__host__ __device__ __forceinline__ R from_store(const Params<R>& P, int l, int i, S v)
{
  return R(v) * dec_scale<S, R>(P, l, i);
}

// Fixed-point storage: after a lattice's stores, set bit 0 of the context's range
// flag when a value passed 3/4 of its range (the host then re-ranges the state
// before the margin is used up), and bits 0 and 1 when one was clamped or not
// finite (the state is lost). One atomic per wavefront that sets it. Called after
// the pushes: a branch before them would hold every value of the lattice in
// registers until it (the fused f/g collision took 1.88 instead of 1.30 ms).
template <typename S, typename R>
__host__ __device__ __forceinline__ void range_check(const Params<R>& P, const Rng& rng)
{
  if constexpr (is_fixed16<S>()) {
    // in storage units: |v| past 24576, or past 32766 (clamped, or about to be)
    const bool hit = !(rng.ymax < 32768.0f + 24576.0f && rng.ymin > 32768.0f - 24576.0f);
    const uint64_t any = __ballot(hit);
    if (any) {
      const uint64_t bad = __ballot(hit && !(rng.ymax <= 32768.0f + 32766.0f && rng.ymin >= 32768.0f - 32766.0f));
      if ((int)__lane_id() == __ffsll((unsigned long long)any) - 1) atomicOr(P.range_flag, bad ? 3u : 1u);
    }
  }
}

// Streaming: write the post-collision value of direction i to the neighbour
// x + c_i of the other buffer, or bounce it back at an x wall. Open ends stream
// as periodic here; open_fix_node then rewrites what enters the two boundary
// planes (the wrapped values are exactly the ones an open end drops).
template <typename S, typename R, int BC>
__host__ __device__ __forceinline__ void push(const Params<R>& P, S* __restrict__ dst, const Nbr& b, int l, int i,
                                     int64_t node, S v)
{
  const size_t n = (size_t)P.n;
  const bool xout = (cx(i) < 0 && b.lo) || (cx(i) > 0 && b.hi);
  const bool yout = (cy(i) < 0 && b.ylo) || (cy(i) > 0 && b.yhi);
  // destination direction j and node d (a 32-bit index, as every node index here)
  int j = i;
  uint32_t d = b.x[cx(i) + 1] + b.y[cy(i) + 1] + b.z[cz(i) + 1];
  if (xbc(BC) == BC_WALLS && xout) {
    j = opp(i);                                       // half-way bounce-back
    d = (uint32_t)node;
  } else if (xbc(BC) == BC_JETS && xout && !((BC & BC_YOUT) && yout) &&
             !nozzle_row(P, (int)b.yy + cy(i))) {
    // beside a nozzle: free-slip wall, specular reflection (c_x reversed) at the
    // node's own x; through a nozzle the value wraps into a slot that
    // jets_fix_node overwrites with the inlet equilibrium
    j = i - 18 * cx(i);
    d = b.x[1] + b.y[cy(i) + 1] + b.z[cz(i) + 1];
  } else if ((BC & BC_YSLIP) && yout) {
    // free-slip y wall: specular reflection (c_y reversed) at the node's own y
    j = i - 6 * cy(i);
    d = b.x[cx(i) + 1] + b.y[1] + b.z[cz(i) + 1];
  }
  // cached stores: the shifted pushes of a wavefront merge into whole lines in the
  // cache. The buffer resource must be the same for every lane of the wavefront,
  // so the buffer store takes only values that keep their direction; a value
  // reflected into another direction (which lanes do depends on their position)
  // takes a global store. A wavefront away from every wall skips that branch.
  if (j == i) buf_store<S>(dst + (size_t)(l * Q + i) * n, (uint32_t)n, d, v);
  else dst[(size_t)(l * Q + j) * n + d] = v;
}

// Load the Q stored values of one lattice of a node into v (lat: the lattice's
// first direction array), all issued before any is used: the compiler barrier
// after the loads keeps the scheduler from interleaving each load with its use
// (one load in flight at a time), which it otherwise may do to save registers.
// Where this matters is decided per kernel (GROUP_LOADS in collide_node): holding
// a lattice's values costs registers, which other kernels need more.
template <typename S>
__host__ __device__ __forceinline__ void load_lattice(const S* __restrict__ lat, size_t n, uint32_t node, S v[Q])
{
#pragma unroll
  for (int i = 0; i < Q; ++i) v[i] = buf_load<S, BUF_NT>(lat + (size_t)i * n, (uint32_t)n, node);
  lattice_barrier();
}

// Opposed jets, after the collision has streamed periodically across the x faces'
// nozzle rows and across the y ends into dst (the wrapped values are exactly the
// ones that leave the domain there): what enters a boundary row (y = 0: c_y > 0;
// y = ny - 1: c_y < 0) comes from a ghost row holding the boundary row's
// post-collision state, shifted like any push (beyond an x face too, the nearest
// boundary node's), i.e. the value node (clamp(x - c_x), y_b, z - c_z) pushed into
// row 1 (or ny - 2); what enters a nozzle row's boundary node through its face is
// the inlet equilibrium of that jet. The slots read (rows 1 and ny - 2, directions
// entering those rows from the boundary rows) are never written here: the nodes
// of a launch do not interfere (1 <= noz0 < noz1 <= ny - 1, so ny >= 3).
template <typename S, typename R, int L>
__host__ __device__ __forceinline__ void jets_fix_node(const Params<R>& P, S* __restrict__ dst, int64_t node,
                                                       uint32_t step)
{
  const size_t n = (size_t)P.n;
  const int nx = P.nx, ny = P.ny;
  const int x = (int)((uint32_t)node % (uint32_t)nx);
  const int y = (int)(((uint32_t)node / (uint32_t)nx) % (uint32_t)ny);
  const int64_t row = node - x;                      // node index of (0, y, z)
  if (y == 0 || y == ny - 1) {
    const int cin = y == 0 ? 1 : -1;                 // c_y of the directions entering
    const int64_t inner = row + (int64_t)cin * nx;   // (0, y + cin, z)
#pragma unroll
    for (int l = 0; l < L; ++l)
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        if (cy(i) != cin) continue;
        int xs = x - cx(i);
        xs = xs < 0 ? 0 : (xs >= nx ? nx - 1 : xs);
        dst[(size_t)(l * Q + i) * n + node] = dst[(size_t)(l * Q + i) * n + inner + xs + cx(i)];
      }
  }
  if (nozzle_row(P, y) && (x == 0 || x == nx - 1)) {
#pragma unroll
    for (int l = 0; l < L; ++l) {
      Rng rng(node, l + 16, step);
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        if (x == 0 && cx(i) > 0) dst[(size_t)(l * Q + i) * n + node] = to_store<S, R>(P, l, i, P.inl[l][i], rng);
        if (x == nx - 1 && cx(i) < 0) dst[(size_t)(l * Q + i) * n + node] = to_store<S, R>(P, l, i, P.inl2[l][i], rng);
      }
    }
  }
}

// Open x ends, after the collision has streamed periodically into dst: what
// enters node x = 0 (c_x > 0) is the stored inlet equilibrium; what enters node
// x = nx - 1 (c_x < 0) comes from a ghost beyond it holding the boundary node's
// post-collision state, i.e. the value that node pushed into x = nx - 2 at the
// same (y, z). Reads x = nx - 2 and writes x = 0 and x = nx - 1 in disjoint
// directions (nx >= 2), so the nodes of a launch do not interfere.
template <typename S, typename R, int L>
__host__ __device__ __forceinline__ void open_fix_node(const Params<R>& P, S* __restrict__ dst, int64_t node,
                                              uint32_t step)
{
  const size_t n = (size_t)P.n;
  const uint32_t x = (uint32_t)node % (uint32_t)P.nx;
  if (x == 0) {
#pragma unroll
    for (int l = 0; l < L; ++l) {
      Rng rng(node, l + 16, step);
#pragma unroll
      for (int i = 0; i < Q; ++i)
        if (cx(i) > 0) dst[(size_t)(l * Q + i) * n + node] = to_store<S, R>(P, l, i, P.inl[l][i], rng);
    }
  }
  if (x == (uint32_t)P.nx - 1) {
#pragma unroll
    for (int l = 0; l < L; ++l)
#pragma unroll
      for (int i = 0; i < Q; ++i)
        if (cx(i) < 0) dst[(size_t)(l * Q + i) * n + node] = dst[(size_t)(l * Q + i) * n + node - 1];
  }
}

// --------------------------------------------------------------------------
// Collision of one lattice from its stored values v (already loaded), with the
// exact restoration of the lattice's conserved moments, then streaming. Shared
// by the three-pass step (collide_node) and the two-read step
// (state_species_node, fg_collide_node).
// --------------------------------------------------------------------------
// Precision of the small Stefan--Maxwell source F: FP64 with FP64 storage, else FP32.
template <typename S>
using SrcF = typename std::conditional<sizeof(S) == 8, double, float>::type;

// Face pairs (c = +e_k, -e_k) of the velocity set, k = x, y, z.
constexpr int face_plus(int k) { return k == 0 ? 22 : (k == 1 ? 16 : 14); }

// Store the six face populations of lattice l so that the stored first moment
// equals t1 (the momentum lattice: rho u + X): face holds their unrounded
// post-collision values (indexed by direction), s1 the first moment of the other
// stored values, s0 their sum (the faces' stored values are added to it). Each
// pair keeps its unrounded sum; the difference of the pair is what restores t1.
template <typename S, typename R>
__host__ __device__ __forceinline__ void restore_faces(const Params<R>& P, int l, const R (&face)[Q], const R (&t1)[3],
                                                       const R (&s1)[3], R& s0, S (&v)[Q], Rng& rng)
{
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int ip = face_plus(k), im = 26 - ip;
    const R sum = face[ip] + face[im];
    const R diff = t1[k] - s1[k];        // required stored value of ip minus that of im
    v[ip] = to_store<S, R>(P, l, ip, R(0.5) * (sum + diff), rng);
    v[im] = to_store<S, R>(P, l, im, R(0.5) * (sum - diff), rng);
    s0 += from_store<S, R>(P, l, ip, v[ip]) + from_store<S, R>(P, l, im, v[im]);
  }
}

// Species lattice a: f' = f + 2 beta (f^eq - f) + (beta - 1) F (eq SMlbm),
// F_ai = sum_b K_ab [Psi_i(u, R_b T) - Psi_i(u + V_b, R_b T)] (eq fstar1), with
// K_ab = P X_a X_b / D_ab, 1/tau_a = sum_b Y_b / tau_ab (eqs tauab, tau). us is
// the velocity the species see, pe the triplets of Psi(us, R_c T) and pd those
// of Psi(us) - Psi(us + V_c) (FP32 unless the storage is FP64: F is a small
// correction); gD the factor (T_ref / T)^s_D of temperature-dependent transport
// (1 otherwise).
template <typename S, typename R, int M, int BC, bool CVT>
__host__ __device__ __forceinline__ void species_relax(const Params<R>& P, const Mix<R, M>& s, const R (&K)[M][M],
                                                       const Trip<SrcF<S>> (&pe)[M][3],
                                                       const Trip<SrcF<S>> (&pd)[M][3], const R (&us)[3], R gD,
                                                       int a, S (&v)[Q], S* __restrict__ dst, const Nbr& b,
                                                       int64_t node, uint32_t step)
{
  using F32 = SrcF<S>;
  R acc = R(0);
#pragma unroll
  for (int c = 0; c < M; ++c) acc += s.Y[c] * P.invD[a][c] * P.inv_m[c];
  R inv_tau = s.T * s.mmix * P.inv_m[a] * acc;
  if constexpr (CVT) inv_tau *= gD;
  const R beta = inv_tau / (R(2) + inv_tau);            // dt / (2 tau_a + dt)
  Trip<R> pa[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) pa[k] = psi_trip<R>(us[k], s.T * P.inv_m[a]);
  R t0 = R(0), s0 = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) t0 += from_store<S, R>(P, a, i, v[i]);
  Rng rng(node, a, step);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (i == 13) continue;
    F32 F = F32(0);
#pragma unroll
    for (int c = 0; c < M; ++c) {
      const F32 ex = pe[c][0](cx(i)), ey = pe[c][1](cy(i)), ez = pe[c][2](cz(i));
      const F32 dx = pd[c][0](cx(i)), dy = pd[c][1](cy(i)), dz = pd[c][2](cz(i));
      F += F32(K[a][c]) * (dx * ey * ez + (ex - dx) * dy * ez + (ex - dx) * (ey - dy) * dz);
    }
    const R fe = s.rho_a[a] * (pa[0](cx(i)) * pa[1](cy(i)) * pa[2](cz(i))) - P.ref[a][crep(i)];
    // f' - f_ref = (f^eq - f_ref) + (1 - 2 beta)(f - f^eq) + (beta - 1) F
    const R dn = fe + (R(1) - R(2) * beta) * (from_store<S, R>(P, a, i, v[i]) - fe) + (beta - R(1)) * R(F);
    v[i] = to_store<S, R>(P, a, i, dn, rng);
    s0 += from_store<S, R>(P, a, i, v[i]);
  }
  // the collision conserves rho_a: the rest population takes the defect of
  // the arithmetic and of the other 26 values' rounding to storage
  v[13] = to_store<S, R>(P, a, 13, t0 - s0, rng);
#pragma unroll
  for (int i = 0; i < Q; ++i) push<S, R, BC>(P, dst, b, a, i, node, v[i]);
  range_check<S, R>(P, rng);
}

// Momentum lattice (stored lattice LF): f' = f + omega (f^eq - f) + A_i . X
// (eqs feq, fwithcorrection, Ai) at the node's rho, u and theta = R T; Xc is the
// isotropy correction X_a = -d_a G_a (eq Xalpha). The rounding defect of mass and
// momentum goes to the rest and face populations, which carry no other moment up
// to second order.
template <typename S, typename R, int BC>
__host__ __device__ __forceinline__ void momentum_relax(const Params<R>& P, int LF, R rho, const R (&u)[3], R theta,
                                                        R omega, const R (&Xc)[3], S (&v)[Q], S* __restrict__ dst,
                                                        const Nbr& b, int64_t node, uint32_t step)
{
  Trip<R> pf[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) pf[k] = psi_trip<R>(u[k], theta);
  R t0 = R(0), t1[3] = {R(0), R(0), R(0)}, s0 = R(0), s1[3] = {R(0), R(0), R(0)};
  Rng rng(node, LF, step);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R d = from_store<S, R>(P, LF, i, v[i]);
    t0 += d;
    acc_c(t1[0], cx(i), d);
    acc_c(t1[1], cy(i), d);
    acc_c(t1[2], cz(i), d);
  }
  // the source A_i . X adds X to the momentum (A_i = c_i / 2 on the six faces)
#pragma unroll
  for (int k = 0; k < 3; ++k) t1[k] += Xc[k];
  // all but the rest and face populations: collide and round to storage
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (csq(i) <= 1) continue;
    const R fe = rho * (pf[0](cx(i)) * pf[1](cy(i)) * pf[2](cz(i))) - P.ref[LF][crep(i)];
    const R dn = fe + (R(1) - omega) * (from_store<S, R>(P, LF, i, v[i]) - fe);
    v[i] = to_store<S, R>(P, LF, i, dn, rng);
    const R d = from_store<S, R>(P, LF, i, v[i]);
    s0 += d;
    acc_c(s1[0], cx(i), d);
    acc_c(s1[1], cy(i), d);
    acc_c(s1[2], cz(i), d);
  }
  // the face pairs carry the momentum defect, the rest population the mass
  // defect: each face pair keeps its equilibrium-relaxed sum and takes the
  // difference that restores rho u + X exactly
  R face[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (csq(i) != 1) continue;
    const R fe = rho * (pf[0](cx(i)) * pf[1](cy(i)) * pf[2](cz(i))) - P.ref[LF][crep(i)];
    face[i] = fe + (R(1) - omega) * (from_store<S, R>(P, LF, i, v[i]) - fe);
  }
  restore_faces<S, R>(P, LF, face, t1, s1, s0, v, rng);
  v[13] = to_store<S, R>(P, LF, 13, t0 - s0, rng);
#pragma unroll
  for (int i = 0; i < Q; ++i) push<S, R, BC>(P, dst, b, LF, i, node, v[i]);
  range_check<S, R>(P, rng);
}

// Energy lattice (stored lattice LG), eq g in the form
// g' = g + omega (g^eq - g) + w_i c_i . dq / theta (eqs gieq, gistar), the exact
// rewrite of eqs g, gistar, gstareq1mom, interdiffusion and corrFourier that has
// no pole at omega = omega_1; dq = (omega - omega_1)(q - q^eq - u.(P - P^eq))
// + omega_1 rho sum_a H_a Y_a V_a + (2 - omega_1)/2 P sum_a H_a d Y_a is formed
// by the caller. H is the mixture enthalpy, theta = R T.
template <typename S, typename R, int BC>
__host__ __device__ __forceinline__ void energy_relax(const Params<R>& P, int LG, R rho, const R (&u)[3], R usq,
                                                      R theta, R H, R omega, const R (&dq)[3], S (&v)[Q],
                                                      S* __restrict__ dst, const Nbr& b, int64_t node, uint32_t step)
{
  const R hyd = H + R(0.5) * usq;
  const R inv_theta = R(1) / theta;
  const R rhoE = rho * (H - theta + R(0.5) * usq);   // rho (U + u^2/2), U = H - R T
  R qeq[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) qeq[k] = hyd * rho * u[k];
  // closed form of R^eq - rho E theta I for T_0 = 0: rho theta^2 I + kappa u u
  const R kappa = rho * (hyd + theta);
  const R rt2 = rho * theta * theta;
  const R zf = (R(1) - R(3) * theta) * R(0.5) * inv_theta;
  const R Z[3] = {zf * (rt2 + kappa * u[0] * u[0]), zf * (rt2 + kappa * u[1] * u[1]), zf * (rt2 + kappa * u[2] * u[2])};
  const Trip<R> wt = w_trip<R>(theta);
  const R h2 = R(0.5) * inv_theta * inv_theta;
  R t0 = R(0), s0 = R(0);
  Rng rng(node, LG, step);
#pragma unroll
  for (int i = 0; i < Q; ++i) t0 += from_store<S, R>(P, LG, i, v[i]);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (i == 13) continue;
    const R w = wt(cx(i)) * wt(cy(i)) * wt(cz(i));
    const R cu = R(cx(i)) * u[0] + R(cy(i)) * u[1] + R(cz(i)) * u[2];
    const R cqe = R(cx(i)) * qeq[0] + R(cy(i)) * qeq[1] + R(cz(i)) * qeq[2];
    const R cdq = R(cx(i)) * dq[0] + R(cy(i)) * dq[1] + R(cz(i)) * dq[2];
    R bz = R(0);
    if (csq(i) == 1) bz = -R(0.5) * (cx(i) ? Z[0] : (cy(i) ? Z[1] : Z[2]));
    const R ge = w * (rhoE + cqe * inv_theta +
                      (rt2 * (R(csq(i)) - R(3) * theta) + kappa * (cu * cu - theta * usq)) * h2) + bz -
                 P.ref[LG][crep(i)];
    const R dn = ge + (R(1) - omega) * (from_store<S, R>(P, LG, i, v[i]) - ge) + w * cdq * inv_theta;
    v[i] = to_store<S, R>(P, LG, i, dn, rng);
    s0 += from_store<S, R>(P, LG, i, v[i]);
  }
  // the collision conserves rho E: the rest population takes the defect
  v[13] = to_store<S, R>(P, LG, 13, t0 - s0, rng);
#pragma unroll
  for (int i = 0; i < Q; ++i) push<S, R, BC>(P, dst, b, LG, i, node, v[i]);
  range_check<S, R>(P, rng);
}

// Load the Q stored values of lattice l of a node (one at a time: each load is
// followed by its use).
template <typename S>
__host__ __device__ __forceinline__ void load_lattice_seq(const S* __restrict__ lat, size_t n, uint32_t node, S (&v)[Q])
{
#pragma unroll
  for (int i = 0; i < Q; ++i) v[i] = buf_load<S, BUF_NT>(lat + (size_t)i * n, (uint32_t)n, node);
}

// --------------------------------------------------------------------------
// Pass 3 of the three-pass step: collide every lattice from the node record and
// push (stream) to the other buffer. PART selects the lattices: 0 all, 1 the
// stored species lattices, 2 the momentum and energy lattices (a split collision
// in two launches computes the same step).
// --------------------------------------------------------------------------
template <typename S, typename R, typename Rec, int M, int BC, int PART = 0, bool WEAK = false, bool CVT = false>
__host__ __device__ __forceinline__ void collide_node(const Params<R>& P, const S* __restrict__ src,
                                             S* __restrict__ dst, const Rec* __restrict__ rec,
                                             const Rec* __restrict__ G, int64_t node, uint32_t step)
{
  const size_t n = (size_t)P.n;
  constexpr int NS = Lat<M, WEAK>::NS, LF = Lat<M, WEAK>::LF, LG = Lat<M, WEAK>::LG;
  using RL = RecLayout<M, WEAK, CVT>;
  // issue a lattice's loads together (load_lattice) where the scheduler otherwise
  // serialises them: 16-bit storage, and the unsplit collision of three or more
  // species (one wave per SIMD, registers to spare); elsewhere each load is
  // followed by its use
  constexpr bool GROUP_LOADS = sizeof(S) == 2 || (PART == 0 && M >= 3);
  const Nbr b = neighbours(P, node);
  auto get = [&](int f) -> R { return R(*at32(rec + (size_t)f * n, (uint32_t)node)); };
  auto load = [&](int l, S (&v)[Q]) {
    if constexpr (GROUP_LOADS) load_lattice(src + (size_t)l * Q * n, n, (uint32_t)node, v);
    else load_lattice_seq(src + (size_t)l * Q * n, n, (uint32_t)node, v);
  };

  // ---- node state from the record
  const R rho = get(REC_RHO);
  R rho_s[M];
#pragma unroll
  for (int a = 0; a < NS; ++a) rho_s[a] = get(REC_RHOA + a);
  if constexpr (!WEAK) rho_s[M - 1] = R(0);
  Mix<R, M> s;
  R rs = rho;                     // the species subsystem's density
  {
    s.rho = rho;
    s.inv_rho = R(1) / rho;
    s.usq = R(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      s.u[k] = get(REC_UX + k);
      s.usq += s.u[k] * s.u[k];
    }
    R inv_rs = s.inv_rho;
    if constexpr (WEAK) {
      rs = R(0);
#pragma unroll
      for (int a = 0; a < M; ++a) {
        s.rho_a[a] = rho_s[a];
        rs += rho_s[a];
      }
      inv_rs = R(1) / rs;
    } else {
      R deficit = rho;
#pragma unroll
      for (int a = 0; a < M - 1; ++a) {
        s.rho_a[a] = rho_s[a];
        deficit -= rho_s[a];
      }
      s.rho_a[M - 1] = deficit;
    }
    R inv_m = R(0), Cp = R(0);
#pragma unroll
    for (int a = 0; a < M; ++a) {
      s.Y[a] = s.rho_a[a] * inv_rs;
      inv_m += s.Y[a] * P.inv_m[a];
      Cp += s.Y[a] * P.cp[a];
    }
    s.Rg = inv_m;
    s.mmix = R(1) / inv_m;
#pragma unroll
    for (int a = 0; a < M; ++a) s.X[a] = s.Y[a] * s.mmix * P.inv_m[a];
    s.Cp = Cp;
    s.T = get(REC_T);
    s.P = rho * s.Rg * s.T;
  }
  const R theta = s.Rg * s.T;
  const R omega = get(REC_OMEGA);
  const R omega1 = get(REC_OMEGA1);

  // ---- non-local terms: X_a = -d_a G_a (eq Xalpha) and d_a C_p (sum_a H_a d Y_a = T d C_p);
  // with C_v(T), the gradients of Y_a, a < M-1 (sum_a d Y_a = 0 gives the last)
  R dG[3] = {R(0), R(0), R(0)}, gcp[3] = {R(0), R(0), R(0)};
  R gY[CVT ? M - 1 : 1][3] = {};
  if constexpr (PART != 1) {
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (csq(i) == 0) continue;
    const uint32_t nb = stencil_index<BC>(b, cx(i), cy(i), cz(i));
    const R w3 = R(3.0 * w13(i));
    if constexpr (CVT) {
#pragma unroll
      for (int a = 0; a < M - 1; ++a) {
        const R yn = w3 * R(*at32(rec + (size_t)(RL::YF + a) * n, nb));
        acc_c(gY[a][0], cx(i), yn);
        acc_c(gY[a][1], cy(i), yn);
        acc_c(gY[a][2], cz(i), yn);
      }
    } else {
      const R cpn = w3 * R(*at32(rec + (size_t)REC_CP * n, nb));
      acc_c(gcp[0], cx(i), cpn);
      acc_c(gcp[1], cy(i), cpn);
      acc_c(gcp[2], cz(i), cpn);
    }
    if (cx(i)) acc_c(dG[0], cx(i), w3 * R(*at32(G, nb)));
    if (cy(i)) acc_c(dG[1], cy(i), w3 * R(*at32(G + n, nb)));
    if (cz(i)) acc_c(dG[2], cz(i), w3 * R(*at32(G + 2 * n, nb)));
  }
  }
  const R Xc[3] = {-dG[0], -dG[1], -dG[2]};

  // ---- species lattices (eqs SMlbm, fstar1)
  if constexpr (PART != 2) {
    // velocity and pressure of the species subsystem: the mixture's under strong
    // coupling; u_s (eq uSPEC) and the Dalton pressure under weak coupling
    R us[3] = {s.u[0], s.u[1], s.u[2]};
    R Pk = s.P;
    if constexpr (WEAK) {
#pragma unroll
      for (int k = 0; k < 3; ++k) us[k] = get(RL::US + k);
      Pk = rs * s.Rg * s.T;
    }
    bool present[M];
    species_present<R, M>(P, s.rho_a, s.rho, present);
    R K[M][M];
    R gD = R(1);                       // (T_ref / T)^s_D with temperature-dependent transport
    if constexpr (CVT) {
      gD = inv_diffusivity_factor<R>(P, s.T);
      Pk *= gD;
    }
    friction_matrix<R, M>(P, s, Pk, present, K);
      Trip<SrcF<S>> pe[M][3], pd[M][3];
#pragma unroll
    for (int c = 0; c < M; ++c) {
      const SrcF<S> zeta = SrcF<S>(s.T * P.inv_m[c]);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        pe[c][k] = psi_trip<SrcF<S>>(SrcF<S>(us[k]), zeta);
        pd[c][k] = psi_diff_trip<SrcF<S>>(SrcF<S>(us[k]), SrcF<S>(get(RL::V + 3 * c + k)));
      }
    }
#pragma unroll
    for (int a = 0; a < NS; ++a) {
      S v[Q];
      load(a, v);
      species_relax<S, R, M, BC, CVT>(P, s, K, pe, pd, us, gD, a, v, dst, b, node, step);
      lattice_barrier();
    }
  }

  // ---- momentum lattice
  if constexpr (PART != 1) {
    S v[Q];
    load(LF, v);
    momentum_relax<S, R, BC>(P, LF, rho, s.u, theta, omega, Xc, v, dst, b, node, step);
    lattice_barrier();
  }

  // ---- energy lattice: dq from the record's non-equilibrium flux, the diffusion
  // velocities and the enthalpy-weighted composition gradients
  if constexpr (PART != 1) {
    R H = s.Cp * s.T;
    R ha[CVT ? M : 1];                 // with C_v(T): H_a(T) = U_a(T) + R_a T (eq specHa)
    if constexpr (CVT) {
      H = R(0);
#pragma unroll
      for (int a = 0; a < M; ++a) {
        ha[a] = poly_U<R>(P.cvc[a], s.T) + s.T * P.inv_m[a];
        H += s.Y[a] * ha[a];
      }
    }
    R dq[3];
    R hyv[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int a = 0; a < M; ++a) {
      R ca;
      if constexpr (CVT) ca = ha[a] * s.Y[a];
      else ca = P.cp[a] * s.Y[a];
#pragma unroll
      for (int k = 0; k < 3; ++k) hyv[k] += ca * get(RL::V + 3 * a + k);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if constexpr (CVT) {
        // sum_a H_a d Y_a = sum_{a < M-1} (H_a - H_M) d Y_a
        R hgy = R(0);
#pragma unroll
        for (int a = 0; a < M - 1; ++a) hgy += (ha[a] - ha[M - 1]) * gY[a][k];
        dq[k] = (omega - omega1) * get(REC_QNX + k) + omega1 * rho * hyv[k] +
                R(0.5) * (R(2) - omega1) * s.P * hgy;
      } else {
        dq[k] = (omega - omega1) * get(REC_QNX + k) + omega1 * rho * s.T * hyv[k] +
                R(0.5) * (R(2) - omega1) * s.P * s.T * gcp[k];
      }
    }
    S v[Q];
    load(LG, v);
    energy_relax<S, R, BC>(P, LG, rho, s.u, s.usq, theta, H, omega, dq, v, dst, b, node, step);
  }
}

// --------------------------------------------------------------------------
// The two-read step. The species collisions are local: they use only the node's
// own moments (eqs SMlbm, fstar1, transform12). So the moments pass collides and
// streams the species lattices from the values it has just read, and only the
// momentum and energy lattices, whose collisions need the neighbours' moments
// of the same time level (eqs Xalpha, corrFourier), are read a second time:
//   state_species_node  every lattice's moments -> node record (Phi, omega, C_p
//                       for the stencils; omega_1, R, sum_a C_{a,p} Y_a V_a for
//                       the second pass); species collisions and streaming
//   gfield_node         G_a = (1/omega - 1/2) d_a Phi_a (unchanged)
//   fg_collide_node     re-reads f and g, forms rho, u, T, P and q from them,
//                       collides and streams both lattices
// Constant specific heats only (the temperature needs C_v = C_p - R).
// --------------------------------------------------------------------------
enum {
  REC2_OMEGA1 = 5, REC2_RG = 6,   // omega_1 (eq omega1), mixture gas constant R
  REC2_HYV = 7,                   // sum_a C_{a,p} Y_a V_a (3): the interdiffusion flux of eq interdiffusion over T
  REC2_FIELDS = 10
};

template <typename S, typename R, typename Rec, int M, int BC, bool WEAK = false>
__host__ __device__ __forceinline__ void state_species_node(const Params<R>& P, const S* __restrict__ src,
                                                            S* __restrict__ dst, Rec* __restrict__ rec,
                                                            int64_t node, uint32_t step)
{
  const size_t n = (size_t)P.n;
  const uint32_t nd = (uint32_t)node;
  constexpr int NS = Lat<M, WEAK>::NS, LF = Lat<M, WEAK>::LF, LG = Lat<M, WEAK>::LG;
  // species lattices: kept in registers for their collision below when there is
  // one (binary, strong coupling); with more, the state's registers are needed
  // for the larger Stefan--Maxwell system, and the values are read again for the
  // collision (the first read is a cached load, so the second mostly hits L2)
  constexpr bool HOLD = NS == 1;
  S vs[HOLD ? NS : 1][Q];
  R rho_s[M], js[M][3];
#pragma unroll
  for (int a = 0; a < NS; ++a) {
    S (&va)[Q] = vs[HOLD ? a : 0];
    if constexpr (HOLD) load_lattice(src + (size_t)a * Q * n, n, nd, va);
    else
#pragma unroll
      for (int i = 0; i < Q; ++i) va[i] = buf_load<S>(src + (size_t)(a * Q + i) * n, (uint32_t)n, nd);
    R r = R(0), ja[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R d = from_store<S, R>(P, a, i, va[i]);
      r += d;
      acc_c(ja[0], cx(i), d);
      acc_c(ja[1], cy(i), d);
      acc_c(ja[2], cz(i), d);
    }
    rho_s[a] = P.ref0[a] + r;
#pragma unroll
    for (int k = 0; k < 3; ++k) js[a][k] = ja[k];
  }
  if constexpr (!WEAK) rho_s[M - 1] = R(0);
  // mixture moments: rho, rho u (momentum lattice) and rho E (energy lattice)
  R rho = R(0), j[3] = {R(0), R(0), R(0)}, rhoE = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R d = from_store<S, R>(P, LF, i, buf_load<S, BUF_NT>(src + (size_t)(LF * Q + i) * n, (uint32_t)n, nd));
    rho += d;
    acc_c(j[0], cx(i), d);
    acc_c(j[1], cy(i), d);
    acc_c(j[2], cz(i), d);
    rhoE += from_store<S, R>(P, LG, i, buf_load<S, BUF_NT>(src + (size_t)(LG * Q + i) * n, (uint32_t)n, nd));
  }
  rho += P.ref0[LF];
  rhoE += P.ref0[LG];
  Mix<R, M> s;
  mixture_state<R, M, WEAK, false>(P, rho, j, rhoE, rho_s, s);
  R us[3], Pk = s.P;                     // velocity and pressure of the species subsystem
  if constexpr (WEAK) {
    R rs = R(0);
#pragma unroll
    for (int a = 0; a < M; ++a) rs += s.rho_a[a];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      R jt = R(0);
#pragma unroll
      for (int a = 0; a < M; ++a) jt += js[a][k];
      us[k] = jt / rs;                   // eq uSPEC
    }
    Pk = rs * s.Rg * s.T;                // Dalton: sum_a rho_a R_a T
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) {        // slaved species momentum: the deficit (eq uMATCH)
      R jm = j[k];
#pragma unroll
      for (int a = 0; a < M - 1; ++a) jm -= js[a][k];
      js[M - 1][k] = jm;
      us[k] = s.u[k];
    }
  }
  bool present[M];
  species_present<R, M>(P, s.rho_a, s.rho, present);
  R K[M][M], V[M][3];
  friction_matrix<R, M>(P, s, Pk, present, K);
  diffusion_velocities<R, M>(s, present, K, js, us, V);
  const R theta = s.Rg * s.T;
  const R mu_mix = mixture_viscosity<R, M>(P, s.X);
  const R lam_mix = mixture_conductivity<R, M>(P, s.X);
  const R omega = R(2) * s.P / (s.P + R(2) * mu_mix);
  const R omega1 = R(2) * s.P * s.Cp / (s.P * s.Cp + R(2) * lam_mix);
  auto put = [&](int f, R v) { buf_store<Rec, BUF_NT>(rec + (size_t)f * n, (uint32_t)n, nd, Rec(v)); };
#pragma unroll
  for (int k = 0; k < 3; ++k) put(REC_PHIX + k, j[k] * (R(1) - R(3) * theta) - j[k] * s.u[k] * s.u[k]);
  put(REC_OMEGA, omega);
  put(REC_CP, s.Cp);
  put(REC2_OMEGA1, omega1);
  put(REC2_RG, s.Rg);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    R h = R(0);
#pragma unroll
    for (int a = 0; a < M; ++a) h += P.cp[a] * s.Y[a] * V[a][k];
    put(REC2_HYV + k, h);
  }
  // species collisions and streaming
  Trip<SrcF<S>> pe[M][3], pd[M][3];
#pragma unroll
  for (int c = 0; c < M; ++c) {
    const SrcF<S> zeta = SrcF<S>(s.T * P.inv_m[c]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      pe[c][k] = psi_trip<SrcF<S>>(SrcF<S>(us[k]), zeta);
      pd[c][k] = psi_diff_trip<SrcF<S>>(SrcF<S>(us[k]), SrcF<S>(V[c][k]));
    }
  }
  const Nbr b = neighbours(P, node);
#pragma unroll
  for (int a = 0; a < NS; ++a) {
    S (&va)[Q] = vs[HOLD ? a : 0];
    if constexpr (!HOLD) load_lattice(src + (size_t)a * Q * n, n, nd, va);
    species_relax<S, R, M, BC, false>(P, s, K, pe, pd, us, R(1), a, va, dst, b, node, step);
    lattice_barrier();
  }
}

template <typename S, typename R, typename Rec, int M, int BC, bool WEAK = false>
__host__ __device__ __forceinline__ void fg_collide_node(const Params<R>& P, const S* __restrict__ src,
                                                         S* __restrict__ dst, const Rec* __restrict__ rec,
                                                         const Rec* __restrict__ G, int64_t node, uint32_t step)
{
  const size_t n = (size_t)P.n;
  const uint32_t nd = (uint32_t)node;
  constexpr int LF = Lat<M, WEAK>::LF, LG = Lat<M, WEAK>::LG;
  S vf[Q], vg[Q];
  load_lattice(src + (size_t)LF * Q * n, n, nd, vf);
  load_lattice(src + (size_t)LG * Q * n, n, nd, vg);
  // moments: rho, rho u, the pressure tensor sum_i f_i c_i c_i, rho E and q
  R rho = R(0), j[3] = {R(0), R(0), R(0)}, Pd[3] = {R(0), R(0), R(0)}, Pxy = R(0), Pxz = R(0), Pyz = R(0);
  R rhoE = R(0), q[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R d = from_store<S, R>(P, LF, i, vf[i]);
    rho += d;
    acc_c(j[0], cx(i), d);
    acc_c(j[1], cy(i), d);
    acc_c(j[2], cz(i), d);
    if (cx(i)) Pd[0] += d;
    if (cy(i)) Pd[1] += d;
    if (cz(i)) Pd[2] += d;
    acc_c(Pxy, cx(i) * cy(i), d);
    acc_c(Pxz, cx(i) * cz(i), d);
    acc_c(Pyz, cy(i) * cz(i), d);
    const R e = from_store<S, R>(P, LG, i, vg[i]);
    rhoE += e;
    acc_c(q[0], cx(i), e);
    acc_c(q[1], cy(i), e);
    acc_c(q[2], cz(i), e);
  }
  rho += P.ref0[LF];
  rhoE += P.ref0[LG];
#pragma unroll
  for (int k = 0; k < 3; ++k) Pd[k] += P.ref2[LF][k];
  auto get = [&](int f) -> R { return R(*at32(rec + (size_t)f * n, nd)); };
  const R omega = get(REC_OMEGA), omega1 = get(REC2_OMEGA1), Cp = get(REC_CP), Rg = get(REC2_RG);
  const R inv_rho = R(1) / rho;
  R u[3], usq = R(0);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    u[k] = j[k] * inv_rho;
    usq += u[k] * u[k];
  }
  const R T = (rhoE * inv_rho - R(0.5) * usq) / (Cp - Rg);   // eq temperature2, C_v = C_p - R
  const R theta = Rg * T;
  const R Pp = rho * Rg * T;
  // non-local terms: X_a = -d_a G_a (eq Xalpha) and d C_p (sum_a H_a d Y_a = T d C_p)
  const Nbr b = neighbours(P, node);
  R dG[3] = {R(0), R(0), R(0)}, gcp[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (csq(i) == 0) continue;
    const uint32_t nb = stencil_index<BC>(b, cx(i), cy(i), cz(i));
    const R w3 = R(3.0 * w13(i));
    const R cpn = w3 * R(*at32(rec + (size_t)REC_CP * n, nb));
    acc_c(gcp[0], cx(i), cpn);
    acc_c(gcp[1], cy(i), cpn);
    acc_c(gcp[2], cz(i), cpn);
    if (cx(i)) acc_c(dG[0], cx(i), w3 * R(*at32(G, nb)));
    if (cy(i)) acc_c(dG[1], cy(i), w3 * R(*at32(G + n, nb)));
    if (cz(i)) acc_c(dG[2], cz(i), w3 * R(*at32(G + 2 * n, nb)));
  }
  const R Xc[3] = {-dG[0], -dG[1], -dG[2]};
  // energy source: the non-equilibrium flux q - q^eq - u.(P - P^eq) of this node
  const R H = Cp * T;
  const R hyd = H + R(0.5) * usq;
  const R Pn[3][3] = {{Pd[0], Pxy, Pxz}, {Pxy, Pd[1], Pyz}, {Pxz, Pyz, Pd[2]}};
  R dq[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    R up = R(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) up += u[c] * (Pn[c][k] - (c == k ? Pp : R(0)) - rho * u[c] * u[k]);
    const R qn = q[k] - hyd * rho * u[k] - up;
    dq[k] = (omega - omega1) * qn + omega1 * rho * T * get(REC2_HYV + k) + R(0.5) * (R(2) - omega1) * Pp * T * gcp[k];
  }
  momentum_relax<S, R, BC>(P, LF, rho, u, theta, omega, Xc, vf, dst, b, node, step);
  lattice_barrier();
  energy_relax<S, R, BC>(P, LG, rho, u, usq, theta, H, omega, dq, vg, dst, b, node, step);
}

// --------------------------------------------------------------------------
// Read-back of the macroscopic fields
// --------------------------------------------------------------------------
template <typename S, typename R, int M, bool WEAK = false, bool CVT = false>
__host__ __device__ __forceinline__ void read_node(const Params<R>& P, const S* __restrict__ pop, int64_t node,
                                          double* X, double* rho_o, double* u, double* p, double* T)
{
  const size_t n = (size_t)P.n;
  constexpr int NS = Lat<M, WEAK>::NS, LF = Lat<M, WEAK>::LF, LG = Lat<M, WEAK>::LG;
  R rho_s[M];
#pragma unroll
  for (int a = 0; a < NS; ++a) {
    R sum = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) sum += load_dev<S, R>(pop, (size_t)(a * Q + i) * n + node, dec_scale<S>(P, a, i));
    rho_s[a] = P.ref0[a] + sum;
  }
  if constexpr (!WEAK) rho_s[M - 1] = R(0);
  R rho = R(0), j[3] = {R(0), R(0), R(0)}, rhoE = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R d = load_dev<S, R>(pop, (size_t)(LF * Q + i) * n + node, dec_scale<S>(P, LF, i));
    rho += d;
    if (cx(i)) j[0] += cx(i) > 0 ? d : -d;
    if (cy(i)) j[1] += cy(i) > 0 ? d : -d;
    if (cz(i)) j[2] += cz(i) > 0 ? d : -d;
    rhoE += load_dev<S, R>(pop, (size_t)(LG * Q + i) * n + node, dec_scale<S>(P, LG, i));
  }
  rho += P.ref0[LF];
  rhoE += P.ref0[LG];
  Mix<R, M> s;
  mixture_state<R, M, WEAK, CVT>(P, rho, j, rhoE, rho_s, s);
  if (X)
#pragma unroll
    for (int a = 0; a < M; ++a) X[(size_t)P.xperm[a] * n + node] = (double)s.X[a];
  if (rho_o) rho_o[node] = (double)s.rho;
  if (u)
#pragma unroll
    for (int k = 0; k < 3; ++k) u[(size_t)k * n + node] = (double)s.u[k];
  if (p) p[node] = (double)s.P;
  if (T) T[node] = (double)s.T;
}

// --------------------------------------------------------------------------
// Initialisation at the local equilibrium of (X_a, p, T, u), computed in FP64
// --------------------------------------------------------------------------
template <typename S, int M, bool WEAK = false, bool CVT = false>
__host__ __device__ __forceinline__ int init_node(const Params<double>& P, const double* X,
                                         const double* p, const double* T, const double* u, S* __restrict__ pop,
                                         int64_t node)
{
  const size_t n = (size_t)P.n;
  constexpr int NS = Lat<M, WEAK>::NS, LF = Lat<M, WEAK>::LF, LG = Lat<M, WEAK>::LG;
  double Xa[M], mmix = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    Xa[a] = X[(size_t)P.xperm[a] * n + node];
    mmix += Xa[a] * P.m[a];
  }
  const double Tn = T[node], pn = p[node];
  const double uu[3] = {u[node], u[n + node], u[2 * n + node]};
  const double usq = uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2];
  const double Rg = 1.0 / mmix;
  const double rho = pn / (Rg * Tn);
  double Cv = 0.0, Cp = 0.0, Y[M];
#pragma unroll
  for (int a = 0; a < M; ++a) {
    Y[a] = Xa[a] * P.m[a] / mmix;
    Cv += Y[a] * P.cv[a];
    Cp += Y[a] * P.cp[a];
  }
  int bad = (Tn > 0.0 && pn > 0.0) ? 0 : 1;
#pragma unroll
  for (int a = 0; a < NS; ++a) {
    const double zeta = Tn * P.inv_m[a];
    if (!(zeta + usq < 1.0)) bad = 1;
    Trip<double> t[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) t[k] = psi_trip<double>(uu[k], zeta);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double f = rho * Y[a] * (t[0](cx(i)) * t[1](cy(i)) * t[2](cz(i)));
      pop[(size_t)(a * Q + i) * n + node] = init_store<S>(P, a, i, f - P.ref[a][i]);
    }
  }
  const double theta = Rg * Tn;
  if (!(theta + usq < 1.0)) bad = 1;
  {
    Trip<double> t[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) t[k] = psi_trip<double>(uu[k], theta);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double f = rho * (t[0](cx(i)) * t[1](cy(i)) * t[2](cz(i)));
      pop[(size_t)(LF * Q + i) * n + node] = init_store<S>(P, LF, i, f - P.ref[LF][i]);
    }
  }
  {
    double U = Cv * Tn, H = Cp * Tn;        // specific internal energy and enthalpy
    if constexpr (CVT) {                     // eqs Umix, specH with C_v(T)
      double c[4];
      mix_cv_poly<double, M>(P, Y, c);
      U = poly_U<double>(c, Tn);
      H = U + Rg * Tn;
    }
    const double rhoE = rho * (U + 0.5 * usq);
    const double hyd = H + 0.5 * usq;
    const double kappa = rho * (hyd + theta);
    const double rt2 = rho * theta * theta;
    const double zf = (1.0 - 3.0 * theta) * 0.5 / theta;
    const double Z[3] = {zf * (rt2 + kappa * uu[0] * uu[0]), zf * (rt2 + kappa * uu[1] * uu[1]),
                         zf * (rt2 + kappa * uu[2] * uu[2])};
    const Trip<double> wt = w_trip<double>(theta);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double w = wt(cx(i)) * wt(cy(i)) * wt(cz(i));
      const double cu = cx(i) * uu[0] + cy(i) * uu[1] + cz(i) * uu[2];
      double bz = 0.0;
      if (csq(i) == 0) bz = Z[0] + Z[1] + Z[2];
      if (csq(i) == 1) bz = -0.5 * (cx(i) ? Z[0] : (cy(i) ? Z[1] : Z[2]));
      const double g = w * (rhoE + hyd * rho * cu / theta +
                            (rt2 * (csq(i) - 3.0 * theta) + kappa * (cu * cu - theta * usq)) * 0.5 / (theta * theta)) +
                       bz;
      pop[(size_t)(LG * Q + i) * n + node] = init_store<S>(P, LG, i, g - P.ref[LG][i]);
    }
  }
  return bad;
}

// --------------------------------------------------------------------------
// Conserved sums of a node in FP64: rho_1..rho_M (rho_M slaved under strong
// coupling, from its own lattice under weak), rho, rho u, rho E, plus a flag for
// non-finite values or a negative density of species M.
// --------------------------------------------------------------------------
template <typename S, int M, bool WEAK = false>
__host__ __device__ __forceinline__ void conserved_node(const Params<double>& P, const S* __restrict__ pop,
                                               int64_t node, double* out /*[M+6]*/)
{
  const size_t n = (size_t)P.n;
  constexpr int NS = Lat<M, WEAK>::NS, LF = Lat<M, WEAK>::LF, LG = Lat<M, WEAK>::LG;
  double rest = 0.0;
#pragma unroll
  for (int a = 0; a < NS; ++a) {
    double sum = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) sum += (double)pop[(size_t)(a * Q + i) * n + node] * dec_scale<S>(P, a, i);
    out[a] = P.ref0[a] + sum;
    rest += out[a];
  }
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0}, rhoE = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double d = (double)pop[(size_t)(LF * Q + i) * n + node] * dec_scale<S>(P, LF, i);
    rho += d;
    j[0] += cx(i) * d;
    j[1] += cy(i) * d;
    j[2] += cz(i) * d;
    rhoE += (double)pop[(size_t)(LG * Q + i) * n + node] * dec_scale<S>(P, LG, i);
  }
  rho += P.ref0[LF];
  rhoE += P.ref0[LG];
  if constexpr (!WEAK) out[M - 1] = rho - rest;
  out[M] = rho;
  out[M + 1] = j[0];
  out[M + 2] = j[1];
  out[M + 3] = j[2];
  out[M + 4] = rhoE;
  bool ok = out[M - 1] >= 0.0 && rho > 0.0;
#pragma unroll
  for (int k = 0; k < M + 5; ++k) ok = ok && (out[k] - out[k] == 0.0);
  out[M + 5] = ok ? 0.0 : 1.0;
}

// Moles of every species at a node, rho_a / m_a (R_U = 1; under strong coupling
// the slaved species from the deficit, eq rhoMATCH), in slot [h][a] of out[2 M], h = 0 for x < nx / 2 and
// h = 1 otherwise (the other half's slots zero): summed over a tube, the moles in
// each half of a Loschmidt tube, whose ratios are the half-tube mean mole
// fractions of Sec. 4.2.
template <typename S, int M, bool WEAK = false>
__host__ __device__ __forceinline__ void half_moles_node(const Params<double>& P, const S* __restrict__ pop,
                                                int64_t node, double* out /*[2 M]*/)
{
  const size_t n = (size_t)P.n;
  constexpr int NS = Lat<M, WEAK>::NS, LF = Lat<M, WEAK>::LF;
  double rho_a[M], rest = 0.0;
#pragma unroll
  for (int a = 0; a < NS; ++a) {
    double sum = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) sum += (double)pop[(size_t)(a * Q + i) * n + node] * dec_scale<S>(P, a, i);
    rho_a[a] = P.ref0[a] + sum;
    rest += rho_a[a];
  }
  if constexpr (!WEAK) {
    double rho = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) rho += (double)pop[(size_t)(LF * Q + i) * n + node] * dec_scale<S>(P, LF, i);
    rho_a[M - 1] = rho + P.ref0[LF] - rest;
  }
  const int h = (int)(node % P.nx) >= P.nx / 2 ? 1 : 0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    out[h * M + a] = rho_a[a] * P.inv_m[a];
    out[(1 - h) * M + a] = 0.0;
  }
}

}  // namespace mclbm
