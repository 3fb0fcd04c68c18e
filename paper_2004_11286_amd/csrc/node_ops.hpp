// node_ops.hpp -- per-node work of one time step of the M+2-lattice mixture
// lattice Boltzmann model (Sawant, Dorschner, Karlin, arXiv 2004.11286),
// written as inlined functions that the HIP kernels call once per lattice node.
//
// Storage: pop[l][i][n] with l = 0..M-2 the stored species (species M is slaved
// to the momentum lattice under strong coupling, Sec. 3.6.2, and no quantity
// ever reads its populations), l = M-1 the momentum lattice f, l = M the energy
// lattice g; n = x + nx (y + ny z). Stored values are d = s_l (f - f_ref,l,i).
//
// A step is three passes: moments_node writes a per-node record
// {Phi_x, Phi_y, Phi_z, omega, C_p}; gfield_node forms
// G_a = (1/omega - 1/2) d_a Phi_a; collide_node collides every lattice and
// pushes the post-collision values to their neighbours (streaming), bouncing
// them back at x walls.
#pragma once

#include "lattice.hpp"

namespace mclbm {

// Record layout (structure of arrays): rec[k * n + node].
enum { REC_PHIX = 0, REC_PHIY = 1, REC_PHIZ = 2, REC_OMEGA = 3, REC_CP = 4, REC_FIELDS = 5 };

// Macroscopic state of a node (Secs. 2.1, 3.1, 3.2; strong coupling Sec. 3.6.2).
template <typename R, int M>
struct Mix {
  R rho, inv_rho, u[3], usq, rhoE;
  R rho_a[M], Y[M], X[M];
  R mmix, Rg, Cv, Cp, T, P;
};

// rho_s[0..M-2]: stored species densities; the slaved species takes the deficit.
template <typename R, int M>
__host__ __device__ inline void mixture_state(const Params<R>& P, R rho, const R j[3], R rhoE,
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
  R deficit = rho;
#pragma unroll
  for (int a = 0; a < M - 1; ++a) {
    s.rho_a[a] = rho_s[a];
    deficit -= rho_s[a];
  }
  s.rho_a[M - 1] = deficit;
  R inv_m = R(0), Cv = R(0), Cp = R(0);
#pragma unroll
  for (int a = 0; a < M; ++a) {
    s.Y[a] = s.rho_a[a] * s.inv_rho;
    inv_m += s.Y[a] * P.inv_m[a];
    Cv += s.Y[a] * P.cv[a];
    Cp += s.Y[a] * P.cp[a];
  }
  s.Rg = inv_m;                      // R = R_U / m with R_U = 1
  s.mmix = R(1) / inv_m;
#pragma unroll
  for (int a = 0; a < M; ++a) s.X[a] = s.Y[a] * s.mmix * P.inv_m[a];
  s.Cv = Cv;
  s.Cp = Cp;
  s.T = (rhoE * s.inv_rho - R(0.5) * s.usq) / Cv;   // constant specific heats, T_0 = 0
  s.P = rho * s.Rg * s.T;
}

// Wilke's mixture viscosity and Mathur's mixture conductivity (Sec. 3.4).
template <typename R, int M>
__host__ __device__ inline R mixture_viscosity(const Params<R>& P, const R X[M])
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
__host__ __device__ inline R mixture_conductivity(const Params<R>& P, const R X[M])
{
  R lin = R(0), harm = R(0);
#pragma unroll
  for (int a = 0; a < M; ++a) {
    lin += X[a] * P.lam[a];
    harm += X[a] * P.inv_lam[a];
  }
  return R(0.5) * (lin + R(1) / harm);
}

template <typename S, typename R>
__host__ __device__ inline R load_dev(const S* __restrict__ p, size_t idx, R inv_scale)
{
  return R(p[idx]) * inv_scale;
}

// Neighbour offsets of a node: x positions, y and z strides, wrapped periodically.
struct Nbr {
  int64_t x[3], y[3], z[3];   // index contributions for c = -1, 0, +1
  bool lo, hi;                // node touches the x = 0 / x = nx-1 wall
};

template <typename R>
__host__ __device__ inline Nbr neighbours(const Params<R>& P, int64_t node)
{
  Nbr b;
  // node counts fit in 32 bits (checked at context creation): 32-bit division
  const uint32_t nx = (uint32_t)P.nx, ny = (uint32_t)P.ny, nz = (uint32_t)P.nz;
  const uint32_t nd = (uint32_t)node;
  const uint32_t x = nd % nx;
  const uint32_t t = nd / nx;
  const uint32_t y = t % ny;
  const uint32_t z = t / ny;
  const int64_t sy = nx, sz = (int64_t)nx * ny;
  b.x[0] = x == 0 ? nx - 1 : x - 1;
  b.x[1] = x;
  b.x[2] = x == nx - 1 ? 0 : x + 1;
  b.y[0] = (int64_t)(y == 0 ? ny - 1 : y - 1) * sy;
  b.y[1] = (int64_t)y * sy;
  b.y[2] = (int64_t)(y == ny - 1 ? 0 : y + 1) * sy;
  b.z[0] = (int64_t)(z == 0 ? nz - 1 : z - 1) * sz;
  b.z[1] = (int64_t)z * sz;
  b.z[2] = (int64_t)(z == nz - 1 ? 0 : z + 1) * sz;
  b.lo = x == 0;
  b.hi = x == nx - 1;
  return b;
}

// Stencil neighbour index: at an x wall the ghost node mirrors the boundary node.
template <bool WALLS>
__host__ __device__ inline int64_t stencil_index(const Nbr& b, int ci, int cj, int ck)
{
  int64_t xi = b.x[ci + 1];
  if (WALLS) {
    if (ci < 0 && b.lo) xi = b.x[1];
    if (ci > 0 && b.hi) xi = b.x[1];
  }
  return xi + b.y[cj + 1] + b.z[ck + 1];
}

template <bool WALLS>
__host__ __device__ inline bool is_ghost(const Nbr& b, int ci)
{
  return WALLS && ((ci < 0 && b.lo) || (ci > 0 && b.hi));
}

// --------------------------------------------------------------------------
// Pass 1: moments -> record {Phi, omega, C_p}
// --------------------------------------------------------------------------
template <typename S, typename R, int M>
__host__ __device__ inline void moments_node(const Params<R>& P, const S* __restrict__ pop,
                                             R* __restrict__ rec, int64_t node)
{
  const size_t n = (size_t)P.n;
  constexpr int LF = M - 1, LG = M;
  R rho_s[M];
#pragma unroll
  for (int a = 0; a < M - 1; ++a) {
    R sum = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) sum += load_dev<S, R>(pop, (size_t)(a * Q + i) * n + node, P.inv_scale[a]);
    rho_s[a] = P.ref0[a] + sum;
  }
  rho_s[M - 1] = R(0);
  R rho = R(0), j[3] = {R(0), R(0), R(0)}, rhoE = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    R d = load_dev<S, R>(pop, (size_t)(LF * Q + i) * n + node, P.inv_scale[LF]);
    rho += d;
    if (cx(i)) j[0] += cx(i) > 0 ? d : -d;
    if (cy(i)) j[1] += cy(i) > 0 ? d : -d;
    if (cz(i)) j[2] += cz(i) > 0 ? d : -d;
    rhoE += load_dev<S, R>(pop, (size_t)(LG * Q + i) * n + node, P.inv_scale[LG]);
  }
  rho += P.ref0[LF];
  rhoE += P.ref0[LG];
  Mix<R, M> s;
  mixture_state<R, M>(P, rho, j, rhoE, rho_s, s);
  R theta = s.Rg * s.T;
  R mu = mixture_viscosity<R, M>(P, s.X);
  R omega = R(2) * s.P / (s.P + R(2) * mu);
#pragma unroll
  for (int k = 0; k < 3; ++k)   // Phi_a = rho u_a (1 - 3 R T) - rho u_a^3 (eq Xalpha)
    rec[(size_t)k * n + node] = j[k] * (R(1) - R(3) * theta) - j[k] * s.u[k] * s.u[k];
  rec[(size_t)REC_OMEGA * n + node] = omega;
  rec[(size_t)REC_CP * n + node] = s.Cp;
}

// --------------------------------------------------------------------------
// Pass 2: G_a = (1/omega - 1/2) d_a Phi_a, with d_a = 3 sum_i w_i c_ia (.)(x + c_i)
// --------------------------------------------------------------------------
template <typename R, bool WALLS>
__host__ __device__ inline void gfield_node(const Params<R>& P, const R* __restrict__ rec,
                                            R* __restrict__ G, int64_t node)
{
  const size_t n = (size_t)P.n;
  Nbr b = neighbours(P, node);
  R dphi[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (csq(i) == 0) continue;
    int64_t nb = stencil_index<WALLS>(b, cx(i), cy(i), cz(i));
    const R w3 = R(3.0 * w13(i));
    if (cx(i)) {
      R v = rec[(size_t)REC_PHIX * n + nb];
      if (is_ghost<WALLS>(b, cx(i))) v = -v;        // Phi_x is odd under the wall mirror
      dphi[0] += cx(i) > 0 ? w3 * v : -(w3 * v);
    }
    if (cy(i)) {
      R v = rec[(size_t)REC_PHIY * n + nb];
      dphi[1] += cy(i) > 0 ? w3 * v : -(w3 * v);
    }
    if (cz(i)) {
      R v = rec[(size_t)REC_PHIZ * n + nb];
      dphi[2] += cz(i) > 0 ? w3 * v : -(w3 * v);
    }
  }
  R om = rec[(size_t)REC_OMEGA * n + node];
  R f = R(1) / om - R(0.5);
#pragma unroll
  for (int k = 0; k < 3; ++k) G[(size_t)k * n + node] = f * dphi[k];
}

// --------------------------------------------------------------------------
// Pass 3: collide every lattice and push (stream) to the other buffer
// --------------------------------------------------------------------------
template <typename S, typename R, bool WALLS>
__host__ __device__ inline void push(const Params<R>& P, S* __restrict__ dst, const Nbr& b, int l, int i,
                                     int64_t node, R dev)
{
  const size_t n = (size_t)P.n;
  S v = S(dev * P.scale[l]);
  if (WALLS && ((cx(i) < 0 && b.lo) || (cx(i) > 0 && b.hi))) {
    dst[(size_t)(l * Q + opp(i)) * n + node] = v;    // half-way bounce-back
  } else {
    int64_t d = b.x[cx(i) + 1] + b.y[cy(i) + 1] + b.z[cz(i) + 1];
    dst[(size_t)(l * Q + i) * n + d] = v;
  }
}

template <typename S, typename R, int M, bool WALLS>
__host__ __device__ inline void collide_node(const Params<R>& P, const S* __restrict__ src,
                                             S* __restrict__ dst, const R* __restrict__ rec,
                                             const R* __restrict__ G, int64_t node)
{
  const size_t n = (size_t)P.n;
  constexpr int LF = M - 1, LG = M;
  const Nbr b = neighbours(P, node);

  // ---- moments of the momentum and energy lattices
  R rho = R(0), j[3] = {R(0), R(0), R(0)}, Pf[3] = {R(0), R(0), R(0)}, Pxy = R(0), Pxz = R(0), Pyz = R(0);
  R rhoE = R(0), q[3] = {R(0), R(0), R(0)};
  R df[Q], dg[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    df[i] = load_dev<S, R>(src, (size_t)(LF * Q + i) * n + node, P.inv_scale[LF]);
    dg[i] = load_dev<S, R>(src, (size_t)(LG * Q + i) * n + node, P.inv_scale[LG]);
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R d = df[i];
    rho += d;
    if (cx(i)) { j[0] += cx(i) > 0 ? d : -d; Pf[0] += d; }
    if (cy(i)) { j[1] += cy(i) > 0 ? d : -d; Pf[1] += d; }
    if (cz(i)) { j[2] += cz(i) > 0 ? d : -d; Pf[2] += d; }
    if (cx(i) && cy(i)) Pxy += cx(i) * cy(i) > 0 ? d : -d;
    if (cx(i) && cz(i)) Pxz += cx(i) * cz(i) > 0 ? d : -d;
    if (cy(i) && cz(i)) Pyz += cy(i) * cz(i) > 0 ? d : -d;
    const R e = dg[i];
    rhoE += e;
    if (cx(i)) q[0] += cx(i) > 0 ? e : -e;
    if (cy(i)) q[1] += cy(i) > 0 ? e : -e;
    if (cz(i)) q[2] += cz(i) > 0 ? e : -e;
  }
  rho += P.ref0[LF];
  rhoE += P.ref0[LG];
#pragma unroll
  for (int k = 0; k < 3; ++k) Pf[k] += P.ref2[LF];

  // ---- species moments
  R ds[M > 1 ? M - 1 : 1][Q];
  R rho_s[M], js[M][3];
#pragma unroll
  for (int a = 0; a < M - 1; ++a) {
    R r = R(0), ja[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R d = load_dev<S, R>(src, (size_t)(a * Q + i) * n + node, P.inv_scale[a]);
      ds[a][i] = d;
      r += d;
      if (cx(i)) ja[0] += cx(i) > 0 ? d : -d;
      if (cy(i)) ja[1] += cy(i) > 0 ? d : -d;
      if (cz(i)) ja[2] += cz(i) > 0 ? d : -d;
    }
    rho_s[a] = P.ref0[a] + r;
#pragma unroll
    for (int k = 0; k < 3; ++k) js[a][k] = ja[k];
  }
  rho_s[M - 1] = R(0);
  Mix<R, M> s;
  mixture_state<R, M>(P, rho, j, rhoE, rho_s, s);
  // slaved species momentum is the deficit (eq uMATCH)
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    R jm = j[k];
#pragma unroll
    for (int a = 0; a < M - 1; ++a) jm -= js[a][k];
    js[M - 1][k] = jm;
  }
  const R theta = s.Rg * s.T;
  const R mu = mixture_viscosity<R, M>(P, s.X);
  const R lam = mixture_conductivity<R, M>(P, s.X);
  const R omega = R(2) * s.P / (s.P + R(2) * mu);
  const R omega1 = R(2) * s.P * s.Cp / (s.P * s.Cp + R(2) * lam);

  // ---- non-local terms: X_a = -d_a G_a and d_a C_p (sum_a H_a d Y_a = T d C_p)
  R Xc[3] = {R(0), R(0), R(0)}, gcp[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (csq(i) == 0) continue;
    const int64_t nb = stencil_index<WALLS>(b, cx(i), cy(i), cz(i));
    const R w3 = R(3.0 * w13(i));
    const R cpn = rec[(size_t)REC_CP * n + nb];
    if (cx(i)) {
      R g = G[nb];
      Xc[0] += cx(i) > 0 ? w3 * g : -(w3 * g);
      gcp[0] += cx(i) > 0 ? w3 * cpn : -(w3 * cpn);
    }
    if (cy(i)) {
      R g = G[n + nb];
      Xc[1] += cy(i) > 0 ? w3 * g : -(w3 * g);
      gcp[1] += cy(i) > 0 ? w3 * cpn : -(w3 * cpn);
    }
    if (cz(i)) {
      R g = G[2 * n + nb];
      Xc[2] += cz(i) > 0 ? w3 * g : -(w3 * g);
      gcp[2] += cz(i) > 0 ? w3 * cpn : -(w3 * cpn);
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) Xc[k] = -Xc[k];

  // ---- species: Stefan--Maxwell rates (eqs tauab, tau), K_ab = P X_a X_b / D_ab
  R K[M][M], beta[M];
#pragma unroll
  for (int a = 0; a < M; ++a) {
    R acc = R(0);
#pragma unroll
    for (int c = 0; c < M; ++c) {
      K[a][c] = s.P * s.X[a] * s.X[c] * P.invD[a][c];
      acc += s.Y[c] * P.invD[a][c] * P.inv_m[c];
    }
    const R inv_tau = s.T * s.mmix * P.inv_m[a] * acc;
    beta[a] = inv_tau / (R(2) + inv_tau);              // dt / (2 tau_a + dt)
  }
  // diffusion velocities: rho_a V_a + 1/2 sum_b K_ab (V_a - V_b) = j_a - rho_a u (eq transform12)
  R A[M][M], rhs[M][3], V[M][3];
#pragma unroll
  for (int a = 0; a < M; ++a) {
    R diag = s.rho_a[a];
#pragma unroll
    for (int c = 0; c < M; ++c) {
      if (c == a) continue;
      diag += R(0.5) * K[a][c];
      A[a][c] = -R(0.5) * K[a][c];
    }
    A[a][a] = diag;
#pragma unroll
    for (int k = 0; k < 3; ++k) rhs[a][k] = js[a][k] - s.rho_a[a] * s.u[k];
  }
  // Gaussian elimination without pivoting: the matrix is column diagonally
  // dominant wherever rho_a != 0; an absent species has a zero row and column.
  bool present[M];
#pragma unroll
  for (int c = 0; c < M; ++c) {
    const R piv = A[c][c];
    present[c] = piv > P.pivot_tiny || piv < -P.pivot_tiny;
    const R inv = present[c] ? R(1) / piv : R(0);
#pragma unroll
    for (int r = c + 1; r < M; ++r) {
      const R f = A[r][c] * inv;
#pragma unroll
      for (int cc2 = c + 1; cc2 < M; ++cc2) A[r][cc2] -= f * A[c][cc2];
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
      V[r][k] = present[r] ? acc / A[r][r] : R(0);
    }
  }

  // ---- species collision: f' = f + 2 beta (f^eq - f) + (beta - 1) F (eq SMlbm),
  // F_ai = sum_b K_ab [Psi_i(u, R_b T) - Psi_i(u + V_b, R_b T)] (eq fstar1)
  Trip<R> pe[M][3], pv[M][3], pd[M][3];
#pragma unroll
  for (int c = 0; c < M; ++c) {
    const R zeta = s.T * P.inv_m[c];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      pe[c][k] = psi_trip<R>(s.u[k], zeta);
      pv[c][k] = psi_trip<R>(s.u[k] + V[c][k], zeta);
      pd[c][k] = psi_diff_trip<R>(s.u[k], V[c][k]);
    }
  }
  // Non-equilibrium parts f - f^eq of every stored species. In finite precision
  // the rounded equilibria do not sum exactly to rho_a; that defect is taken out
  // of the rest population so that the collision conserves rho_a up to the
  // rounding of the (small) non-equilibrium part. The rest population carries
  // no first or second moment, so nothing else changes.
#pragma unroll
  for (int a = 0; a < M - 1; ++a) {
    R s0 = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R feq = s.rho_a[a] * (pe[a][0](cx(i)) * pe[a][1](cy(i)) * pe[a][2](cz(i)));
      ds[a][i] = ds[a][i] - (feq - P.ref[a][i]);   // now holds the deviation's non-equilibrium part
      s0 += ds[a][i];
    }
    ds[a][13] -= s0;
  }
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    R dpsi[M];
#pragma unroll
    for (int c = 0; c < M; ++c)
      dpsi[c] = pd[c][0](cx(i)) * pe[c][1](cy(i)) * pe[c][2](cz(i)) +
                pv[c][0](cx(i)) * pd[c][1](cy(i)) * pe[c][2](cz(i)) +
                pv[c][0](cx(i)) * pv[c][1](cy(i)) * pd[c][2](cz(i));
#pragma unroll
    for (int a = 0; a < M - 1; ++a) {
      R F = R(0);
#pragma unroll
      for (int c = 0; c < M; ++c) F += K[a][c] * dpsi[c];
      const R feq = s.rho_a[a] * (pe[a][0](cx(i)) * pe[a][1](cy(i)) * pe[a][2](cz(i)));
      const R neq = ds[a][i];
      // f' - f_ref = (f^eq - f_ref) + (1 - 2 beta)(f - f^eq) + (beta - 1) F
      const R dn = (feq - P.ref[a][i]) + (R(1) - R(2) * beta[a]) * neq + (beta[a] - R(1)) * F;
      push<S, R, WALLS>(P, dst, b, a, i, node, dn);
    }
  }

  // ---- momentum lattice: f' = f + omega (f^eq - f) + A_i . X (eqs fwithcorrection, Ai);
  // the rounding defect of the equilibrium's mass and momentum is moved onto the
  // rest and face populations (which carry no other moment up to second order).
  {
    Trip<R> pf[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) pf[k] = psi_trip<R>(s.u[k], theta);
    R fe[Q];
    R s0 = R(0), s1[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      fe[i] = rho * (pf[0](cx(i)) * pf[1](cy(i)) * pf[2](cz(i))) - P.ref[LF][i];
      df[i] = df[i] - fe[i];                      // non-equilibrium part
      s0 += df[i];
      if (cx(i)) s1[0] += cx(i) > 0 ? df[i] : -df[i];
      if (cy(i)) s1[1] += cy(i) > 0 ? df[i] : -df[i];
      if (cz(i)) s1[2] += cz(i) > 0 ? df[i] : -df[i];
    }
    df[13] -= s0;
    df[22] -= R(0.5) * s1[0]; df[4] += R(0.5) * s1[0];    // faces +-x
    df[16] -= R(0.5) * s1[1]; df[10] += R(0.5) * s1[1];   // faces +-y
    df[14] -= R(0.5) * s1[2]; df[12] += R(0.5) * s1[2];   // faces +-z
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      R dn = fe[i] + (R(1) - omega) * df[i];
      if (csq(i) == 1) {
        const R ax = cx(i) ? (cx(i) > 0 ? Xc[0] : -Xc[0]) : (cy(i) ? (cy(i) > 0 ? Xc[1] : -Xc[1])
                                                                   : (cz(i) > 0 ? Xc[2] : -Xc[2]));
        dn += R(0.5) * ax;
      }
      push<S, R, WALLS>(P, dst, b, LF, i, node, dn);
    }
  }

  // ---- energy lattice (eq g), in the form g' = g + omega (g^eq - g) + w_i c_i . dq / theta,
  // dq = (omega - omega_1)(q - q^eq - u.(P - P^eq)) + omega_1 rho sum_a H_a Y_a V_a
  //      + (2 - omega_1)/2 P sum_a H_a d Y_a
  {
    const R H = s.Cp * s.T;
    const R hyd = H + R(0.5) * s.usq;
    const R inv_theta = R(1) / theta;
    R qeq[3], dq[3];
    const R Pxx = Pf[0], Pyy = Pf[1], Pzz = Pf[2];
    const R Pn[3][3] = {{Pxx, Pxy, Pxz}, {Pxy, Pyy, Pyz}, {Pxz, Pyz, Pzz}};
    R hyv[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int a = 0; a < M; ++a) {
      const R ca = P.cp[a] * s.Y[a];
#pragma unroll
      for (int k = 0; k < 3; ++k) hyv[k] += ca * V[a][k];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      qeq[k] = hyd * rho * s.u[k];
      R up = R(0);
#pragma unroll
      for (int c = 0; c < 3; ++c) up += s.u[c] * (Pn[c][k] - (c == k ? s.P : R(0)) - rho * s.u[c] * s.u[k]);
      dq[k] = (omega - omega1) * (q[k] - qeq[k] - up) + omega1 * rho * s.T * hyv[k] +
              R(0.5) * (R(2) - omega1) * s.P * s.T * gcp[k];
    }
    // closed form of R^eq - rho E theta I for T_0 = 0: rho theta^2 I + kappa u u
    const R kappa = rho * (hyd + theta);
    const R rt2 = rho * theta * theta;
    const R zf = (R(1) - R(3) * theta) * R(0.5) * inv_theta;
    const R Z[3] = {zf * (rt2 + kappa * s.u[0] * s.u[0]), zf * (rt2 + kappa * s.u[1] * s.u[1]),
                    zf * (rt2 + kappa * s.u[2] * s.u[2])};
    const Trip<R> wt = w_trip<R>(theta);
    const R h2 = R(0.5) * inv_theta * inv_theta;
    R ge[Q];
    R s0 = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R w = wt(cx(i)) * wt(cy(i)) * wt(cz(i));
      const R cu = R(cx(i)) * s.u[0] + R(cy(i)) * s.u[1] + R(cz(i)) * s.u[2];
      const R cqe = R(cx(i)) * qeq[0] + R(cy(i)) * qeq[1] + R(cz(i)) * qeq[2];
      R bz = R(0);
      if (csq(i) == 0) bz = Z[0] + Z[1] + Z[2];
      if (csq(i) == 1) bz = -R(0.5) * (cx(i) ? Z[0] : (cy(i) ? Z[1] : Z[2]));
      const R geq = w * (rhoE + cqe * inv_theta +
                         (rt2 * (R(csq(i)) - R(3) * theta) + kappa * (cu * cu - theta * s.usq)) * h2) + bz;
      ge[i] = geq - P.ref[LG][i];
      dg[i] = dg[i] - ge[i];                      // non-equilibrium part
      s0 += dg[i];
    }
    dg[13] -= s0;                                 // energy defect onto the rest population
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const R w = wt(cx(i)) * wt(cy(i)) * wt(cz(i));
      const R cdq = R(cx(i)) * dq[0] + R(cy(i)) * dq[1] + R(cz(i)) * dq[2];
      const R dn = ge[i] + (R(1) - omega) * dg[i] + w * cdq * inv_theta;
      push<S, R, WALLS>(P, dst, b, LG, i, node, dn);
    }
  }
}

// --------------------------------------------------------------------------
// Read-back of the macroscopic fields
// --------------------------------------------------------------------------
template <typename S, typename R, int M>
__host__ __device__ inline void read_node(const Params<R>& P, const S* __restrict__ pop, int64_t node,
                                          double* X, double* rho_o, double* u, double* p, double* T)
{
  const size_t n = (size_t)P.n;
  constexpr int LF = M - 1, LG = M;
  R rho_s[M];
#pragma unroll
  for (int a = 0; a < M - 1; ++a) {
    R sum = R(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) sum += load_dev<S, R>(pop, (size_t)(a * Q + i) * n + node, P.inv_scale[a]);
    rho_s[a] = P.ref0[a] + sum;
  }
  rho_s[M - 1] = R(0);
  R rho = R(0), j[3] = {R(0), R(0), R(0)}, rhoE = R(0);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R d = load_dev<S, R>(pop, (size_t)(LF * Q + i) * n + node, P.inv_scale[LF]);
    rho += d;
    if (cx(i)) j[0] += cx(i) > 0 ? d : -d;
    if (cy(i)) j[1] += cy(i) > 0 ? d : -d;
    if (cz(i)) j[2] += cz(i) > 0 ? d : -d;
    rhoE += load_dev<S, R>(pop, (size_t)(LG * Q + i) * n + node, P.inv_scale[LG]);
  }
  rho += P.ref0[LF];
  rhoE += P.ref0[LG];
  Mix<R, M> s;
  mixture_state<R, M>(P, rho, j, rhoE, rho_s, s);
  if (X)
#pragma unroll
    for (int a = 0; a < M; ++a) X[(size_t)a * n + node] = (double)s.X[a];
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
template <typename S, int M>
__host__ __device__ inline int init_node(const Params<double>& P, const double* X,
                                         const double* p, const double* T, const double* u, S* __restrict__ pop,
                                         int64_t node)
{
  const size_t n = (size_t)P.n;
  constexpr int LF = M - 1, LG = M;
  double Xa[M], mmix = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    Xa[a] = X[(size_t)a * n + node];
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
  for (int a = 0; a < M - 1; ++a) {
    const double zeta = Tn * P.inv_m[a];
    if (!(zeta + usq < 1.0)) bad = 1;
    Trip<double> t[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) t[k] = psi_trip<double>(uu[k], zeta);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double f = rho * Y[a] * (t[0](cx(i)) * t[1](cy(i)) * t[2](cz(i)));
      pop[(size_t)(a * Q + i) * n + node] = S((f - P.ref[a][i]) * P.scale[a]);
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
      pop[(size_t)(LF * Q + i) * n + node] = S((f - P.ref[LF][i]) * P.scale[LF]);
    }
  }
  {
    const double rhoE = rho * (Cv * Tn + 0.5 * usq);
    const double hyd = Cp * Tn + 0.5 * usq;
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
      pop[(size_t)(LG * Q + i) * n + node] = S((g - P.ref[LG][i]) * P.scale[LG]);
    }
  }
  return bad;
}

// --------------------------------------------------------------------------
// Conserved sums of a node in FP64: rho_1..rho_M (rho_M slaved), rho, rho u, rho E,
// plus a flag for non-finite values or a negative slaved density.
// --------------------------------------------------------------------------
template <typename S, int M>
__host__ __device__ inline void conserved_node(const Params<double>& P, const S* __restrict__ pop,
                                               int64_t node, double* out /*[M+6]*/)
{
  const size_t n = (size_t)P.n;
  constexpr int LF = M - 1, LG = M;
  double rest = 0.0;
#pragma unroll
  for (int a = 0; a < M - 1; ++a) {
    double sum = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) sum += (double)pop[(size_t)(a * Q + i) * n + node] * P.inv_scale[a];
    out[a] = P.ref0[a] + sum;
    rest += out[a];
  }
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0}, rhoE = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const double d = (double)pop[(size_t)(LF * Q + i) * n + node] * P.inv_scale[LF];
    rho += d;
    j[0] += cx(i) * d;
    j[1] += cy(i) * d;
    j[2] += cz(i) * d;
    rhoE += (double)pop[(size_t)(LG * Q + i) * n + node] * P.inv_scale[LG];
  }
  rho += P.ref0[LF];
  rhoE += P.ref0[LG];
  out[M - 1] = rho - rest;
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

}  // namespace mclbm
