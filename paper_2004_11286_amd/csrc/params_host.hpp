// params_host.hpp -- host-side construction of the per-context parameter block:
// species data, Wilke factors, and the reference equilibria that the stored
// population deviations are taken from.
#pragma once

#include <cmath>
#include <cstring>

#include "lattice.hpp"

namespace mclbm {

struct HostSpecies {
  int M;
  double m[MAXM], cv[MAXM], mu[MAXM], lam[MAXM];
  double D[MAXM][MAXM];
  int cvt;                  // 1: C_{a,v}(T) = sum_k cvc[a][k] T^k, else the constant cv
  double cvc[MAXM][4];      // (the constant case holds cv[a], 0, 0, 0)
  double s_mu[MAXM], s_lam[MAXM], s_D, T_ref;   // transport exponents (0 and 1: constant)
  int trn;                  // 1: transport exponents given
};

// Mean state used for the reference equilibria (zero velocity).
struct RefState {
  double X[MAXM];
  double p, T;
};

// Reference and scale tables of one tube's stored lattices (also the per-tube
// part of a checkpoint): ref[l][i] the reference populations, ref0 and ref2 their
// zeroth and diagonal second moments; scale[l] the factor of floating-point
// deviations; qs[l][k] and inv_qs[l][k] the encoding and decoding factors of
// fixed-point storage per direction class k (zero otherwise).
struct RefTables {
  double ref[MAXL][Q];
  double ref0[MAXL];
  double ref2[MAXL][3];
  double scale[MAXL];
  double qs[MAXL][NCLS], inv_qs[MAXL][NCLS];
};

// Moments ref0 and ref2 of the reference populations of lattices 0..L-1.
inline void reference_moments(RefTables& t, int L)
{
  for (int l = 0; l < L; ++l) {
    t.ref0[l] = 0.0;
    for (int k = 0; k < 3; ++k) t.ref2[l][k] = 0.0;
    for (int i = 0; i < Q; ++i) {
      t.ref0[l] += t.ref[l][i];
      for (int k = 0; k < 3; ++k) t.ref2[l][k] += t.ref[l][i] * cc(i, k) * cc(i, k);
    }
  }
}

// Wilke's phi_ab (Sec. 3.3, eq wilkePhi).
inline double wilke_phi(const HostSpecies& h, int a, int b)
{
  double num = 1.0 + std::sqrt((h.mu[a] / h.mu[b]) * std::sqrt(h.m[b] / h.m[a]));
  return num * num / (std::sqrt(8.0) * std::sqrt(1.0 + h.m[a] / h.m[b]));
}

// Reference populations of every stored lattice at the mean state, zero
// velocity: species rho_a Psi(0, R_a T) for the ns stored species (M-1 under
// strong coupling, M under weak), momentum rho Psi(0, R T) at lattice ns, energy
// the energy-lattice equilibrium with zero flux at ns + 1. All are symmetric
// under c -> -c.
inline void reference_tables(const HostSpecies& h, int ns, const RefState& rs, RefTables& tab)
{
  double (&ref)[MAXL][Q] = tab.ref;
  const int M = h.M;
  double mmix = 0.0;
  for (int a = 0; a < M; ++a) mmix += rs.X[a] * h.m[a];
  const double Rg = 1.0 / mmix;
  const double rho = rs.p / (Rg * rs.T);
  double Cv = 0.0;
  for (int a = 0; a < M; ++a) Cv += rs.X[a] * h.m[a] / mmix * h.cv[a];
  double U = 0.0;           // with C_v(T): specific internal energy at the mean state (eq Umix)
  if (h.cvt) {
    for (int a = 0; a < M; ++a) {
      const double* c = h.cvc[a];
      const double T = rs.T;
      U += rs.X[a] * h.m[a] / mmix * T * (c[0] + T * (c[1] / 2 + T * (c[2] / 3 + T * c[3] / 4)));
    }
  }
  std::memset(ref, 0, sizeof(double) * MAXL * Q);
  auto fill_psi = [&](int l, double dens, double zeta) {
    Trip<double> t = psi_trip<double>(0.0, zeta);
    for (int i = 0; i < Q; ++i) ref[l][i] = dens * t(cx(i)) * t(cy(i)) * t(cz(i));
  };
  for (int a = 0; a < ns; ++a) fill_psi(a, rho * rs.X[a] * h.m[a] / mmix, rs.T / h.m[a]);
  fill_psi(ns, rho, Rg * rs.T);
  {
    const double theta = Rg * rs.T;
    const double rhoE = h.cvt ? rho * U : rho * Cv * rs.T;
    const double rt2 = rho * theta * theta;
    const double zf = (1.0 - 3.0 * theta) * 0.5 / theta;
    const Trip<double> wt = w_trip<double>(theta);
    for (int i = 0; i < Q; ++i) {
      const double w = wt(cx(i)) * wt(cy(i)) * wt(cz(i));
      double bz = 0.0;
      if (csq(i) == 0) bz = 3.0 * zf * rt2;
      if (csq(i) == 1) bz = -0.5 * zf * rt2;
      ref[ns + 1][i] = w * (rhoE + rt2 * (csq(i) - 3.0 * theta) * 0.5 / (theta * theta)) + bz;
    }
  }
  reference_moments(tab, ns + 2);
}

// Fill a parameter block. scale[l] multiplies stored floating-point deviations (1
// for FP64 and FP32 storage; a range-fitting factor for 16-bit floating point);
// range_flag is the context's device word that fixed-point kernels report to.
template <typename R>
inline void fill_params(Params<R>& P, const HostSpecies& h, int nx, int ny, int nz, int wall_x, int L,
                        const RefTables& t, double absent_tol, uint32_t* range_flag, const int32_t* xperm,
                        int noz0 = 0, int noz1 = 0)
{
  std::memset(&P, 0, sizeof(P));
  P.M = h.M;
  P.nx = nx;
  P.ny = ny;
  P.nz = nz;
  P.wall_x = wall_x;
  P.noz0 = noz0;
  P.noz1 = noz1;
  P.n = (int64_t)nx * ny * nz;
  for (int a = 0; a < h.M; ++a) {
    P.m[a] = R(h.m[a]);
    P.inv_m[a] = R(1.0 / h.m[a]);
    P.cv[a] = R(h.cv[a]);
    P.cp[a] = R(h.cv[a] + 1.0 / h.m[a]);       // Mayer: C_{a,p} - C_{a,v} = R_a
    P.mu[a] = R(h.mu[a]);
    P.lam[a] = R(h.lam[a]);
    for (int k = 0; k < 4; ++k) P.cvc[a][k] = R(h.cvc[a][k]);
    P.s_mu[a] = R(h.s_mu[a]);
    P.s_lam[a] = R(h.s_lam[a]);
    P.inv_lam[a] = R(1.0 / h.lam[a]);
    for (int b = 0; b < h.M; ++b) {
      P.invD[a][b] = R(1.0 / h.D[a][b]);
      P.phi[a][b] = R(wilke_phi(h, a, b));
    }
  }
  for (int l = 0; l < L; ++l) {
    for (int i = 0; i < Q; ++i) P.ref[l][i] = R(t.ref[l][i]);
    P.ref0[l] = R(t.ref0[l]);
    for (int k = 0; k < 3; ++k) P.ref2[l][k] = R(t.ref2[l][k]);
    P.scale[l] = R(t.scale[l]);
    P.inv_scale[l] = R(1.0 / t.scale[l]);
    for (int k = 0; k < NCLS; ++k) {
      P.qs[l][k] = R(t.qs[l][k]);
      P.inv_qs[l][k] = R(t.inv_qs[l][k]);
    }
  }
  P.range_flag = range_flag;
  for (int a = 0; a < MAXM; ++a) P.xperm[a] = a < h.M ? xperm[a] : a;
  P.absent_tol = R(absent_tol);
  P.s_D = R(h.s_D);
  P.trn = h.trn;
  P.T_ref = R(h.T_ref);
}

}  // namespace mclbm
