// lattice.hpp -- D3Q27 velocity set, product-form triplets and the per-context
// parameter block shared by the device kernels of libmclbm.
//
// Velocity index i = 9 (c_x + 1) + 3 (c_y + 1) + (c_z + 1), so the opposite
// direction is 26 - i. All loops over i are fully unrolled, which turns every
// c_{i,a} below into a compile-time constant.
#pragma once

#include <cstddef>
#include <cstdint>

namespace mclbm {

constexpr int Q = 27;
constexpr int MAXM = 8;           // species per context
constexpr int MAXL = MAXM + 2;    // stored lattices: up to M species, momentum f, energy g

// Stored lattices of an M-species context. Strong coupling (Sec. 3.5.2) stores
// species 1..M-1 (the slaved species' populations are never read); weak
// coupling (Sec. 3.5.1) stores all M species. Then the momentum lattice f (LF)
// and the energy lattice g (LG).
template <int M, bool WEAK>
struct Lat {
  static constexpr int NS = WEAK ? M : M - 1;
  static constexpr int LF = NS, LG = NS + 1, L = NS + 2;
};

__host__ __device__ constexpr int cx(int i) { return i / 9 - 1; }
__host__ __device__ constexpr int cy(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int cz(int i) { return i % 3 - 1; }
__host__ __device__ constexpr int cc(int i, int a) { return a == 0 ? cx(i) : (a == 1 ? cy(i) : cz(i)); }
__host__ __device__ constexpr int csq(int i) { return cx(i) * cx(i) + cy(i) * cy(i) + cz(i) * cz(i); }
__host__ __device__ constexpr int opp(int i) { return 26 - i; }
// Class of a direction under the reflections of the three axes: the directions
// with the same |c_x|, |c_y|, |c_z| (8 classes; the rest direction is class 0).
__host__ __device__ constexpr int ccls(int i)
{
  return (cx(i) != 0 ? 1 : 0) + (cy(i) != 0 ? 2 : 0) + (cz(i) != 0 ? 4 : 0);
}
constexpr int NCLS = 8;
// The first direction of i's class: reference tables are the same over a class,
// so reading them at the representative leaves 8 distinct values per lattice in
// scalar registers instead of 27.
__host__ __device__ constexpr int crep(int i)
{
  return (cx(i) != 0 ? 0 : 9) + (cy(i) != 0 ? 0 : 3) + (cz(i) != 0 ? 0 : 1);
}

// Values of a one-dimensional triplet at c = -1, 0, +1.
template <typename R>
struct Trip {
  R m, z, p;
  __host__ __device__ constexpr R operator()(int c) const { return c < 0 ? m : (c == 0 ? z : p); }
};

// Psi_{-1,0,+1}(xi, zeta) of the product-form equilibrium (Sec. 2.4).
template <typename R>
__host__ __device__ inline Trip<R> psi_trip(R xi, R zeta)
{
  R s = xi * xi + zeta;
  return {(s - xi) * R(0.5), R(1) - s, (s + xi) * R(0.5)};
}

// Psi(u) - Psi(u + V) per component, written without cancellation:
// c = 0: (u+V)^2 - u^2 = V (2u + V); c = +-1: (-+V - V (2u + V)) / 2.
template <typename R>
__host__ __device__ inline Trip<R> psi_diff_trip(R u, R V)
{
  R s = V * (R(2) * u + V);
  return {(V - s) * R(0.5), s, (-V - s) * R(0.5)};
}

// Weight triplet w_{-1,0,+1}(theta) = (theta/2, 1 - theta, theta/2), eq w0.
template <typename R>
__host__ __device__ inline Trip<R> w_trip(R theta)
{
  return {theta * R(0.5), R(1) - theta, theta * R(0.5)};
}

// Weights at theta = 1/3 used by the isotropic derivative 3 sum_i w_i c_i phi(x + c_i).
__host__ __device__ constexpr double w13_1d(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
__host__ __device__ constexpr double w13(int i) { return w13_1d(cx(i)) * w13_1d(cy(i)) * w13_1d(cz(i)); }

// Per-context constants, resident in device memory and read through uniform loads.
// Populations are stored as scaled deviations d = s_l (f - f_ref,l,i) from a
// reference that is the same for all directions of a class (ccls), so
// f_ref,i = f_ref,opp(i), and its first and mixed second moments vanish: the
// equilibrium at rest of the mean state, or, with 16-bit fixed-point storage, the
// centre of the range each class of each lattice takes.
template <typename R>
struct Params {
  int32_t M, nx, ny, nz;
  int32_t wall_x, trn, noz0, noz1;   // trn: transport exponents given (R19); opposed jets:
                                     // nozzle rows noz0 <= y < noz1 of both x faces
  int64_t n;
  R m[MAXM], inv_m[MAXM], cv[MAXM], cp[MAXM];
  R mu[MAXM], lam[MAXM], inv_lam[MAXM];
  R cvc[MAXM][4];         // C_{a,v}(T) = sum_k cvc[a][k] T^k (temperature-dependent kernels only)
  R s_mu[MAXM], s_lam[MAXM], s_D, T_ref;   // transport exponents about T_ref (same kernels)
  R invD[MAXM][MAXM];     // 1 / D_ab
  R phi[MAXM][MAXM];      // Wilke's phi_ab
  R ref[MAXL][Q];         // reference populations f_ref
  R ref0[MAXL];           // sum_i f_ref (zeroth moment)
  R ref2[MAXL][3];        // sum_i f_ref c_ia^2 (diagonal second moments)
  R scale[MAXL], inv_scale[MAXL];
  // 16-bit fixed-point storage: a stored integer v of lattice l, direction i is
  // f = f_ref,l,i + v inv_qs[l][ccls(i)]; qs is the encoding factor
  R qs[MAXL][NCLS], inv_qs[MAXL][NCLS];
  uint32_t* range_flag;   // fixed-point storage: bit 0 a value passed 3/4 of its range, bit 1 one was clamped
  R inl[MAXL][Q];         // open x ends and the jet at x = 0: inlet equilibrium minus f_ref, per stored lattice
  R inl2[MAXL][Q];        // opposed jets: the jet at x = nx - 1
  R absent_tol;           // |rho_a| <= absent_tol * rho: species absent, V_a = 0
  int32_t xperm[MAXM];    // the caller's index of species a (the slaved species is a = M-1
                          // here and may be any species to the caller): plane of X read
                          // by initialisation and written by the read-back
};

}  // namespace mclbm
