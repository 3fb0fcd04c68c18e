/*
 * mclbm_oracle.c -- plain FP64 CPU oracle of one time step of the consistent
 * multicomponent lattice Boltzmann model (Sawant, Dorschner, Karlin,
 * arXiv 2004.11286).
 *
 * TEST INFRASTRUCTURE: written to be read against the paper, not to be fast.
 * Only tests, the smoke check and the benchmark's CPU-baseline leg use it; the
 * GPU library never links or calls it. Compiled with -O2 -ffp-contract=off.
 *
 * One time step, in the paper's order:
 *   1. moments of every lattice; strong coupling slaves species M to the
 *      momentum lattice (Sec. 3.5.2, eqs rhoMATCH, uMATCH); weak coupling
 *      (Sec. 3.5.1) evolves every species lattice with its own conservation law;
 *      temperature from the energy lattice: with constant specific heats in
 *      closed form (eq temperature2, T_0=0), with specific heats polynomial in T
 *      by Newton's method on eq temperature;
 *   2. mixture viscosity (Wilke, eq viscosityMixture) and conductivity (Mathur,
 *      eq conductivityMixture), relaxation rates omega, omega_1 (eqs omega, omega1);
 *   3. the non-local terms at the same time level: the isotropy correction X
 *      (eq Xalpha) and the mass-fraction gradients of the correction flux
 *      (eq corrFourier), with second-order isotropic lattice derivatives (Sec. 4.1);
 *   4. species collision (eqs SMlbm, fstar1, transform12);
 *   5. momentum collision (eq fwithcorrection with eqs feq, Ai);
 *   6. energy collision (eq g with eqs gieq, gistar, gstareq1mom, interdiffusion,
 *      corrFourier, and the ansatz eqs gansatz, grad, weights, w0,
 *      RcorrectionPrime, Bi);
 *   7. streaming along c_i; periodic, or half-way bounce-back at x walls for
 *      all populations (Sec. 4.2).
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes of the repository):
 *   - lattice units R_U = 1, dt = dx = 1;
 *   - the self-diffusivity D_aa is an input (the sums in eqs tau and fStar run
 *     over b = a);
 *   - derivative operator d_a phi(x) = 3 sum_i w_i c_ia phi(x + c_i) with the
 *     D3Q27 weights at theta = 1/3; the nested derivative of eq Xalpha applies
 *     it twice with (1/omega - 1/2) taken per node in between;
 *   - walls: ghost nodes mirror the interior about the wall half-way between
 *     nodes; the x component of the momentum-like field Phi changes sign;
 *   - a species with rho_a == 0 exactly has an identically zero row in
 *     eq transform12; its diffusion velocity is set to zero;
 *   - initial populations are the local equilibria of the given fields;
 *   - weak coupling: the species see the species-barycentric velocity
 *     u_s = sum_a j_a / sum_a rho_a (in J_a = j_a - rho_a u_s of eq transform12
 *     and in the species equilibria), and the composition is Y_a = rho_a /
 *     sum_b rho_b; the mixture density, velocity, temperature and pressure come
 *     from the momentum and energy lattices as under strong coupling.
 *
 * Pins (tests run on the CPU): moment identities of the equilibria and of the
 * energy ansatz, the correction vectors, the derivative operator's symbol,
 * conservation, the equilibrium fixed point, the mid-point identity of the
 * species collision, binary erf interdiffusion, ternary half-tube means against
 * an independent Maxwell--Stefan solver, the printed gas constants and sound
 * speeds of S1-S4, Kirchhoff sound attenuation, shear and thermal decay with
 * the Wilke and Mathur mixing rules, temperature uniformity under
 * interdiffusion, and the viscous heating pattern of a decaying shear wave
 * against linearised Navier--Stokes (which pins the -u.(P - P^eq) term of
 * eq gstareq1mom). Weak coupling, temperature-dependent heat capacities and
 * transport, and open x ends have pins of their own.
 */
#include "mclbm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 27
#define MAXM ORACLE_MAXM

/* ------------------------------------------------------------------------- */
/* D3Q27 velocities, eq d3q27vel: i = 9 (c_x + 1) + 3 (c_y + 1) + (c_z + 1).   */
/* ------------------------------------------------------------------------- */
static int cvel(int i, int axis)
{
  if (axis == 0) return i / 9 - 1;
  if (axis == 1) return (i / 3) % 3 - 1;
  return i % 3 - 1;
}

static int opposite(int i)
{
  int cx = -cvel(i, 0), cy = -cvel(i, 1), cz = -cvel(i, 2);
  return 9 * (cx + 1) + 3 * (cy + 1) + (cz + 1);
}

void oracle_velocities(int32_t c[27 * 3])
{
  for (int i = 0; i < Q; ++i)
    for (int a = 0; a < 3; ++a) c[3 * i + a] = cvel(i, a);
}

/* The one-dimensional triplet Psi_{-1}, Psi_0, Psi_{+1} of Sec. 2.4. */
static double psi_1d(int c, double xi, double zeta)
{
  double s = xi * xi + zeta;
  if (c == 0) return 1.0 - s;
  if (c == 1) return (xi + s) / 2.0;
  return (-xi + s) / 2.0;
}

/* Product form, eq prod. */
void oracle_psi(const double xi[3], double zeta, double out[27])
{
  for (int i = 0; i < Q; ++i)
    out[i] = psi_1d(cvel(i, 0), xi[0], zeta) * psi_1d(cvel(i, 1), xi[1], zeta) *
             psi_1d(cvel(i, 2), xi[2], zeta);
}

/* Weights in product form, eqs weights and w0. */
static double w_1d(int c, double theta) { return c == 0 ? 1.0 - theta : theta / 2.0; }

void oracle_weights(double theta, double out[27])
{
  for (int i = 0; i < Q; ++i)
    out[i] = w_1d(cvel(i, 0), theta) * w_1d(cvel(i, 1), theta) * w_1d(cvel(i, 2), theta);
}

/* Vectors A_i (eq Ai) and B_i (eq Bi). */
static double A_table(int i, int a)
{
  int c2 = cvel(i, 0) * cvel(i, 0) + cvel(i, 1) * cvel(i, 1) + cvel(i, 2) * cvel(i, 2);
  return c2 == 1 ? 0.5 * cvel(i, a) : 0.0;
}

static double B_table(int i, int a)
{
  int c2 = cvel(i, 0) * cvel(i, 0) + cvel(i, 1) * cvel(i, 1) + cvel(i, 2) * cvel(i, 2);
  if (c2 == 0) return 1.0;
  if (c2 == 1) return -0.5 * abs(cvel(i, a));
  return 0.0;
}

void oracle_tables(double A[27 * 3], double B[27 * 3])
{
  for (int i = 0; i < Q; ++i)
    for (int a = 0; a < 3; ++a) {
      A[3 * i + a] = A_table(i, a);
      B[3 * i + a] = B_table(i, a);
    }
}

/* Energy-lattice ansatz G_i(theta, M0, m, M), eqs gansatz, grad, RcorrectionPrime. */
void oracle_gansatz(double theta, double M0, const double m[3], const double Mt[9],
                    double out[27])
{
  double Z[3];
  for (int a = 0; a < 3; ++a)
    Z[a] = (1.0 - 3.0 * theta) / (2.0 * theta) * (Mt[3 * a + a] - theta * M0);
  double w[Q];
  oracle_weights(theta, w);
  for (int i = 0; i < Q; ++i) {
    double c[3] = {cvel(i, 0), cvel(i, 1), cvel(i, 2)};
    double mc = 0.0;
    for (int a = 0; a < 3; ++a) mc += m[a] * c[a];
    double contraction = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double Mab = Mt[3 * a + b] - (a == b ? M0 * theta : 0.0);
        double Cab = c[a] * c[b] - (a == b ? theta : 0.0);
        contraction += Mab * Cab;
      }
    double h = w[i] * (M0 + mc / theta + contraction / (2.0 * theta * theta));
    double BZ = 0.0;
    for (int a = 0; a < 3; ++a) BZ += B_table(i, a) * Z[a];
    out[i] = h + BZ;
  }
}

/* ------------------------------------------------------------------------- */
/* Simulation state                                                           */
/* ------------------------------------------------------------------------- */
struct oracle_sim {
  int M, nx, ny, nz, wall_x, wall_y, keep_slaved, weak, flags;
  long n;
  double m[MAXM], cv[MAXM], D[MAXM][MAXM], mu[MAXM], lam[MAXM];
  int cvt;                 /* 1: C_{a,v}(T) = sum_k cvc[a][k] T^k, else the constant cv[a] */
  double cvc[MAXM][4];
  double fin[MAXM + 2][Q]; /* open x ends and jets: populations of the inlet equilibrium at x = 0 */
  double fin2[MAXM + 2][Q];/* jets: populations of the inlet equilibrium at x = nx - 1 */
  int ny0, ny1;            /* jets: nozzle rows ny0 <= y < ny1 */
  int trn;                 /* 1: transport coefficients as powers of T / T_ref */
  double s_mu[MAXM], s_lam[MAXM], s_D, T_ref;
  double *pop;   /* [(M+2)][Q][n] pre-collision populations */
  double *post;  /* [(M+2)][Q][n] post-collision populations */
  /* node fields used by the non-local terms */
  double *Phi;   /* [3][n] rho u_a (1 - 3 R T) - rho u_a^3      */
  double *om;    /* [n]    omega                                 */
  double *Yf;    /* [M][n] mass fractions                        */
  double *G;     /* [3][nz][ny][nx+2] (1/omega - 1/2) d_a Phi_a, one ghost layer in x */
  double *Xc;    /* [3][n] isotropy correction X_a               */
  double *gY;    /* [M][3][n] mass-fraction gradients            */
  int err;
};

#define POP(s, buf, l, i, node) ((buf)[((long)(l) * Q + (i)) * (s)->n + (node)])
#define LAT_F(s) ((s)->M)
#define LAT_G(s) ((s)->M + 1)

static long node_index(const oracle_sim *s, int x, int y, int z)
{
  return (long)x + (long)s->nx * ((long)y + (long)s->ny * (long)z);
}

static int wrap(int v, int n) { return ((v % n) + n) % n; }

int oracle_set_threads(int32_t nthreads)
{
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  return 0;
}

int oracle_threads(void)
{
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static int local_equilibrium(const oracle_sim *s, const double *Xa, double Pn, double Tn, const double uu[3],
                             double out[][Q]);

int oracle_create(const oracle_params *p, oracle_sim **out)
{
  if (!p || !out) return -1;
  *out = NULL;
  if (p->M < 2 || p->M > MAXM || p->nx < 1 || p->ny < 1 || p->nz < 1) return -1;
  if (p->wall_x && p->nx < 2) return -1;
  if (p->wall_x < 0 || p->wall_x > 3 || (p->wall_x >= 2 && !p->inlet)) return -1;
  /* opposed jets: two nozzles, free-slip walls beside them, outlets at the y ends */
  if ((p->wall_x == 3) != (p->wall_y == 2)) return -1;
  if (p->wall_x == 3 && (!p->inlet_right || p->nozzle_y0 < 1 || p->nozzle_y1 > p->ny - 1 ||
                         p->nozzle_y0 >= p->nozzle_y1))
    return -1;
  if (!p->molar_mass || !p->cv || !p->D || !p->mu || !p->lambda) return -1;
  oracle_sim *s = (oracle_sim *)calloc(1, sizeof(oracle_sim));
  if (!s) return -1;
  s->M = p->M;
  s->nx = p->nx; s->ny = p->ny; s->nz = p->nz;
  s->wall_x = p->wall_x;
  s->wall_y = p->wall_y == 2 ? 2 : (p->wall_y ? 1 : 0);
  if (s->wall_y == 1 && (p->ny < 2 || s->wall_x >= 2)) {
    free(s);
    return -1;
  }
  s->ny0 = p->nozzle_y0;
  s->ny1 = p->nozzle_y1;
  s->weak = p->weak ? 1 : 0;
  s->keep_slaved = (p->keep_slaved || s->weak) ? 1 : 0;   /* weak coupling evolves every species */
  s->flags = p->debug_flags;
  s->n = (long)p->nx * p->ny * p->nz;
  s->cvt = p->cv_coef ? 1 : 0;
  s->trn = p->transport_exp ? 1 : 0;
  if (s->trn) {
    for (int a = 0; a < s->M; ++a) {
      s->s_mu[a] = p->transport_exp[a];
      s->s_lam[a] = p->transport_exp[s->M + a];
    }
    s->s_D = p->transport_exp[2 * s->M];
    s->T_ref = p->transport_exp[2 * s->M + 1];
    if (!(s->T_ref > 0)) {
      free(s);
      return -1;
    }
  }
  for (int a = 0; a < s->M; ++a) {
    s->m[a] = p->molar_mass[a];
    s->cv[a] = p->cv[a];
    if (s->cvt) {
      for (int k = 0; k < 4; ++k) {
        s->cvc[a][k] = p->cv_coef[a * 4 + k];
        if (!(k == 0 ? s->cvc[a][k] > 0 : s->cvc[a][k] >= 0)) {
          free(s);
          return -1;
        }
      }
    }
    s->mu[a] = p->mu[a];
    s->lam[a] = p->lambda[a];
    if (!(s->m[a] > 0) || !(s->cv[a] > 0) || !(s->mu[a] > 0) || !(s->lam[a] > 0)) {
      free(s);
      return -1;
    }
    for (int b = 0; b < s->M; ++b) {
      s->D[a][b] = p->D[a * s->M + b];
      if (!(s->D[a][b] > 0) || p->D[a * s->M + b] != p->D[b * s->M + a]) {
        free(s);
        return -1;
      }
    }
  }
  long n = s->n;
  int L = s->M + 2;
  s->pop = (double *)calloc((size_t)L * Q * n, sizeof(double));
  s->post = (double *)calloc((size_t)L * Q * n, sizeof(double));
  s->Phi = (double *)calloc((size_t)3 * n, sizeof(double));
  s->om = (double *)calloc((size_t)n, sizeof(double));
  s->Yf = (double *)calloc((size_t)s->M * n, sizeof(double));
  s->G = (double *)calloc((size_t)3 * (s->nx + 2) * s->ny * s->nz, sizeof(double));
  s->Xc = (double *)calloc((size_t)3 * n, sizeof(double));
  s->gY = (double *)calloc((size_t)s->M * 3 * n, sizeof(double));
  if (!s->pop || !s->post || !s->Phi || !s->om || !s->Yf || !s->G || !s->Xc || !s->gY) {
    oracle_destroy(s);
    return -1;
  }
  if (s->wall_x >= 2) {
    /* inlet fields: X (M), p, T, u (3) */
    const double *in = p->inlet;
    const double uin[3] = {in[s->M + 2], in[s->M + 3], in[s->M + 4]};
    if (local_equilibrium(s, in, in[s->M], in[s->M + 1], uin, s->fin) != 0) {
      oracle_destroy(s);
      return -1;
    }
  }
  if (s->wall_x == 3) {
    const double *in = p->inlet_right;
    const double uin[3] = {in[s->M + 2], in[s->M + 3], in[s->M + 4]};
    if (local_equilibrium(s, in, in[s->M], in[s->M + 1], uin, s->fin2) != 0) {
      oracle_destroy(s);
      return -1;
    }
  }
  *out = s;
  return 0;
}

void oracle_destroy(oracle_sim *s)
{
  if (!s) return;
  free(s->pop); free(s->post); free(s->Phi); free(s->om); free(s->Yf);
  free(s->G); free(s->Xc); free(s->gY);
  free(s);
}

/* ------------------------------------------------------------------------- */
/* Macroscopic state of a node                                               */
/* ------------------------------------------------------------------------- */
typedef struct {
  double rho_a[MAXM], j_a[MAXM][3];
  double rho, j[3], rhoE;
  double u[3], us[3], Y[MAXM], X[MAXM], mmix, R, Cv, Cp, T, P, Ps;
  double Ha[MAXM], H;
  double mu, lam, omega, omega1;
} state_t;

/* Wilke's factor phi_ab, eq wilkePhi, for species viscosities mu_a, mu_b. */
static double wilke_phi(const oracle_sim *s, int a, int b, double mu_a, double mu_b)
{
  double num = 1.0 + sqrt((mu_a / mu_b) * sqrt(s->m[b] / s->m[a]));
  return num * num / (sqrt(8.0) * sqrt(1.0 + s->m[a] / s->m[b]));
}

/* Species transport coefficients at temperature T: the given constants, or, with
 * temperature exponents, mu_a (T / T_ref)^s_mu,a, lambda_a (T / T_ref)^s_lam,a and
 * D_ab (T / T_ref)^s_D. */
static double species_mu(const oracle_sim *s, int a, double T)
{
  return s->trn ? s->mu[a] * pow(T / s->T_ref, s->s_mu[a]) : s->mu[a];
}

static double species_lam(const oracle_sim *s, int a, double T)
{
  return s->trn ? s->lam[a] * pow(T / s->T_ref, s->s_lam[a]) : s->lam[a];
}

static double diffusivity(const oracle_sim *s, int a, int b, double T)
{
  return s->trn ? s->D[a][b] * pow(T / s->T_ref, s->s_D) : s->D[a][b];
}

/* Specific heat of species a at temperature T (polynomial case), and its
 * internal energy U_a(T), the integral of C_{a,v} from T_0 = 0 (eq specUa). */
static double species_cv(const oracle_sim *s, int a, double T)
{
  const double *c = s->cvc[a];
  return c[0] + c[1] * T + c[2] * T * T + c[3] * T * T * T;
}

static double species_U(const oracle_sim *s, int a, double T)
{
  const double *c = s->cvc[a];
  return c[0] * T + c[1] * T * T / 2.0 + c[2] * T * T * T / 3.0 + c[3] * T * T * T * T / 4.0;
}

/* Temperature from eq temperature, sum_a Y_a U_a(T) = e, by Newton's method:
 * U is increasing and convex for c_0 > 0, c_k >= 0, so the iteration started at
 * e / sum_a Y_a c_a0 (an upper bound) decreases monotonically to the root. */
static double solve_temperature(const oracle_sim *s, const double *Y, double e)
{
  double c0 = 0.0;
  for (int a = 0; a < s->M; ++a) c0 += Y[a] * s->cvc[a][0];
  double T = e / c0;
  for (int it = 0; it < 100; ++it) {
    double U = 0.0, Cv = 0.0;
    for (int a = 0; a < s->M; ++a) {
      U += Y[a] * species_U(s, a, T);
      Cv += Y[a] * species_cv(s, a, T);
    }
    double dT = (U - e) / Cv;
    T -= dT;
    if (fabs(dT) <= 1e-15 * fabs(T)) break;
  }
  return T;
}

static void node_state(const oracle_sim *s, const double *pop, long node, state_t *st)
{
  const int M = s->M;
  memset(st, 0, sizeof(*st));
  /* momentum and energy lattices: eqs f0momDensity, f1momMomentum, g0momTotalEnergy */
  for (int i = 0; i < Q; ++i) {
    double fi = POP(s, pop, LAT_F(s), i, node);
    st->rho += fi;
    for (int a = 0; a < 3; ++a) st->j[a] += fi * cvel(i, a);
    st->rhoE += POP(s, pop, LAT_G(s), i, node);
  }
  /* species 1..M-1 (all M under weak coupling): eqs densitya, auxua */
  const int nown = s->weak ? M : M - 1;
  for (int a = 0; a < nown; ++a)
    for (int i = 0; i < Q; ++i) {
      double fai = POP(s, pop, a, i, node);
      st->rho_a[a] += fai;
      for (int k = 0; k < 3; ++k) st->j_a[a][k] += fai * cvel(i, k);
    }
  if (!s->weak) {
    /* strong coupling: the slaved species takes the deficits, eqs rhoMATCH, uMATCH */
    st->rho_a[M - 1] = st->rho;
    for (int k = 0; k < 3; ++k) st->j_a[M - 1][k] = st->j[k];
    for (int a = 0; a < M - 1; ++a) {
      st->rho_a[M - 1] -= st->rho_a[a];
      for (int k = 0; k < 3; ++k) st->j_a[M - 1][k] -= st->j_a[a][k];
    }
  }
  for (int k = 0; k < 3; ++k) st->u[k] = st->j[k] / st->rho;
  /* the species' own density: rho under strong coupling, sum_a rho_a under weak */
  double rho_sp = st->rho;
  if (s->weak) {
    rho_sp = 0.0;
    for (int a = 0; a < M; ++a) rho_sp += st->rho_a[a];
  }
  /* velocity the species relax towards: u, or the species-barycentric one */
  for (int k = 0; k < 3; ++k) {
    st->us[k] = st->u[k];
    if (s->weak && !(s->flags & ORACLE_WEAK_MIXTURE_U)) {
      double js = 0.0;
      for (int a = 0; a < M; ++a) js += st->j_a[a][k];
      st->us[k] = js / rho_sp;
    }
  }
  /* composition, Sec. 2.1 */
  double inv_m = 0.0;
  for (int a = 0; a < M; ++a) {
    st->Y[a] = st->rho_a[a] / rho_sp;
    inv_m += st->Y[a] / s->m[a];
  }
  st->mmix = 1.0 / inv_m;
  for (int a = 0; a < M; ++a) st->X[a] = (st->mmix / s->m[a]) * st->Y[a];
  st->R = 1.0 / st->mmix;                                /* eq defineSpecificGasContant */
  double usq = st->u[0] * st->u[0] + st->u[1] * st->u[1] + st->u[2] * st->u[2];
  if (s->cvt) {
    /* specific heats polynomial in T: eq temperature, then eq Cvmix at that T */
    st->T = solve_temperature(s, st->Y, st->rhoE / st->rho - usq / 2.0);
    for (int a = 0; a < M; ++a) st->Cv += st->Y[a] * species_cv(s, a, st->T);
    st->Cp = st->Cv + st->R;                             /* Mayer */
  } else {
    /* caloric properties, Sec. 3.1 with constant C_{a,v} and C_{a,p} = C_{a,v} + R_a */
    for (int a = 0; a < M; ++a) {
      st->Cv += st->Y[a] * s->cv[a];
      st->Cp += st->Y[a] * (s->cv[a] + 1.0 / s->m[a]);
    }
    st->T = (st->rhoE / st->rho - usq / 2.0) / st->Cv;   /* eq temperature2, T_0 = 0 */
  }
  st->P = st->rho * st->R * st->T;                       /* eq eosIdealGas */
  /* pressure of the species subsystem in its friction terms: P under strong
   * coupling, sum_a rho_a R_a T of the species' own densities under weak */
  st->Ps = (s->weak && !(s->flags & ORACLE_WEAK_MIXTURE_P)) ? rho_sp * st->R * st->T : st->P;
  for (int a = 0; a < M; ++a) {
    if (s->cvt && (s->flags & ORACLE_CVT_HA_CPT))
      st->Ha[a] = (species_cv(s, a, st->T) + 1.0 / s->m[a]) * st->T;
    else if (s->cvt)
      st->Ha[a] = species_U(s, a, st->T) + st->T / s->m[a];            /* eq specHa */
    else st->Ha[a] = (s->cv[a] + 1.0 / s->m[a]) * st->T;
    st->H += st->Y[a] * st->Ha[a];                       /* eq specH */
  }
  /* transport, eqs viscosityMixture and conductivityMixture */
  double mu_a[MAXM], lam_a[MAXM];
  for (int a = 0; a < M; ++a) {
    mu_a[a] = species_mu(s, a, st->T);
    lam_a[a] = species_lam(s, a, st->T);
  }
  for (int a = 0; a < M; ++a) {
    double den = 0.0;
    for (int b = 0; b < M; ++b) den += wilke_phi(s, a, b, mu_a[a], mu_a[b]) * st->X[b];
    st->mu += mu_a[a] * st->X[a] / den;
  }
  double lin = 0.0, harm = 0.0;
  for (int a = 0; a < M; ++a) {
    lin += st->X[a] * lam_a[a];
    harm += st->X[a] / lam_a[a];
  }
  st->lam = 0.5 * (lin + 1.0 / harm);
  st->omega = 2.0 * st->P / (st->P + 2.0 * st->mu);                     /* eq omega  */
  st->omega1 = 2.0 * st->P * st->Cp / (st->P * st->Cp + 2.0 * st->lam); /* eq omega1 */
}

/* ------------------------------------------------------------------------- */
/* Non-local terms                                                           */
/* ------------------------------------------------------------------------- */
/* Value of a node field at integer position (x, y, z): periodic in z; in x
 * periodic, or mirrored about the walls at x = -1/2 and x = nx - 1/2, or, at open
 * x ends, the boundary node's value (zero gradient); in y periodic, or mirrored
 * about free-slip walls at y = -1/2 and y = ny - 1/2. comp is the vector
 * component the field is (-1 for a scalar): a mirror flips the sign of the
 * component normal to it. */
static int nozzle_row(const oracle_sim *s, int y) { return y >= s->ny0 && y < s->ny1; }

static double field_at(const oracle_sim *s, const double *fld, int x, int y, int z, int comp)
{
  double sign = 1.0;
  z = wrap(z, s->nz);
  if (s->wall_y == 2) {
    if (y < 0) y = 0;                 /* outlets: zero gradient */
    else if (y >= s->ny) y = s->ny - 1;
  } else if (s->wall_y) {
    if (y < 0) { y = -1 - y; if (comp == 1) sign = -sign; }
    else if (y >= s->ny) { y = 2 * s->ny - 1 - y; if (comp == 1) sign = -sign; }
  } else {
    y = wrap(y, s->ny);
  }
  if (s->wall_x == 3) {
    /* jets: zero gradient beyond a nozzle, the mirror beyond a free-slip wall */
    if (x < 0) {
      if (nozzle_row(s, y)) x = 0;
      else { x = -1 - x; if (comp == 0) sign = -sign; }
    } else if (x >= s->nx) {
      if (nozzle_row(s, y)) x = s->nx - 1;
      else { x = 2 * s->nx - 1 - x; if (comp == 0) sign = -sign; }
    }
  } else if (s->wall_x == 1) {
    if (x < 0) { x = -1 - x; if (comp == 0) sign = -sign; }
    else if (x >= s->nx) { x = 2 * s->nx - 1 - x; if (comp == 0) sign = -sign; }
  } else if (s->wall_x == 2) {
    if (x < 0) x = 0;
    else if (x >= s->nx) x = s->nx - 1;
  } else {
    x = wrap(x, s->nx);
  }
  return sign * fld[node_index(s, x, y, z)];
}

/* Second-order isotropic derivative along axis k (the reading of the operators
 * named in Sec. 4.1): d_k phi(x) = 3 sum_i w_i(1/3) c_ik phi(x + c_i). Every
 * derivative the oracle takes goes through this one routine; the field is read
 * through an accessor that applies the boundary rule. */
typedef double (*accessor_fn)(const void *ctx, int x, int y, int z);

static double W13[Q];

static void init_w13(void)
{
  static int done = 0;
  if (!done) {
    oracle_weights(1.0 / 3.0, W13);
    done = 1;
  }
}

static double iso_deriv(accessor_fn get, const void *ctx, int x, int y, int z, int k)
{
  double d = 0.0;
  for (int i = 0; i < Q; ++i) {
    if (cvel(i, k) == 0) continue;
    d += 3.0 * W13[i] * cvel(i, k) * get(ctx, x + cvel(i, 0), y + cvel(i, 1), z + cvel(i, 2));
  }
  return d;
}

/* accessor: node field with the simulation's boundary rule */
typedef struct { const oracle_sim *s; const double *fld; int comp; } node_field_ctx;

static double node_field_get(const void *ctx, int x, int y, int z)
{
  const node_field_ctx *c = (const node_field_ctx *)ctx;
  return field_at(c->s, c->fld, x, y, z, c->comp);
}

/* accessor: plain periodic field on an nx*ny*nz grid */
typedef struct { int nx, ny, nz; const double *fld; } periodic_ctx;

static double periodic_get(const void *ctx, int x, int y, int z)
{
  const periodic_ctx *c = (const periodic_ctx *)ctx;
  return c->fld[wrap(x, c->nx) + (long)c->nx * (wrap(y, c->ny) + (long)c->ny * wrap(z, c->nz))];
}

int oracle_gradient(int32_t nx, int32_t ny, int32_t nz, const double *phi, double *grad)
{
  if (nx < 1 || ny < 1 || nz < 1 || !phi || !grad) return -1;
  init_w13();
  long n = (long)nx * ny * nz;
  periodic_ctx ctx = {nx, ny, nz, phi};
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        long node = x + (long)nx * (y + (long)ny * z);
        for (int k = 0; k < 3; ++k) grad[(long)k * n + node] = iso_deriv(periodic_get, &ctx, x, y, z, k);
      }
  return 0;
}

/* G field with one ghost layer in x: index (k, z, y, x+1). */
static long gidx(const oracle_sim *s, int k, int x, int y, int z)
{
  return (long)(x + 1) + (long)(s->nx + 2) * ((long)y + (long)s->ny * ((long)z + (long)s->nz * k));
}

/* accessor: component k of G on nodes and the x ghost layer (periodic in y, z;
 * in x periodic, or read from the ghost layer next to a wall) */
typedef struct { const oracle_sim *s; int k; } g_ctx;

static double g_get(const void *ctx, int x, int y, int z)
{
  const g_ctx *c = (const g_ctx *)ctx;
  const oracle_sim *s = c->s;
  if (!s->wall_x) x = wrap(x, s->nx);
  /* free-slip y walls: every G_k is even under the y mirror (d_y Phi_y is);
   * outlets: the boundary node's G (zero gradient) */
  if (s->wall_y == 2) y = y < 0 ? 0 : (y >= s->ny ? s->ny - 1 : y);
  else if (s->wall_y) y = y < 0 ? -1 - y : (y >= s->ny ? 2 * s->ny - 1 - y : y);
  return s->G[gidx(s, c->k, x, wrap(y, s->ny), wrap(z, s->nz))];
}

static void compute_nonlocal(oracle_sim *s)
{
  const int nx = s->nx, ny = s->ny, nz = s->nz, M = s->M;
  const long n = s->n;
  init_w13();
  /* G_k = (1/omega - 1/2) d_k Phi_k at the nodes and at one ghost layer beyond
   * each x end (there Phi and omega are the mirrored values). */
#pragma omp parallel for schedule(static) if (n >= 512)
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = -1; x <= nx; ++x)
        for (int k = 0; k < 3; ++k) {
          node_field_ctx phi = {s, s->Phi + (long)k * n, k};
          double omega = field_at(s, s->om, x, y, z, -1);
          s->G[gidx(s, k, x, y, z)] = (1.0 / omega - 0.5) * iso_deriv(node_field_get, &phi, x, y, z, k);
        }
  /* open x ends and the jets' x faces: G beyond the boundary is the boundary
   * node's (zero gradient at a nozzle; beside it, the even mirror image that a
   * free-slip wall gives away from the nozzle's edge, taken on every wall row) */
  if (s->wall_x >= 2)
    for (int k = 0; k < 3; ++k)
      for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y) {
          s->G[gidx(s, k, -1, y, z)] = s->G[gidx(s, k, 0, y, z)];
          s->G[gidx(s, k, nx, y, z)] = s->G[gidx(s, k, nx - 1, y, z)];
        }
  /* X_k = - d_k G_k (eq Xalpha, dt = 1) and the mass-fraction gradients */
#pragma omp parallel for schedule(static) if (n >= 512)
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        long node = node_index(s, x, y, z);
        for (int k = 0; k < 3; ++k) {
          g_ctx gc = {s, k};
          s->Xc[(long)k * n + node] = -iso_deriv(g_get, &gc, x, y, z, k);
        }
        for (int a = 0; a < M; ++a) {
          node_field_ctx yc = {s, s->Yf + (long)a * n, -1};
          for (int k = 0; k < 3; ++k)
            s->gY[((long)a * 3 + k) * n + node] = iso_deriv(node_field_get, &yc, x, y, z, k);
        }
      }
}

/* ------------------------------------------------------------------------- */
/* Diffusion velocities, eq transform12                                       */
/* ------------------------------------------------------------------------- */
/* Solve rho_a V_a - 1/2 sum_b K_ab (V_b - V_a) = j_a - rho_a u_s for the three
 * components, u_s being the velocity the species relax towards (the mixture
 * velocity under strong coupling), by Gaussian elimination with partial
 * pivoting on the species present (rho_a != 0). An absent species has an
 * identically zero row and column; its V_a is set to zero. */
static void diffusion_velocities(int M, const state_t *st, double K[MAXM][MAXM],
                                 double V[MAXM][3])
{
  int idx[MAXM], np = 0;
  for (int a = 0; a < M; ++a) {
    for (int k = 0; k < 3; ++k) V[a][k] = 0.0;
    if (st->rho_a[a] != 0.0) idx[np++] = a;
  }
  double A[MAXM][MAXM], rhs[MAXM][3];
  for (int r = 0; r < np; ++r) {
    int a = idx[r];
    for (int c = 0; c < np; ++c) A[r][c] = 0.0;
    A[r][r] += st->rho_a[a];
    for (int c = 0; c < np; ++c) {
      int b = idx[c];
      A[r][c] -= 0.5 * K[a][b];   /* - 1/2 K_ab V_b */
      A[r][r] += 0.5 * K[a][b];   /* + 1/2 K_ab V_a */
    }
    for (int k = 0; k < 3; ++k) rhs[r][k] = st->j_a[a][k] - st->rho_a[a] * st->us[k];
  }
  for (int col = 0; col < np; ++col) {
    int piv = col;
    for (int r = col + 1; r < np; ++r)
      if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
    if (piv != col) {
      for (int c = 0; c < np; ++c) { double t = A[col][c]; A[col][c] = A[piv][c]; A[piv][c] = t; }
      for (int k = 0; k < 3; ++k) { double t = rhs[col][k]; rhs[col][k] = rhs[piv][k]; rhs[piv][k] = t; }
    }
    for (int r = col + 1; r < np; ++r) {
      double f = A[r][col] / A[col][col];
      for (int c = col; c < np; ++c) A[r][c] -= f * A[col][c];
      for (int k = 0; k < 3; ++k) rhs[r][k] -= f * rhs[col][k];
    }
  }
  double sol[MAXM][3];
  for (int r = np - 1; r >= 0; --r)
    for (int k = 0; k < 3; ++k) {
      double acc = rhs[r][k];
      for (int c = r + 1; c < np; ++c) acc -= A[r][c] * sol[c][k];
      sol[r][k] = acc / A[r][r];
    }
  for (int r = 0; r < np; ++r)
    for (int k = 0; k < 3; ++k) V[idx[r]][k] = sol[r][k];
}

/* Stefan--Maxwell rates at a node: 1/tau_ab (eq tauab, R_U = 1), beta_a (Sec. 2.5.2),
 * and K_ab = P X_a X_b / D_ab (eq stefanMaxwellNumerical). */
static void species_rates(const oracle_sim *s, const state_t *st, double inv_tau[MAXM][MAXM],
                          double beta[MAXM], double K[MAXM][MAXM])
{
  const int M = s->M;
  for (int a = 0; a < M; ++a) {
    double inv_tau_a = 0.0;
    for (int b = 0; b < M; ++b) {
      const double Dab = diffusivity(s, a, b, st->T);
      inv_tau[a][b] = (st->T / Dab) * (st->mmix / (s->m[a] * s->m[b]));
      inv_tau_a += st->Y[b] * inv_tau[a][b];             /* eq tau */
      K[a][b] = st->Ps * st->X[a] * st->X[b] / Dab;
    }
    double tau_a = 1.0 / inv_tau_a;
    beta[a] = 1.0 / (2.0 * tau_a + 1.0);
  }
}

/* ------------------------------------------------------------------------- */
/* Collision at one node                                                      */
/* ------------------------------------------------------------------------- */
static int collide_node(oracle_sim *s, long node)
{
  const int M = s->M;
  const long n = s->n;
  state_t st;
  node_state(s, s->pop, node, &st);
  if (!(st.rho > 0.0) || !(st.T > 0.0) || !isfinite(st.T)) return -2;

  /* ---- species, eqs SMlbm, fstar1, transform12 ---- */
  double inv_tau[MAXM][MAXM], beta[MAXM], K[MAXM][MAXM], V[MAXM][3];
  species_rates(s, &st, inv_tau, beta, K);
  diffusion_velocities(M, &st, K, V);
  double feq[MAXM][Q], fstar[MAXM][Q];
  for (int b = 0; b < M; ++b) {
    double RbT = st.T / s->m[b];
    double ub[3] = {st.us[0] + V[b][0], st.us[1] + V[b][1], st.us[2] + V[b][2]};
    double psi_eq[Q], psi_st[Q];
    oracle_psi(st.us, RbT, psi_eq);                         /* eq 27eq  */
    oracle_psi(ub, RbT, psi_st);                            /* eq 27qeq */
    for (int i = 0; i < Q; ++i) {
      feq[b][i] = st.rho_a[b] * psi_eq[i];
      fstar[b][i] = st.rho_a[b] * psi_st[i];
    }
  }
  int nstored = s->keep_slaved ? M : M - 1;
  for (int a = 0; a < nstored; ++a)
    for (int i = 0; i < Q; ++i) {
      double F = 0.0;
      for (int b = 0; b < M; ++b) F += inv_tau[a][b] * (feq[b][i] - fstar[b][i]);
      F *= st.Y[a];
      double f = POP(s, s->pop, a, i, node);
      double fnew = f + 2.0 * beta[a] * (feq[a][i] - f);
      if (!(s->flags & ORACLE_DROP_FSOURCE)) fnew += (beta[a] - 1.0) * F;
      POP(s, s->post, a, i, node) = fnew;
    }

  /* ---- momentum lattice, eqs feq, fwithcorrection, Ai ---- */
  double RT = st.R * st.T;
  double psi_f[Q];
  oracle_psi(st.u, RT, psi_f);
  double X[3];
  for (int k = 0; k < 3; ++k) X[k] = s->Xc[(long)k * n + node];
  double Pf[3][3] = {{0}};
  for (int i = 0; i < Q; ++i) {
    double f = POP(s, s->pop, LAT_F(s), i, node);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) Pf[a][b] += f * cvel(i, a) * cvel(i, b);   /* eq boldP */
    double fnew = f + st.omega * (st.rho * psi_f[i] - f);
    if (!(s->flags & ORACLE_DROP_XCORR))
      for (int k = 0; k < 3; ++k) fnew += A_table(i, k) * X[k];
    POP(s, s->post, LAT_F(s), i, node) = fnew;
  }

  /* ---- energy lattice, eqs g, gieq, gistar ---- */
  double theta = RT;
  double usq = st.u[0] * st.u[0] + st.u[1] * st.u[1] + st.u[2] * st.u[2];
  double q[3] = {0, 0, 0};
  for (int i = 0; i < Q; ++i)
    for (int k = 0; k < 3; ++k) q[k] += POP(s, s->pop, LAT_G(s), i, node) * cvel(i, k);  /* eq q */
  double qeq[3], Peq[9], Req[9];
  for (int a = 0; a < 3; ++a) {
    qeq[a] = (st.H + usq / 2.0) * st.rho * st.u[a];                   /* eq geq1mom */
    for (int b = 0; b < 3; ++b) {
      Peq[3 * a + b] = (a == b ? st.P : 0.0) + st.rho * st.u[a] * st.u[b];  /* eq feq2mom */
      Req[3 * a + b] = (st.H + usq / 2.0) * Peq[3 * a + b] + st.P * st.u[a] * st.u[b]; /* eq geq2mom */
    }
  }
  if (st.omega == st.omega1) return -5;
  double qdiff[3], qcorr[3], qstar[3];
  for (int k = 0; k < 3; ++k) {
    double sdiff = 0.0, scorr = 0.0;
    for (int a = 0; a < M; ++a) {
      sdiff += st.Ha[a] * st.Y[a] * V[a][k];
      scorr += st.Ha[a] * s->gY[((long)a * 3 + k) * n + node];
    }
    qdiff[k] = (st.omega1 / (st.omega - st.omega1)) * st.rho * sdiff;          /* eq interdiffusion */
    qcorr[k] = 0.5 * ((st.omega1 - 2.0) / (st.omega1 - st.omega)) * st.P * scorr; /* eq corrFourier */
    double upneq = 0.0;
    for (int b = 0; b < 3; ++b) upneq += st.u[b] * (Pf[b][k] - Peq[3 * b + k]);
    qstar[k] = q[k];                                                            /* eq gstareq1mom */
    if (!(s->flags & ORACLE_DROP_UPNEQ)) qstar[k] -= upneq;
    if (!(s->flags & ORACLE_DROP_QDIFF)) qstar[k] += qdiff[k];
    if (!(s->flags & ORACLE_DROP_QCORR)) qstar[k] += qcorr[k];
  }
  double geq[Q], gstar[Q];
  oracle_gansatz(theta, st.rhoE, qeq, Req, geq);
  oracle_gansatz(theta, st.rhoE, qstar, Req, gstar);
  for (int i = 0; i < Q; ++i) {
    double g = POP(s, s->pop, LAT_G(s), i, node);
    POP(s, s->post, LAT_G(s), i, node) =
        g + st.omega1 * (geq[i] - g) + (st.omega - st.omega1) * (gstar[i] - g);
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Time step                                                                  */
/* ------------------------------------------------------------------------- */
static void stream(oracle_sim *s)
{
  const int nx = s->nx, ny = s->ny, nz = s->nz;
  const int L = s->M + 2;
  /* every destination slot is written by exactly one source: any split of the
   * loops over threads is free of races */
#pragma omp parallel for collapse(2) schedule(static) if (s->n >= 512)
  for (int z = 0; z < nz; ++z)
    for (int l = 0; l < L; ++l) {
      if (l == s->M - 1 && !s->keep_slaved) continue;
      for (int i = 0; i < Q; ++i)
        for (int y = 0; y < ny; ++y)
          for (int x = 0; x < nx; ++x) {
            long src = node_index(s, x, y, z);
            double v = POP(s, s->post, l, i, src);
            int xd = x + cvel(i, 0);
            int yd = y + cvel(i, 1);
            if (s->wall_y == 2 && (yd < 0 || yd >= ny)) {
              /* outlets: leaves the domain */
            } else if (s->wall_x == 3 && (xd < 0 || xd >= nx)) {
              /* jets: reflected specularly (c_x reversed, at the same x) into a
               * row beside the nozzles (a free-slip wall); into a nozzle row it
               * leaves the domain (the inlet supplies what enters there) */
              if (!nozzle_row(s, yd)) {
                int ix = i - 9 * 2 * cvel(i, 0);
                long dst = node_index(s, x, yd, wrap(z + cvel(i, 2), nz));
                POP(s, s->pop, l, ix, dst) = v;
              }
            } else if (s->wall_x == 2 && (xd < 0 || xd >= nx)) {
              /* open x ends: leaves the domain */
            } else if (s->wall_x && (xd < 0 || xd >= nx)) {
              POP(s, s->pop, l, opposite(i), src) = v;      /* half-way bounce-back */
            } else if (s->wall_y && (yd < 0 || yd >= ny)) {
              /* free-slip y wall: specular reflection, c_y reversed, at the same y */
              int iy = i + 3 * (-2 * cvel(i, 1));
              long dst = node_index(s, wrap(xd, nx), y, wrap(z + cvel(i, 2), nz));
              POP(s, s->pop, l, iy, dst) = v;
            } else {
              long dst = node_index(s, wrap(xd, nx), wrap(y + cvel(i, 1), ny),
                                    wrap(z + cvel(i, 2), nz));
              POP(s, s->pop, l, i, dst) = v;
            }
          }
    }
  if (s->wall_x == 3) {
    /* outlets at the y ends: what enters a boundary row from beyond comes from a
     * ghost row holding the boundary row's post-collision state (zero gradient;
     * beyond an x face too, the nearest boundary node's) */
    for (int z = 0; z < nz; ++z)
      for (int l = 0; l < L; ++l) {
        if (l == s->M - 1 && !s->keep_slaved) continue;
        for (int i = 0; i < Q; ++i) {
          const int cy = cvel(i, 1);
          if (!cy) continue;
          const int yb = cy > 0 ? 0 : ny - 1;
          for (int x = 0; x < nx; ++x) {
            int xs = x - cvel(i, 0);
            xs = xs < 0 ? 0 : (xs >= nx ? nx - 1 : xs);
            POP(s, s->pop, l, i, node_index(s, x, yb, z)) =
                POP(s, s->post, l, i, node_index(s, xs, yb, wrap(z - cvel(i, 2), nz)));
          }
        }
      }
    /* nozzles: what enters from beyond is the inlet equilibrium of that jet */
    for (int z = 0; z < nz; ++z)
      for (int l = 0; l < L; ++l) {
        if (l == s->M - 1 && !s->keep_slaved) continue;
        for (int i = 0; i < Q; ++i)
          for (int y = s->ny0; y < s->ny1; ++y) {
            if (cvel(i, 0) > 0) POP(s, s->pop, l, i, node_index(s, 0, y, z)) = s->fin[l][i];
            if (cvel(i, 0) < 0) POP(s, s->pop, l, i, node_index(s, nx - 1, y, z)) = s->fin2[l][i];
          }
      }
  }
  if (s->wall_x == 2) {
    /* open x ends: what enters node 0 from outside is the inlet equilibrium; what
     * enters node nx-1 from outside comes from a ghost beyond it that holds the
     * boundary node's post-collision state (zero gradient) */
    for (int z = 0; z < nz; ++z)
      for (int l = 0; l < L; ++l) {
        if (l == s->M - 1 && !s->keep_slaved) continue;
        for (int i = 0; i < Q; ++i)
          for (int y = 0; y < ny; ++y) {
            if (cvel(i, 0) > 0) POP(s, s->pop, l, i, node_index(s, 0, y, z)) = s->fin[l][i];
            if (cvel(i, 0) < 0)
              POP(s, s->pop, l, i, node_index(s, nx - 1, y, z)) =
                  POP(s, s->post, l, i, node_index(s, nx - 1, wrap(y - cvel(i, 1), ny), wrap(z - cvel(i, 2), nz)));
          }
      }
  }
}

static int one_step(oracle_sim *s)
{
  const long n = s->n;
  const int M = s->M;
  int bad = 0;
  /* 1-2: moments and the node fields needed by the non-local terms */
#pragma omp parallel for schedule(static) reduction(| : bad) if (n >= 512)
  for (long node = 0; node < n; ++node) {
    state_t st;
    node_state(s, s->pop, node, &st);
    if (!(st.rho > 0.0) || !(st.T > 0.0) || !isfinite(st.T)) bad |= 1;
    double RT = st.R * st.T;
    for (int k = 0; k < 3; ++k) {
      double ru = st.rho * st.u[k];
      s->Phi[(long)k * n + node] = ru * (1.0 - 3.0 * RT) - st.rho * st.u[k] * st.u[k] * st.u[k];
    }
    s->om[node] = st.omega;
    for (int a = 0; a < M; ++a) s->Yf[(long)a * n + node] = st.Y[a];
  }
  if (bad) return -2;
  /* 3: non-local terms at the same time level */
  compute_nonlocal(s);
  /* 4-6: collisions */
  int rc = 0;
#pragma omp parallel for schedule(static) reduction(min : rc) if (n >= 512)
  for (long node = 0; node < n; ++node) {
    int r = collide_node(s, node);
    if (r < rc) rc = r;
  }
  if (rc) return rc;
  /* 7: streaming */
  stream(s);
  return 0;
}

int oracle_step(oracle_sim *s, int64_t nsteps)
{
  if (!s || nsteps < 0) return -1;
  for (int64_t t = 0; t < nsteps; ++t) {
    int rc = one_step(s);
    if (rc) return rc;
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Initialisation and read-back                                               */
/* ------------------------------------------------------------------------- */
/* Populations of every lattice at the local equilibrium of (X, p, T, u) at one
 * node, written through put(l, i, value). Returns 0, 1 for invalid fields, 2 for
 * an infeasible state (R_a T + u^2 >= 1). */
static int local_equilibrium(const oracle_sim *s, const double *Xa, double Pn, double Tn, const double uu[3],
                             double out[][Q])
{
  const int M = s->M;
  int bad = 0;
  double mmix = 0.0, xsum = 0.0;
  for (int a = 0; a < M; ++a) {
    mmix += Xa[a] * s->m[a];                 /* m = sum X_a m_a, equivalent to eq meanMolecularWeight */
    xsum += Xa[a];
    if (Xa[a] < 0.0) bad = 1;
  }
  if (fabs(xsum - 1.0) > 1e-12) bad = 1;
  if (!(Tn > 0.0) || !(Pn > 0.0)) return 1;
  double usq = uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2];
  double R = 1.0 / mmix;
  double rho = Pn / (R * Tn);                /* eq eosIdealGas */
  double Y[MAXM], Cv = 0.0, Cp = 0.0;
  for (int a = 0; a < M; ++a) {
    Y[a] = Xa[a] * s->m[a] / mmix;           /* eq moleFractionDefinition */
    Cv += Y[a] * s->cv[a];
    Cp += Y[a] * (s->cv[a] + 1.0 / s->m[a]);
  }
  double rhoE = rho * (Cv * Tn + usq / 2.0);
  double H = Cp * Tn;
  if (s->cvt) {                              /* eqs Umix, specH with U_a(T) */
    double U = 0.0;
    for (int a = 0; a < M; ++a) U += Y[a] * species_U(s, a, Tn);
    rhoE = rho * (U + usq / 2.0);
    H = U + R * Tn;
  }
  double psi[Q];
  for (int a = 0; a < M; ++a) {
    if (a == M - 1 && !s->keep_slaved) continue;
    double RaT = Tn / s->m[a];
    if (!(RaT + usq < 1.0)) bad = 2;
    oracle_psi(uu, RaT, psi);
    for (int i = 0; i < Q; ++i) out[a][i] = rho * Y[a] * psi[i];
  }
  oracle_psi(uu, R * Tn, psi);
  for (int i = 0; i < Q; ++i) out[LAT_F(s)][i] = rho * psi[i];
  double qeq[3], Req[9];
  for (int a = 0; a < 3; ++a) {
    qeq[a] = (H + usq / 2.0) * rho * uu[a];
    for (int b = 0; b < 3; ++b) {
      double Peq = (a == b ? Pn : 0.0) + rho * uu[a] * uu[b];
      Req[3 * a + b] = (H + usq / 2.0) * Peq + Pn * uu[a] * uu[b];
    }
  }
  oracle_gansatz(R * Tn, rhoE, qeq, Req, out[LAT_G(s)]);
  return bad;
}

int oracle_init_fields(oracle_sim *s, const double *X, const double *p, const double *T,
                       const double *u)
{
  if (!s || !X || !p || !T || !u) return -1;
  const int M = s->M;
  const long n = s->n;
  int bad = 0;
  memset(s->pop, 0, sizeof(double) * (size_t)(M + 2) * Q * n);
  for (long node = 0; node < n; ++node) {
    double Xa[MAXM], eq[MAXM + 2][Q];
    memset(eq, 0, sizeof(eq));
    for (int a = 0; a < M; ++a) Xa[a] = X[(long)a * n + node];
    double uu[3] = {u[node], u[n + node], u[2 * n + node]};
    int b = local_equilibrium(s, Xa, p[node], T[node], uu, eq);
    if (b > bad) bad = b;
    if (b == 1) continue;
    for (int l = 0; l < M + 2; ++l)
      for (int i = 0; i < Q; ++i) POP(s, s->pop, l, i, node) = eq[l][i];
  }
  if (bad == 2) return -2;
  return bad ? -1 : 0;
}

int oracle_read_moments(oracle_sim *s, double *X, double *rho, double *u, double *p, double *T)
{
  if (!s) return -1;
  const long n = s->n;
  for (long node = 0; node < n; ++node) {
    state_t st;
    node_state(s, s->pop, node, &st);
    if (X)
      for (int a = 0; a < s->M; ++a) X[(long)a * n + node] = st.X[a];
    if (rho) rho[node] = st.rho;
    if (u)
      for (int k = 0; k < 3; ++k) u[(long)k * n + node] = st.u[k];
    if (p) p[node] = st.P;
    if (T) T[node] = st.T;
  }
  return 0;
}

int oracle_conservation(oracle_sim *s, double *out)
{
  if (!s || !out) return -1;
  const int M = s->M;
  for (int k = 0; k < M + 5; ++k) out[k] = 0.0;
  for (long node = 0; node < s->n; ++node) {
    state_t st;
    node_state(s, s->pop, node, &st);
    for (int a = 0; a < M; ++a) out[a] += st.rho_a[a];
    out[M] += st.rho;
    for (int k = 0; k < 3; ++k) out[M + 1 + k] += st.j[k];
    out[M + 4] += st.rhoE;
  }
  return 0;
}

int oracle_get_populations(const oracle_sim *s, double *out)
{
  if (!s || !out) return -1;
  memcpy(out, s->pop, sizeof(double) * (size_t)(s->M + 2) * Q * s->n);
  return 0;
}

int oracle_set_populations(oracle_sim *s, const double *in)
{
  if (!s || !in) return -1;
  memcpy(s->pop, in, sizeof(double) * (size_t)(s->M + 2) * Q * s->n);
  return 0;
}

int oracle_node_info_at(oracle_sim *s, int32_t x, int32_t y, int32_t z, oracle_node_info *out)
{
  if (!s || !out || x < 0 || y < 0 || z < 0 || x >= s->nx || y >= s->ny || z >= s->nz) return -1;
  long node = node_index(s, x, y, z);
  state_t st;
  node_state(s, s->pop, node, &st);
  memset(out, 0, sizeof(*out));
  out->rho = st.rho;
  for (int k = 0; k < 3; ++k) out->u[k] = st.u[k];
  out->rhoE = st.rhoE; out->T = st.T; out->P = st.P; out->R = st.R;
  out->Cv = st.Cv; out->Cp = st.Cp; out->H = st.H;
  out->mu = st.mu; out->lambda = st.lam; out->omega = st.omega; out->omega1 = st.omega1;
  double inv_tau[MAXM][MAXM], beta[MAXM], K[MAXM][MAXM], V[MAXM][3];
  species_rates(s, &st, inv_tau, beta, K);
  diffusion_velocities(s->M, &st, K, V);
  for (int a = 0; a < s->M; ++a) {
    out->rho_a[a] = st.rho_a[a];
    out->Y[a] = st.Y[a];
    out->X[a] = st.X[a];
    out->beta[a] = beta[a];
    for (int k = 0; k < 3; ++k) {
      out->j_a[a][k] = st.j_a[a][k];
      out->V[a][k] = V[a][k];
    }
    for (int b = 0; b < s->M; ++b) out->K[a][b] = K[a][b];
  }
  return 0;
}
