/*
 * mclbm_oracle.h -- plain FP64 CPU oracle of the M+2-lattice mixture lattice
 * Boltzmann step of Sawant, Dorschner and Karlin, "Consistent lattice Boltzmann
 * model for multicomponent mixtures" (arXiv 2004.11286).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load this library. It shares no code with the GPU
 * library (this header is written independently of include/mclbm.h).
 *
 * Lattice units throughout: dt = dx = 1, universal gas constant R_U = 1,
 * constant specific heats with reference temperature T_0 = 0 (Sec. 4.1).
 * All arrays are structure-of-arrays with x fastest: node n = x + nx*(y + ny*z).
 * Every function returns 0 on success and a negative code on error
 * (-1 bad argument, -2 infeasible state, -5 the omega == omega_1 pole of the
 * printed energy quasi-equilibrium).
 */
#ifndef MCLBM_ORACLE_H
#define MCLBM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_MAXM 8

/* Planted-mistake switches, used only by tests that show a pin catches them. */
enum {
  ORACLE_DROP_QDIFF = 1,      /* omit the interdiffusion energy flux (eq interdiffusion) */
  ORACLE_DROP_QCORR = 2,      /* omit the correction flux (eq corrFourier)               */
  ORACLE_DROP_XCORR = 4,      /* omit the A_i . X isotropy correction (eq fwithcorrection) */
  ORACLE_DROP_UPNEQ = 8,      /* omit -u.(P - P^eq) in the quasi-equilibrium flux         */
  ORACLE_DROP_FSOURCE = 16,   /* omit the (beta_a - 1) F_ai term (eq SMlbm)               */
  ORACLE_WEAK_MIXTURE_U = 32, /* weak coupling: species relax towards the momentum lattice's u */
  ORACLE_WEAK_MIXTURE_P = 64, /* weak coupling: friction K_ab with the momentum lattice's P  */
  ORACLE_CVT_HA_CPT = 128     /* polynomial C_v: H_a = C_{a,p}(T) T, not the integral of eq specHa */
};

typedef struct {
  int32_t M;            /* number of species, 2..8                                      */
  int32_t nx, ny, nz;   /* lattice size                                                 */
  int32_t wall_x;       /* 0 periodic in x; 1 half-way bounce-back walls at both x ends;
                           2 open x ends: equilibrium inlet at x = 0 (fields `inlet`),
                           zero-gradient outlet at x = nx - 1;
                           3 opposed jets (Sec. 4.3): on both x faces the rows
                           nozzle_y0 <= y < nozzle_y1 are equilibrium inlets (`inlet`
                           at x = 0, `inlet_right` at x = nx - 1), the other rows
                           free-slip walls (specular reflection); needs wall_y = 2 */
  int32_t keep_slaved;  /* 1: store and evolve the slaved species' lattice literally    */
  int32_t debug_flags;  /* ORACLE_DROP_* planted mistakes (tests only), else 0          */
  int32_t weak;         /* 1: weak coupling (Sec. 3.5.1): all M species lattices evolve
                           with their own conservation laws (implies keep_slaved)     */
  const double *molar_mass; /* [M] molar masses m_a                                     */
  const double *cv;         /* [M] mass-based constant specific heats C_{a,v}           */
  const double *D;          /* [M*M] symmetric binary diffusivities, diagonal included  */
  const double *mu;         /* [M] species dynamic viscosities                          */
  const double *lambda;     /* [M] species thermal conductivities                       */
  const double *cv_coef;    /* NULL: constant cv; else [M][4]: C_{a,v}(T) = sum_k c_k T^k,
                               c_0 > 0, c_k >= 0 (cv is then not used)                  */
  const double *inlet;      /* wall_x = 2: [M+5] inlet fields X (M), p, T, u (3)        */
  const double *transport_exp; /* NULL: constant transport coefficients; else [2M+2]:
                               s_mu (M), s_lam (M), s_D, T_ref: mu_a (T/T_ref)^s_mu,a,
                               lambda_a (T/T_ref)^s_lam,a, D_ab (T/T_ref)^s_D          */
  int32_t wall_y;           /* 1: free-slip walls at both y ends (specular reflection);
                               needs ny >= 2 and wall_x 0 or 1. 2: zero-gradient outlets
                               at both y ends (what enters from beyond is the boundary
                               node's post-collision state); only with wall_x = 3       */
  int32_t reserved2;
  const double *inlet_right; /* wall_x = 3: [M+5] fields of the jet entering at x = nx - 1 */
  int32_t nozzle_y0, nozzle_y1; /* wall_x = 3: nozzle rows, 1 <= y0 < y1 <= ny - 1          */
} oracle_params;

typedef struct oracle_sim oracle_sim;

/* Per-node diagnostic record of the macroscopic state (Secs. 2.5, 3.1-3.4). */
typedef struct {
  double rho, u[3], rhoE, T, P, R, Cv, Cp, H;
  double mu, lambda, omega, omega1;
  double rho_a[ORACLE_MAXM], Y[ORACLE_MAXM], X[ORACLE_MAXM];
  double j_a[ORACLE_MAXM][3];
  double beta[ORACLE_MAXM];
  double V[ORACLE_MAXM][3];            /* diffusion velocities from eq transform12 */
  double K[ORACLE_MAXM][ORACLE_MAXM];  /* P X_a X_b / D_ab                          */
} oracle_node_info;

int  oracle_create(const oracle_params *p, oracle_sim **out);
void oracle_destroy(oracle_sim *s);
/* X [M][n] mole fractions, p [n] pressure, T [n] temperature, u [3][n] velocity. */
int  oracle_init_fields(oracle_sim *s, const double *X, const double *p,
                        const double *T, const double *u);
int  oracle_step(oracle_sim *s, int64_t nsteps);
/* X [M][n], rho [n], u [3][n], p [n], T [n]; any output pointer may be NULL. */
int  oracle_read_moments(oracle_sim *s, double *X, double *rho, double *u,
                         double *p, double *T);
/* out [M+5]: total rho_1..rho_M, rho, rho u_x, rho u_y, rho u_z, rho E. */
int  oracle_conservation(oracle_sim *s, double *out);
/* Populations, [(M+2)][27][n]: species 1..M, then momentum f, then energy g. */
int  oracle_get_populations(const oracle_sim *s, double *out);
int  oracle_set_populations(oracle_sim *s, const double *in);
int  oracle_node_info_at(oracle_sim *s, int32_t x, int32_t y, int32_t z,
                         oracle_node_info *out);
int  oracle_set_threads(int32_t nthreads);     /* <= 0: leave OpenMP's default */
int  oracle_threads(void);

/* Building blocks, exported so tests can pin them against the paper. */
void oracle_velocities(int32_t c[27 * 3]);
void oracle_psi(const double xi[3], double zeta, double out[27]);           /* eq prod    */
void oracle_weights(double theta, double out[27]);                          /* eq weights */
void oracle_gansatz(double theta, double M0, const double m[3],
                    const double Mt[9], double out[27]);                    /* eq gansatz */
void oracle_tables(double A[27 * 3], double B[27 * 3]);                     /* eqs Ai, Bi */
/* Isotropic gradient of a periodic scalar field on an nx*ny*nz grid. */
int  oracle_gradient(int32_t nx, int32_t ny, int32_t nz, const double *phi,
                     double *grad /* [3][n] */);

#ifdef __cplusplus
}
#endif
#endif
