/*
 * sanitize_main.c -- TEST INFRASTRUCTURE: a small driver that runs the FP64
 * oracle through every boundary, coupling and property mode on ragged grids,
 * built with AddressSanitizer and UndefinedBehaviorSanitizer (make sanitize) so
 * that an out-of-bounds access, a use after free or undefined arithmetic in the
 * oracle ends the run with a report. It checks that every call succeeds, that
 * every field stays finite and that mass is conserved where no open end feeds
 * or drains the domain. Exit status 0 on success.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mclbm_oracle.h"

static int fail(const char *what, int rc)
{
  fprintf(stderr, "sanitize: %s failed (%d)\n", what, rc);
  return 1;
}

/* One case: M species on nx x ny x nz, a composition step along x, a small
 * shear velocity, nsteps steps; returns 0 on success. */
static int run_case(int M, int nx, int ny, int nz, int wall_x, int wall_y, int weak, int cvt, int trn,
                    int nsteps)
{
  const int n = nx * ny * nz;
  double m[ORACLE_MAXM], cv[ORACLE_MAXM], mu[ORACLE_MAXM], lam[ORACLE_MAXM];
  double D[ORACLE_MAXM * ORACLE_MAXM], cvc[ORACLE_MAXM * 4], tex[2 * ORACLE_MAXM + 2], inlet[ORACLE_MAXM + 5];
  const double masses[4] = {2.0, 16.0, 28.0, 40.0};
  const double T0 = 0.3;
  for (int a = 0; a < M; ++a) {
    m[a] = masses[a];
    cv[a] = 1.5 / m[a];
    mu[a] = 0.02;
    lam[a] = 0.05;
    for (int k = 0; k < 4; ++k) cvc[4 * a + k] = k == 0 ? cv[a] : cv[a] * 0.1 * (a + 1) / pow(T0, k);
    tex[a] = 0.7;
    tex[M + a] = 0.8;
    for (int b = 0; b < M; ++b) D[a * M + b] = 0.03 + 0.01 * (a + b);
  }
  tex[2 * M] = 1.75;
  tex[2 * M + 1] = T0 / 1.2;
  double *X = calloc((size_t)M * n, sizeof(double)), *p = calloc(n, sizeof(double));
  double *T = calloc(n, sizeof(double)), *u = calloc(3 * (size_t)n, sizeof(double));
  double *Xo = calloc((size_t)M * n, sizeof(double)), *rho = calloc(n, sizeof(double));
  double *uo = calloc(3 * (size_t)n, sizeof(double)), *po = calloc(n, sizeof(double));
  double *To = calloc(n, sizeof(double));
  double c0[ORACLE_MAXM + 5], c1[ORACLE_MAXM + 5];
  int rc = 0, bad = 0;
  if (!X || !p || !T || !u || !Xo || !rho || !uo || !po || !To) { bad = fail("calloc", -1); goto done; }
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const int i = x + nx * (y + ny * z);
        const double left = x < nx / 2 ? 1.0 : 0.0;
        double s = 0.0;
        for (int a = 0; a < M; ++a) {
          X[(size_t)a * n + i] = 0.1 + 0.2 * (a + 1) * (left ? 1.0 : 0.5) + 0.05 * a;
          s += X[(size_t)a * n + i];
        }
        for (int a = 0; a < M; ++a) X[(size_t)a * n + i] /= s;
        p[i] = 0.02;
        T[i] = T0;
        u[i] = wall_x == 2 ? 0.03 : 0.0;
        u[(size_t)2 * n + i] = 0.01 * sin(6.283185307179586 * y / ny);
      }
  for (int a = 0; a < M; ++a) inlet[a] = X[(size_t)a * n];
  inlet[M] = 0.02;
  inlet[M + 1] = T0;
  inlet[M + 2] = 0.03;
  inlet[M + 3] = inlet[M + 4] = 0.0;
  oracle_params P;
  memset(&P, 0, sizeof P);
  P.M = M;
  P.nx = nx;
  P.ny = ny;
  P.nz = nz;
  P.wall_x = wall_x;
  P.wall_y = wall_y;
  P.weak = weak;
  P.molar_mass = m;
  P.cv = cv;
  P.D = D;
  P.mu = mu;
  P.lambda = lam;
  P.cv_coef = cvt ? cvc : NULL;
  P.transport_exp = trn ? tex : NULL;
  P.inlet = wall_x == 2 ? inlet : NULL;
  oracle_sim *sim = NULL;
  if ((rc = oracle_create(&P, &sim))) { bad = fail("oracle_create", rc); goto done; }
  if ((rc = oracle_init_fields(sim, X, p, T, u))) { bad = fail("oracle_init_fields", rc); goto out; }
  if ((rc = oracle_conservation(sim, c0))) { bad = fail("oracle_conservation", rc); goto out; }
  if ((rc = oracle_step(sim, nsteps))) { bad = fail("oracle_step", rc); goto out; }
  if ((rc = oracle_read_moments(sim, Xo, rho, uo, po, To))) { bad = fail("oracle_read_moments", rc); goto out; }
  if ((rc = oracle_conservation(sim, c1))) { bad = fail("oracle_conservation", rc); goto out; }
  for (int i = 0; i < n; ++i) {
    double v = rho[i] + po[i] + To[i] + uo[i] + uo[n + i] + uo[2 * n + i];
    for (int a = 0; a < M; ++a) v += Xo[(size_t)a * n + i];
    if (!isfinite(v)) { bad = fail("finite fields", i); goto out; }
  }
  if (wall_x != 2 && fabs(c1[M] / c0[M] - 1.0) > 1e-12) { bad = fail("mass conservation", -1); goto out; }
out:
  oracle_destroy(sim);
done:
  free(X); free(p); free(T); free(u); free(Xo); free(rho); free(uo); free(po); free(To);
  if (!bad) printf("ok M=%d %dx%dx%d wall_x=%d wall_y=%d weak=%d cvt=%d trn=%d\n", M, nx, ny, nz, wall_x, wall_y, weak, cvt, trn);
  return bad;
}

int main(void)
{
  int bad = 0;
  oracle_set_threads(2);
  for (int M = 2; M <= 4; ++M)
    for (int wx = 0; wx <= 2; ++wx)
      for (int wy = 0; wy <= (wx < 2 ? 1 : 0); ++wy)
        for (int weak = 0; weak <= 1; ++weak)
          for (int props = 0; props <= 1; ++props)
            bad |= run_case(M, 7, 5, 3, wx, wy, weak, props, props, 6);
  /* single-node cross-sections and the smallest grids */
  bad |= run_case(3, 9, 1, 1, 1, 0, 0, 0, 0, 10);
  bad |= run_case(2, 2, 2, 1, 2, 0, 1, 1, 1, 10);
  bad |= run_case(2, 1, 1, 1, 0, 0, 0, 0, 0, 3);
  if (!bad) printf("sanitize: all cases ok\n");
  return bad;
}
