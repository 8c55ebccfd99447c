/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg may load
 * this file's library. The product path never calls it.
 *
 * Plain, untiled, loop-by-loop FP64 definition of the 3D compressible
 * Navier-Stokes proxy: the class of code the paper runs as OpenSBLI's
 * Taylor-Green vortex case (Section 5.1: compressible Navier-Stokes, a
 * third-order Runge-Kutta scheme without adaptive step, no reductions in the
 * bulk of the computation).  The concrete scheme is a textbook one written
 * for this proxy; constants are readings:
 *   - conserved q = (rho, rho u, rho v, rho w, rho E); ideal gas gamma = 1.4;
 *     nondimensional p = rho T / (gamma M^2) with M = 0.1; mu = 1/Re (Re =
 *     1600 unless set), heat conductivity mu / ((gamma-1) M^2 Pr), Pr = 0.71;
 *   - first derivative: 4th-order central, D f = (8 (f[+1]-f[-1]) - (f[+2]-f[-2])) / (12 h);
 *   - viscous and heat fluxes from stored first derivatives of u, v, w and T,
 *     differentiated again (reach 2 + 2 = 4 = the halo);
 *   - R(q) = - sum_a D_a(F_a), F_a = convective - viscous flux along axis a;
 *   - 2N-storage RK3 (Williamson): dq = A_s dq + dt R; q = q + B_s dq with
 *     A = (0, -5/9, -153/128), B = (1/3, 15/16, 8/15);
 *   - x and y periodic, z bounded by mirror walls (rho w odd, the rest even),
 *     or periodic in z (a test option).
 * Domain [0, 2 pi]^3, n cell-centred points per axis, halo 4.
 * Build: gcc -O2 -ffp-contract=off -fopenmp.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NH 4
#define GAMMA 1.4
#define MACH 0.1
#define PRANDTL 0.71
#define TWO_PI 6.283185307179586  /* the double nearest 2 pi */

enum {
  Q_R, Q_RU, Q_RV, Q_RW, Q_RE,          /* conserved */
  D_R, D_RU, D_RV, D_RW, D_RE,          /* RK increments */
  P_R, P_U, P_V, P_W, P_P,              /* primitives */
  G_UX, G_UY, G_UZ, G_VX, G_VY, G_VZ, G_WX, G_WY, G_WZ, G_TX, G_TY, G_TZ, /* gradients */
  NF_NS
};

typedef struct {
  int n;
  long s1, s2;  /* strides of y and z */
  double h, mu, kappa;
  int periodic_z;
  double *f[NF_NS];
} ns_state;

#define IDX(s, i, j, k) ((long)((k) + NH) * (s)->s2 + (long)((j) + NH) * (s)->s1 + ((i) + NH))
#define F(s, fld, i, j, k) ((s)->f[fld][IDX(s, i, j, k)])

ns_state *ns_create(int n, double re) {
  ns_state *s = (ns_state *)calloc(1, sizeof(ns_state));
  s->n = n;
  s->s1 = n + 2 * NH;
  s->s2 = s->s1 * (n + 2 * NH);
  s->h = TWO_PI / n;
  s->mu = 1.0 / re;
  s->kappa = s->mu / (((GAMMA - 1.0) * (MACH * MACH)) * PRANDTL);
  for (int f = 0; f < NF_NS; f++)
    s->f[f] = (double *)calloc((size_t)(s->s2 * (n + 2 * NH)), sizeof(double));
  return s;
}

void ns_destroy(ns_state *s) {
  for (int f = 0; f < NF_NS; f++) free(s->f[f]);
  free(s);
}

double *ns_field(ns_state *s, int f) { return s->f[f]; }
void ns_set_periodic_z(ns_state *s, int on) { s->periodic_z = on; }
double ns_mu(ns_state *s) { return s->mu; }

/* conserved from primitives over the interior */
void ns_init(ns_state *s) {
  const int n = s->n;
#pragma omp parallel for
  for (int k = 0; k < n; k++)
    for (int j = 0; j < n; j++)
      for (int i = 0; i < n; i++) {
        double r = F(s, P_R, i, j, k), u = F(s, P_U, i, j, k), v = F(s, P_V, i, j, k);
        double w = F(s, P_W, i, j, k), p = F(s, P_P, i, j, k);
        F(s, Q_R, i, j, k) = r;
        F(s, Q_RU, i, j, k) = r * u;
        F(s, Q_RV, i, j, k) = r * v;
        F(s, Q_RW, i, j, k) = r * w;
        F(s, Q_RE, i, j, k) = p / (GAMMA - 1.0) + 0.5 * r * ((u * u + v * v) + w * w);
      }
}

/* halos of the conserved variables: x then y periodic (y over the x halo too),
 * then z mirror (or periodic) over the full x-y extent */
static void halos(ns_state *s) {
  const int n = s->n;
#pragma omp parallel for
  for (int k = 0; k < n; k++)
    for (int j = 0; j < n; j++)
      for (int m = 0; m < NH; m++)
        for (int f = Q_R; f <= Q_RE; f++) {
          F(s, f, -NH + m, j, k) = F(s, f, -NH + m + n, j, k);
          F(s, f, n + m, j, k) = F(s, f, m, j, k);
        }
#pragma omp parallel for
  for (int k = 0; k < n; k++)
    for (int m = 0; m < NH; m++)
      for (int i = -NH; i < n + NH; i++)
        for (int f = Q_R; f <= Q_RE; f++) {
          F(s, f, i, -NH + m, k) = F(s, f, i, -NH + m + n, k);
          F(s, f, i, n + m, k) = F(s, f, i, m, k);
        }
  for (int m = 0; m < NH; m++)
#pragma omp parallel for
    for (int j = -NH; j < n + NH; j++)
      for (int i = -NH; i < n + NH; i++)
        for (int f = Q_R; f <= Q_RE; f++) {
          if (s->periodic_z) {
            F(s, f, i, j, -1 - m) = F(s, f, i, j, n - 1 - m);
            F(s, f, i, j, n + m) = F(s, f, i, j, m);
          } else {
            const double sg = f == Q_RW ? -1.0 : 1.0;
            F(s, f, i, j, -1 - m) = sg * F(s, f, i, j, m);
            F(s, f, i, j, n + m) = sg * F(s, f, i, j, n - 1 - m);
          }
        }
}

/* primitives everywhere (interior and halo) */
static void primitives(ns_state *s) {
  const int n = s->n;
#pragma omp parallel for
  for (int k = -NH; k < n + NH; k++)
    for (int j = -NH; j < n + NH; j++)
      for (int i = -NH; i < n + NH; i++) {
        double r = F(s, Q_R, i, j, k);
        double u = F(s, Q_RU, i, j, k) / r, v = F(s, Q_RV, i, j, k) / r, w = F(s, Q_RW, i, j, k) / r;
        F(s, P_R, i, j, k) = r;
        F(s, P_U, i, j, k) = u;
        F(s, P_V, i, j, k) = v;
        F(s, P_W, i, j, k) = w;
        F(s, P_P, i, j, k) =
            (GAMMA - 1.0) * (F(s, Q_RE, i, j, k) - 0.5 * ((F(s, Q_RU, i, j, k) * u + F(s, Q_RV, i, j, k) * v) +
                                                        F(s, Q_RW, i, j, k) * w));
      }
}

/* temperature from the primitives at a point */
static double temp(ns_state *s, int i, int j, int k) {
  return ((GAMMA * (MACH * MACH)) * F(s, P_P, i, j, k)) / F(s, P_R, i, j, k);
}

/* fourth-order first derivative along axis a of a function g(i,j,k) */
#define DERIV(expr_m2, expr_m1, expr_p1, expr_p2, inv) \
  ((8.0 * ((expr_p1) - (expr_m1)) - ((expr_p2) - (expr_m2))) * (inv))

static void gradients(ns_state *s) {
  const int n = s->n;
  const double inv = 1.0 / (12.0 * s->h);
#pragma omp parallel for
  for (int k = -2; k < n + 2; k++)
    for (int j = -2; j < n + 2; j++)
      for (int i = -2; i < n + 2; i++) {
        const int vel[3] = {P_U, P_V, P_W};
        for (int c = 0; c < 3; c++) {
          const int f = vel[c];
          F(s, G_UX + 3 * c, i, j, k) = DERIV(F(s, f, i - 2, j, k), F(s, f, i - 1, j, k), F(s, f, i + 1, j, k), F(s, f, i + 2, j, k), inv);
          F(s, G_UX + 3 * c + 1, i, j, k) = DERIV(F(s, f, i, j - 2, k), F(s, f, i, j - 1, k), F(s, f, i, j + 1, k), F(s, f, i, j + 2, k), inv);
          F(s, G_UX + 3 * c + 2, i, j, k) = DERIV(F(s, f, i, j, k - 2), F(s, f, i, j, k - 1), F(s, f, i, j, k + 1), F(s, f, i, j, k + 2), inv);
        }
        F(s, G_TX, i, j, k) = DERIV(temp(s, i - 2, j, k), temp(s, i - 1, j, k), temp(s, i + 1, j, k), temp(s, i + 2, j, k), inv);
        F(s, G_TY, i, j, k) = DERIV(temp(s, i, j - 2, k), temp(s, i, j - 1, k), temp(s, i, j + 1, k), temp(s, i, j + 2, k), inv);
        F(s, G_TZ, i, j, k) = DERIV(temp(s, i, j, k - 2), temp(s, i, j, k - 1), temp(s, i, j, k + 1), temp(s, i, j, k + 2), inv);
      }
}

/* total (convective minus viscous) flux along axis a at a point, 5 components */
static void flux(ns_state *s, int a, int i, int j, int k, double out[5]) {
  const double r = F(s, P_R, i, j, k), p = F(s, P_P, i, j, k);
  const double u[3] = {F(s, P_U, i, j, k), F(s, P_V, i, j, k), F(s, P_W, i, j, k)};
  const double ua = u[a];
  /* velocity gradient g[c][b] = d u_c / d x_b */
  double g[3][3];
  for (int c = 0; c < 3; c++)
    for (int b = 0; b < 3; b++) g[c][b] = F(s, G_UX + 3 * c + b, i, j, k);
  const double div = (g[0][0] + g[1][1]) + g[2][2];
  double tau[3];
  for (int c = 0; c < 3; c++) {
    double t = g[c][a] + g[a][c];
    if (c == a) t -= (2.0 / 3.0) * div;
    tau[c] = s->mu * t;
  }
  const double dT = F(s, G_TX + a, i, j, k);
  const double rE = p / (GAMMA - 1.0) + 0.5 * r * ((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]);
  out[0] = r * ua;
  for (int c = 0; c < 3; c++) out[1 + c] = (r * u[c]) * ua + (c == a ? p : 0.0) - tau[c];
  out[4] = (rE + p) * ua - ((u[0] * tau[0] + u[1] * tau[1]) + u[2] * tau[2]) - s->kappa * dT;
}

/* one RK stage: residual over the interior and the 2N-storage update */
static const double RK_A[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
static const double RK_B[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};

void ns_stage(ns_state *s, int stage, double dt) {
  const int n = s->n;
  const double inv = 1.0 / (12.0 * s->h);
  halos(s);
  primitives(s);
  gradients(s);
#pragma omp parallel for
  for (int k = 0; k < n; k++)
    for (int j = 0; j < n; j++)
      for (int i = 0; i < n; i++) {
        double res[5] = {0, 0, 0, 0, 0};
        for (int a = 0; a < 3; a++) {
          const int di = a == 0, dj = a == 1, dk = a == 2;
          double fm2[5], fm1[5], fp1[5], fp2[5];
          flux(s, a, i - 2 * di, j - 2 * dj, k - 2 * dk, fm2);
          flux(s, a, i - di, j - dj, k - dk, fm1);
          flux(s, a, i + di, j + dj, k + dk, fp1);
          flux(s, a, i + 2 * di, j + 2 * dj, k + 2 * dk, fp2);
          for (int c = 0; c < 5; c++) res[c] -= DERIV(fm2[c], fm1[c], fp1[c], fp2[c], inv);
        }
        for (int c = 0; c < 5; c++) {
          double d = stage == 0 ? dt * res[c] : RK_A[stage] * F(s, D_R + c, i, j, k) + dt * res[c];
          F(s, D_R + c, i, j, k) = d;
          F(s, Q_R + c, i, j, k) = F(s, Q_R + c, i, j, k) + RK_B[stage] * d;
        }
      }
}

void ns_step(ns_state *s, double dt) {
  for (int st = 0; st < 3; st++) ns_stage(s, st, dt);
}

/* plain interior sum of a field (rows in order) */
double ns_sum(ns_state *s, int f) {
  double tot = 0.0;
  for (int k = 0; k < s->n; k++)
    for (int j = 0; j < s->n; j++) {
      double row = 0.0;
      for (int i = 0; i < s->n; i++) row += F(s, f, i, j, k);
      tot += row;
    }
  return tot;
}

/* volume-averaged kinetic energy 0.5 |rho u|^2 / rho */
double ns_kinetic(ns_state *s) {
  double tot = 0.0;
  for (int k = 0; k < s->n; k++)
    for (int j = 0; j < s->n; j++)
      for (int i = 0; i < s->n; i++) {
        double r = F(s, Q_R, i, j, k);
        double m2 = (F(s, Q_RU, i, j, k) * F(s, Q_RU, i, j, k) + F(s, Q_RV, i, j, k) * F(s, Q_RV, i, j, k)) +
                    F(s, Q_RW, i, j, k) * F(s, Q_RW, i, j, k);
        tot += 0.5 * m2 / r;
      }
  return tot / ((double)s->n * s->n * s->n);
}
