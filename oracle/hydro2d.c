/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg may load
 * this file's library. The product path never calls it.
 *
 * Plain, untiled, loop-by-loop FP64 definition of the 2D hydro proxy: a
 * staggered-grid Lagrangian step (predictor-corrector) followed by donor-cell
 * remap sweeps in x then y, with reflective walls.  It is the "plain program"
 * that any tiled / out-of-core schedule must reproduce: the paper states that
 * the points of a parallel loop may run in any order (Section 3), and its
 * tiling only reorders loop points across tiles while keeping every data
 * dependence (Section 3, lazy execution and dependency analysis), so the tiled
 * result equals the result of running each loop over its full range in
 * program order -- which is what this file does.
 *
 * The paper names CloverLeaf 2D only by class (compressible Euler, explicit
 * second order, staggered grid, Lagrangian predictor-corrector plus
 * directional advection sweeps; Section 5.1).  The concrete scheme below is a
 * textbook one written for this proxy; its constants are readings, not
 * values from the paper.
 *
 * Index convention: cell (i,j) spans [i*dx,(i+1)*dx] x [j*dy,(j+1)*dy];
 * node (i,j) is its lower-left corner; x-face (i,j) is its left face; y-face
 * (i,j) its bottom face.  Interior cells i in [0,nx), nodes i in [0,nx].
 * All arrays here are allocated with the node extent [-2, n+3) on both axes.
 * Build: gcc -O2 -ffp-contract=off -fopenmp (no fast-math, no contraction).
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define H 2
#define GAMMA 1.4
#define GM1 0.4
#define CQ2 1.0   /* quadratic artificial-viscosity coefficient (reading) */
#define CQ1 0.5   /* linear artificial-viscosity coefficient (reading) */
#define CFL 0.5   /* Courant factor of the time-step bound (reading) */

enum {
  RHO0, RHO1, E0, E1, PRE, CS, VISC, VOL, U0, V0, U1, V1, XAREA, VFX, MFX,
  YAREA, VFY, MFY, W_PRE, W_POST, W_EF, W_NF, W_NMPOST, W_NMPRE, W_MF,
  NF_H2D
};

typedef struct {
  int nx, ny;
  long pitch;  /* nx + 1 + 2H */
  long rows;   /* ny + 1 + 2H */
  double dx, dy;
  double *f[NF_H2D];
} h2d_state;

#define A(s, k, i, j) ((s)->f[k][(long)((j) + H) * (s)->pitch + ((i) + H)])

h2d_state *h2d_create(int nx, int ny) {
  h2d_state *s = (h2d_state *)calloc(1, sizeof(h2d_state));
  s->nx = nx; s->ny = ny;
  s->pitch = nx + 1 + 2 * H;
  s->rows = ny + 1 + 2 * H;
  s->dx = 1.0 / nx; s->dy = 1.0 / ny;
  for (int k = 0; k < NF_H2D; k++)
    s->f[k] = (double *)calloc((size_t)(s->pitch * s->rows), sizeof(double));
  return s;
}

void h2d_destroy(h2d_state *s) {
  for (int k = 0; k < NF_H2D; k++) free(s->f[k]);
  free(s);
}

double *h2d_field(h2d_state *s, int k) { return s->f[k]; }
int oracle_threads(void) { return omp_get_max_threads(); }
long h2d_pitch(h2d_state *s) { return s->pitch; }
long h2d_rows(h2d_state *s) { return s->rows; }

/* ---------------------------------------------------------------- geometry */
/* Uniform Cartesian mesh: cell volume dx*dy, x-face area dy, y-face area dx. */
void h2d_geometry(h2d_state *s) {
  for (int j = -H; j < s->ny + H + 1; j++)
    for (int i = -H; i < s->nx + H + 1; i++) {
      A(s, VOL, i, j) = s->dx * s->dy;
      A(s, XAREA, i, j) = s->dy;
      A(s, YAREA, i, j) = s->dx;
    }
}

/* ------------------------------------------------------ reflective boundary */
/* Mirror copy dst(i,j) = sign * src(i+ox, j+oy) over an index rectangle: the
 * building block of every reflective-wall strip loop. */
static void mirror(h2d_state *s, int k, double sign, int i0, int i1, int j0,
                   int j1, int ox, int oy) {
#pragma omp parallel for
  for (int j = j0; j < j1; j++)
    for (int i = i0; i < i1; i++) A(s, k, i, j) = sign * A(s, k, i + ox, j + oy);
}

/* Reflective walls for the state at the start of a step: cell scalars are even
 * about the wall face (cell -1-k <- k); node velocities are reflected about the
 * wall node (node -k <- k), odd for the wall-normal component.  Sides are done
 * bottom, top, left, right so the corners take both reflections. */
static void bc_state(h2d_state *s) {
  const int nx = s->nx, ny = s->ny;
  const int cells[2] = {RHO0, E0};
  for (int c = 0; c < 2; c++)
    for (int k = 0; k < 2; k++) {
      mirror(s, cells[c], 1.0, -H, nx + H, -1 - k, -k, 0, 2 * k + 1);
      mirror(s, cells[c], 1.0, -H, nx + H, ny + k, ny + k + 1, 0, -2 * k - 1);
    }
  for (int k = 1; k <= 2; k++) {
    mirror(s, U0, 1.0, -H, nx + H + 1, -k, -k + 1, 0, 2 * k);
    mirror(s, V0, -1.0, -H, nx + H + 1, -k, -k + 1, 0, 2 * k);
    mirror(s, U0, 1.0, -H, nx + H + 1, ny + k, ny + k + 1, 0, -2 * k);
    mirror(s, V0, -1.0, -H, nx + H + 1, ny + k, ny + k + 1, 0, -2 * k);
  }
  for (int c = 0; c < 2; c++)
    for (int k = 0; k < 2; k++) {
      mirror(s, cells[c], 1.0, -1 - k, -k, -H, ny + H, 2 * k + 1, 0);
      mirror(s, cells[c], 1.0, nx + k, nx + k + 1, -H, ny + H, -2 * k - 1, 0);
    }
  for (int k = 1; k <= 2; k++) {
    mirror(s, U0, -1.0, -k, -k + 1, -H, ny + H + 1, 2 * k, 0);
    mirror(s, V0, 1.0, -k, -k + 1, -H, ny + H + 1, 2 * k, 0);
    mirror(s, U0, -1.0, nx + k, nx + k + 1, -H, ny + H + 1, -2 * k, 0);
    mirror(s, V0, 1.0, nx + k, nx + k + 1, -H, ny + H + 1, -2 * k, 0);
  }
}

/* ------------------------------------------------------------ Lagrangian */
/* Ideal-gas equation of state: p = (gamma-1) rho e, c = sqrt(gamma p / rho). */
static void eos(h2d_state *s, int rho, int ene, int with_cs, int i0, int i1,
                int j0, int j1) {
#pragma omp parallel for
  for (int j = j0; j < j1; j++)
    for (int i = i0; i < i1; i++) {
      double r = A(s, rho, i, j);
      double p = (GM1 * r) * A(s, ene, i, j);
      A(s, PRE, i, j) = p;
      if (with_cs) A(s, CS, i, j) = sqrt((GAMMA * p) / r);
    }
}

/* Artificial viscosity from the velocity jumps across the cell (its 4 nodes):
 * q = rho (c2 d^2 - c1 c d) where d = du + dv < 0 (compression), else 0. */
static void viscosity(h2d_state *s, int i0, int i1, int j0, int j1) {
#pragma omp parallel for
  for (int j = j0; j < j1; j++)
    for (int i = i0; i < i1; i++) {
      double du = 0.5 * ((A(s, U0, i + 1, j) + A(s, U0, i + 1, j + 1)) -
                         (A(s, U0, i, j) + A(s, U0, i, j + 1)));
      double dv = 0.5 * ((A(s, V0, i, j + 1) + A(s, V0, i + 1, j + 1)) -
                         (A(s, V0, i, j) + A(s, V0, i + 1, j)));
      double d = du + dv;
      double q = 0.0;
      if (d < 0.0) q = A(s, RHO0, i, j) * ((CQ2 * d) * d - (CQ1 * A(s, CS, i, j)) * d);
      A(s, VISC, i, j) = q;
    }
}

/* PdV work: the cell volume change over the step from the face volume fluxes
 * (face velocity = mean of its two nodes; the corrector averages the start and
 * end velocities), then rho1 = rho0 V / V' and e1 = e0 - (p+q) dV / (rho0 V).
 * fac = dt/4 in both phases: the predictor sums two node velocities over half a
 * step, the corrector four over a full step. */
static void pdv(h2d_state *s, int corrector, double dt, int i0, int i1, int j0,
                int j1) {
  const double fac = 0.25 * dt;
#pragma omp parallel for
  for (int j = j0; j < j1; j++)
    for (int i = i0; i < i1; i++) {
      double ul, ur, vb, vt;
      if (corrector) {
        ul = (A(s, U0, i, j) + A(s, U1, i, j)) + (A(s, U0, i, j + 1) + A(s, U1, i, j + 1));
        ur = (A(s, U0, i + 1, j) + A(s, U1, i + 1, j)) + (A(s, U0, i + 1, j + 1) + A(s, U1, i + 1, j + 1));
        vb = (A(s, V0, i, j) + A(s, V1, i, j)) + (A(s, V0, i + 1, j) + A(s, V1, i + 1, j));
        vt = (A(s, V0, i, j + 1) + A(s, V1, i, j + 1)) + (A(s, V0, i + 1, j + 1) + A(s, V1, i + 1, j + 1));
      } else {
        ul = A(s, U0, i, j) + A(s, U0, i, j + 1);
        ur = A(s, U0, i + 1, j) + A(s, U0, i + 1, j + 1);
        vb = A(s, V0, i, j) + A(s, V0, i + 1, j);
        vt = A(s, V0, i, j + 1) + A(s, V0, i + 1, j + 1);
      }
      double fl = (fac * A(s, XAREA, i, j)) * ul;
      double fr = (fac * A(s, XAREA, i + 1, j)) * ur;
      double fb = (fac * A(s, YAREA, i, j)) * vb;
      double ft = (fac * A(s, YAREA, i, j + 1)) * vt;
      double total = (fr - fl) + (ft - fb);
      double vol = A(s, VOL, i, j);
      double r0 = A(s, RHO0, i, j);
      double m = r0 * vol;
      A(s, RHO1, i, j) = m / (vol + total);
      A(s, E1, i, j) = A(s, E0, i, j) - ((A(s, PRE, i, j) + A(s, VISC, i, j)) * total) / m;
    }
}

/* Node acceleration: force = -(gradient of p+q), built as the exact adjoint of
 * the PdV volume-change operator so the Lagrangian step conserves total energy;
 * node mass = quarter of the four surrounding cell masses.  The wall-normal
 * velocity of wall nodes is held at zero. */
static void accelerate(h2d_state *s, double dt, int i0, int i1, int j0, int j1) {
  const int nx = s->nx, ny = s->ny;
#pragma omp parallel for
  for (int j = j0; j < j1; j++)
    for (int i = i0; i < i1; i++) {
      double pbl = A(s, PRE, i - 1, j - 1) + A(s, VISC, i - 1, j - 1);
      double pbr = A(s, PRE, i, j - 1) + A(s, VISC, i, j - 1);
      double ptl = A(s, PRE, i - 1, j) + A(s, VISC, i - 1, j);
      double ptr = A(s, PRE, i, j) + A(s, VISC, i, j);
      double mass = 0.25 * ((A(s, RHO0, i - 1, j - 1) * A(s, VOL, i - 1, j - 1) +
                             A(s, RHO0, i, j - 1) * A(s, VOL, i, j - 1)) +
                            (A(s, RHO0, i - 1, j) * A(s, VOL, i - 1, j) +
                             A(s, RHO0, i, j) * A(s, VOL, i, j)));
      double fx = 0.5 * (A(s, XAREA, i, j - 1) * (pbl - pbr) + A(s, XAREA, i, j) * (ptl - ptr));
      double fy = 0.5 * (A(s, YAREA, i - 1, j) * (pbl - ptl) + A(s, YAREA, i, j) * (pbr - ptr));
      double u = A(s, U0, i, j) + (dt * fx) / mass;
      double v = A(s, V0, i, j) + (dt * fy) / mass;
      if (i == 0 || i == nx) u = 0.0;
      if (j == 0 || j == ny) v = 0.0;
      A(s, U1, i, j) = u;
      A(s, V1, i, j) = v;
    }
}

/* Face volume fluxes of the step (same expression as the PdV corrector's). */
static void flux_calc(h2d_state *s, double dt) {
  const int nx = s->nx, ny = s->ny;
  const double fac = 0.25 * dt;
#pragma omp parallel for
  for (int j = -1; j < ny + 1; j++)
    for (int i = -1; i < nx + 2; i++)
      A(s, VFX, i, j) = (fac * A(s, XAREA, i, j)) *
                        ((A(s, U0, i, j) + A(s, U1, i, j)) + (A(s, U0, i, j + 1) + A(s, U1, i, j + 1)));
#pragma omp parallel for
  for (int j = -1; j < ny + 2; j++)
    for (int i = -1; i < nx + 1; i++)
      A(s, VFY, i, j) = (fac * A(s, YAREA, i, j)) *
                        ((A(s, V0, i, j) + A(s, V1, i, j)) + (A(s, V0, i + 1, j) + A(s, V1, i + 1, j)));
}

/* ------------------------------------------------------------- remap sweeps */
/* Donor-cell (first-order upwind) remap of mass and internal energy, one
 * direction at a time.  dir = 0: x (faces between cells i-1 and i), dir = 1: y.
 * A face with zero volume flux carries no mass. */
static void adv_cell(h2d_state *s, int dir) {
  const int nx = s->nx, ny = s->ny;
  const int VF = dir == 0 ? VFX : VFY, MF = dir == 0 ? MFX : MFY;
  const int di = dir == 0, dj = dir == 1;
  /* pre- and post-sweep volumes */
  if (dir == 0) {
#pragma omp parallel for
    for (int j = -1; j < ny + 1; j++)
      for (int i = -1; i < nx + 1; i++) {
        double dfx = A(s, VFX, i + 1, j) - A(s, VFX, i, j);
        double pre = A(s, VOL, i, j) + (dfx + (A(s, VFY, i, j + 1) - A(s, VFY, i, j)));
        A(s, W_PRE, i, j) = pre;
        A(s, W_POST, i, j) = pre - dfx;
      }
  } else {
#pragma omp parallel for
    for (int j = -1; j < ny + 1; j++)
      for (int i = -1; i < nx + 1; i++) {
        A(s, W_PRE, i, j) = A(s, VOL, i, j) + (A(s, VFY, i, j + 1) - A(s, VFY, i, j));
        A(s, W_POST, i, j) = A(s, VOL, i, j);
      }
  }
  /* mass and energy fluxes through the faces */
  int fi0, fi1, fj0, fj1;
  if (dir == 0) { fi0 = 0; fi1 = nx + 1; fj0 = -1; fj1 = ny + 1; }
  else { fi0 = -1; fi1 = nx + 1; fj0 = 0; fj1 = ny + 1; }
#pragma omp parallel for
  for (int j = fj0; j < fj1; j++)
    for (int i = fi0; i < fi1; i++) {
      double f = A(s, VF, i, j);
      double mf = 0.0, ef = 0.0;
      if (f > 0.0) {
        mf = f * A(s, RHO1, i - di, j - dj);
        ef = mf * A(s, E1, i - di, j - dj);
      } else if (f < 0.0) {
        mf = f * A(s, RHO1, i, j);
        ef = mf * A(s, E1, i, j);
      }
      A(s, MF, i, j) = mf;
      A(s, W_EF, i, j) = ef;
    }
  /* conservative update */
  int ci0, ci1, cj0, cj1;
  if (dir == 0) { ci0 = 0; ci1 = nx; cj0 = -1; cj1 = ny + 1; }
  else { ci0 = -1; ci1 = nx + 1; cj0 = 0; cj1 = ny; }
#pragma omp parallel for
  for (int j = cj0; j < cj1; j++)
    for (int i = ci0; i < ci1; i++) {
      double pm = A(s, RHO1, i, j) * A(s, W_PRE, i, j);
      double post = pm + (A(s, MF, i, j) - A(s, MF, i + di, j + dj));
      double pe = (A(s, E1, i, j) * pm + (A(s, W_EF, i, j) - A(s, W_EF, i + di, j + dj))) / post;
      A(s, RHO1, i, j) = post / A(s, W_POST, i, j);
      A(s, E1, i, j) = pe;
    }
}

/* Donor-cell remap of a node velocity component on the dual (node-centred)
 * mesh: the dual-face mass flux is the mean of the four neighbouring face
 * mass fluxes; node masses after the sweep come from the swept cells, and
 * before it by undoing the dual fluxes. */
static void adv_mom_mass(h2d_state *s, int dir) {
  const int nx = s->nx, ny = s->ny;
  if (dir == 0) {
#pragma omp parallel for
    for (int j = 0; j < ny + 1; j++)
      for (int i = -1; i < nx + 1; i++)
        A(s, W_NF, i, j) = 0.25 * ((A(s, MFX, i, j - 1) + A(s, MFX, i, j)) +
                                   (A(s, MFX, i + 1, j - 1) + A(s, MFX, i + 1, j)));
  } else {
#pragma omp parallel for
    for (int j = -1; j < ny + 1; j++)
      for (int i = 0; i < nx + 1; i++)
        A(s, W_NF, i, j) = 0.25 * ((A(s, MFY, i - 1, j) + A(s, MFY, i, j)) +
                                   (A(s, MFY, i - 1, j + 1) + A(s, MFY, i, j + 1)));
  }
  const int di = dir == 0, dj = dir == 1;
#pragma omp parallel for
  for (int j = 0; j < ny + 1; j++)
    for (int i = 0; i < nx + 1; i++) {
      double post = 0.25 * ((A(s, RHO1, i - 1, j - 1) * A(s, W_POST, i - 1, j - 1) +
                             A(s, RHO1, i, j - 1) * A(s, W_POST, i, j - 1)) +
                            (A(s, RHO1, i - 1, j) * A(s, W_POST, i - 1, j) +
                             A(s, RHO1, i, j) * A(s, W_POST, i, j)));
      A(s, W_NMPOST, i, j) = post;
      A(s, W_NMPRE, i, j) = post + (A(s, W_NF, i, j) - A(s, W_NF, i - di, j - dj));
    }
}

static void adv_mom_vel(h2d_state *s, int dir, int vel) {
  const int nx = s->nx, ny = s->ny;
  const int di = dir == 0, dj = dir == 1;
  int i0 = dir == 0 ? -1 : 0, j0 = dir == 0 ? 0 : -1;
#pragma omp parallel for
  for (int j = j0; j < ny + 1; j++)
    for (int i = i0; i < nx + 1; i++) {
      double f = A(s, W_NF, i, j);
      double mf = 0.0;
      if (f > 0.0) mf = f * A(s, vel, i, j);
      else if (f < 0.0) mf = f * A(s, vel, i + di, j + dj);
      A(s, W_MF, i, j) = mf;
    }
#pragma omp parallel for
  for (int j = 0; j < ny + 1; j++)
    for (int i = 0; i < nx + 1; i++)
      A(s, vel, i, j) = (A(s, vel, i, j) * A(s, W_NMPRE, i, j) +
                         (A(s, W_MF, i - di, j - dj) - A(s, W_MF, i, j))) /
                        A(s, W_NMPOST, i, j);
}

/* Largest stable step of a cell: CFL * min over axes of spacing / (effective
 * sound speed + largest node speed along that axis); the effective sound
 * speed adds the viscous pressure.  Evaluated from the state (rho0 is not
 * needed since q/rho and c only depend on e and the velocities). */
static double dt_cell(h2d_state *s, int i, int j) {
  double c2 = (GAMMA * GM1) * A(s, E0, i, j);
  double du = 0.5 * ((A(s, U0, i + 1, j) + A(s, U0, i + 1, j + 1)) -
                     (A(s, U0, i, j) + A(s, U0, i, j + 1)));
  double dv = 0.5 * ((A(s, V0, i, j + 1) + A(s, V0, i + 1, j + 1)) -
                     (A(s, V0, i, j) + A(s, V0, i + 1, j)));
  double d = du + dv;
  double qr = 0.0;
  if (d < 0.0) qr = (CQ2 * d) * d - (CQ1 * sqrt(c2)) * d;
  double ce = sqrt(c2 + 2.0 * qr);
  double um = fmax(fmax(fabs(A(s, U0, i, j)), fabs(A(s, U0, i + 1, j))),
                   fmax(fabs(A(s, U0, i, j + 1)), fabs(A(s, U0, i + 1, j + 1))));
  double vm = fmax(fmax(fabs(A(s, V0, i, j)), fabs(A(s, V0, i + 1, j))),
                   fmax(fabs(A(s, V0, i, j + 1)), fabs(A(s, V0, i + 1, j + 1))));
  double tx = s->dx / (ce + um);
  double ty = s->dy / (ce + vm);
  return CFL * fmin(tx, ty);
}

double h2d_dt(h2d_state *s) {
  double m = INFINITY;
#pragma omp parallel for reduction(min : m)
  for (int j = 0; j < s->ny; j++)
    for (int i = 0; i < s->nx; i++) {
      double t = dt_cell(s, i, j);
      if (t < m) m = t;
    }
  return m;
}

/* Lagrangian phase of one step (state BC, EOS, viscosity, predictor,
 * predictor EOS, acceleration, corrector).  Afterwards rho1/e1/u1/v1 hold the
 * Lagrangian end state on the moved mesh (volume V + total flux). */
void h2d_lagrangian(h2d_state *s, double dt) {
  const int nx = s->nx, ny = s->ny;
  bc_state(s);
  eos(s, RHO0, E0, 1, -H, nx + H, -H, ny + H);
  viscosity(s, -H, nx + H, -H, ny + H);
  pdv(s, 0, dt, -H, nx + H, -H, ny + H);
  eos(s, RHO1, E1, 0, -H, nx + H, -H, ny + H);
  accelerate(s, dt, -1, nx + H, -1, ny + H);
  pdv(s, 1, dt, -1, nx + 1, -1, ny + 1);
}

/* One full step with time step dt; returns the next time step (min over the
 * interior cells of the new state). */
double h2d_step(h2d_state *s, double dt) {
  const int nx = s->nx, ny = s->ny;
  h2d_lagrangian(s, dt);
  flux_calc(s, dt);
  /* x sweep */
  adv_cell(s, 0);
  mirror(s, RHO1, 1.0, -1, 0, -1, ny + 1, 1, 0);
  mirror(s, E1, 1.0, -1, 0, -1, ny + 1, 1, 0);
  mirror(s, RHO1, 1.0, nx, nx + 1, -1, ny + 1, -1, 0);
  mirror(s, E1, 1.0, nx, nx + 1, -1, ny + 1, -1, 0);
  mirror(s, MFX, -1.0, -1, 0, -1, ny + 1, 2, 0);
  mirror(s, MFX, -1.0, nx + 1, nx + 2, -1, ny + 1, -2, 0);
  adv_mom_mass(s, 0);
  adv_mom_vel(s, 0, U1);
  adv_mom_vel(s, 0, V1);
  mirror(s, U1, 1.0, 0, nx + 1, -1, 0, 0, 2);
  mirror(s, V1, -1.0, 0, nx + 1, -1, 0, 0, 2);
  mirror(s, U1, 1.0, 0, nx + 1, ny + 1, ny + 2, 0, -2);
  mirror(s, V1, -1.0, 0, nx + 1, ny + 1, ny + 2, 0, -2);
  /* y sweep */
  adv_cell(s, 1);
  mirror(s, RHO1, 1.0, -1, nx + 1, -1, 0, 0, 1);
  mirror(s, RHO1, 1.0, -1, nx + 1, ny, ny + 1, 0, -1);
  mirror(s, MFY, -1.0, -1, nx + 1, -1, 0, 0, 2);
  mirror(s, MFY, -1.0, -1, nx + 1, ny + 1, ny + 2, 0, -2);
  adv_mom_mass(s, 1);
  adv_mom_vel(s, 1, U1);
  adv_mom_vel(s, 1, V1);
  /* reset: the remapped state becomes the new state */
#pragma omp parallel for
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      A(s, RHO0, i, j) = A(s, RHO1, i, j);
      A(s, E0, i, j) = A(s, E1, i, j);
    }
#pragma omp parallel for
  for (int j = 0; j < ny + 1; j++)
    for (int i = 0; i < nx + 1; i++) {
      A(s, U0, i, j) = A(s, U1, i, j);
      A(s, V0, i, j) = A(s, V1, i, j);
    }
  return h2d_dt(s);
}

/* Field summary of the current state: the periodic diagnostic that reads
 * many fields, whose separate chain the paper names as a cause of its
 * CloverLeaf 2D gap (Section 5.3).  First the pressure of the state from the
 * equation of state over the interior, then five plain sums over the
 * interior cells, rows in order, each row in x order:
 *   out[0] volume           sum of vol
 *   out[1] mass             sum of rho0 vol
 *   out[2] internal energy  sum of (rho0 vol) e0
 *   out[3] kinetic energy   sum of (rho0 vol) (0.5 w), w = the mean over the
 *                           cell's four nodes of u0^2 + v0^2
 *   out[4] pressure         sum of p vol */
void h2d_field_summary(h2d_state *s, double out[5]) {
  eos(s, RHO0, E0, 0, 0, s->nx, 0, s->ny);
  double tot[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int j = 0; j < s->ny; j++) {
    double row[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < s->nx; i++) {
      const double vol = A(s, VOL, i, j);
      const double m = A(s, RHO0, i, j) * vol;
      double w[4];
      for (int c = 0; c < 4; c++) {
        const int ii = i + (c & 1), jj = j + (c >> 1);
        w[c] = A(s, U0, ii, jj) * A(s, U0, ii, jj) + A(s, V0, ii, jj) * A(s, V0, ii, jj);
      }
      const double wm = 0.25 * ((w[0] + w[1]) + (w[2] + w[3]));
      row[0] += vol;
      row[1] += m;
      row[2] += m * A(s, E0, i, j);
      row[3] += m * (0.5 * wm);
      row[4] += A(s, PRE, i, j) * vol;
    }
    for (int q = 0; q < 5; q++) tot[q] += row[q];
  }
  for (int q = 0; q < 5; q++) out[q] = tot[q];
}

/* Plain sum of f * vol over the interior cells, rows in order, each row in x
 * order (a conservation diagnostic). */
double h2d_sum_cells(h2d_state *s, int k, int times_rho0) {
  double tot = 0.0;
  for (int j = 0; j < s->ny; j++) {
    double row = 0.0;
    for (int i = 0; i < s->nx; i++) {
      double v = A(s, k, i, j) * A(s, VOL, i, j);
      if (times_rho0) v *= A(s, RHO0, i, j);
      row += v;
    }
    tot += row;
  }
  return tot;
}
