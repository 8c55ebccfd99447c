/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 * Only tests/, the smoke check and the benchmark's CPU-baseline leg may load
 * this file's library. The product path never calls it.
 *
 * Plain, untiled, loop-by-loop FP64 definition of the 3D hydro proxy, the
 * three-dimensional form of the 2D proxy in hydro2d.c (the paper names
 * CloverLeaf 3D only by class, Section 5.1: the same physics as the 2D code
 * with sweeps in three directions).  Staggered grid: cell (i,j,k) spans
 * [i dx,(i+1) dx] x [j dy,(j+1) dy] x [k dz,(k+1) dz]; node (i,j,k) is its
 * lowest corner; x/y/z-face (i,j,k) its lower face along that axis.
 *   - Lagrangian step: EOS, viscosity from the velocity jumps across the cell,
 *     predictor / corrector PdV (face flux = area x mean of its 4 node
 *     velocities), node acceleration as the exact adjoint of the PdV volume
 *     change (node mass = an eighth of its 8 cells);
 *   - donor-cell remap of mass, internal energy and momentum, x then y then z;
 *   - reflective walls on all six sides (strip loops, 2 layers).
 * All arrays use the node extent [-2, n+3) on every axis.
 * Build: gcc -O2 -ffp-contract=off -fopenmp.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define H 2
#define GAMMA 1.4
#define GM1 0.4
#define CQ2 1.0
#define CQ1 0.5
#define CFL 0.5

enum {
  RHO0, RHO1, E0, E1, PRE, CS, VISC, VOL,
  U0, V0, W0, U1, V1, W1,
  XAREA, VFX, MFX, YAREA, VFY, MFY, ZAREA, VFZ, MFZ,
  W_PRE, W_POST, W_EF, W_NF, W_NMPOST, W_NMPRE, W_MF,
  NF_H3D
};

typedef struct {
  int n[3];
  long sy, sz;
  double d[3];
  double *f[NF_H3D];
} h3d_state;

#define A3(s, fld, i, j, k) ((s)->f[fld][(long)((k) + H) * (s)->sz + (long)((j) + H) * (s)->sy + ((i) + H)])

h3d_state *h3d_create(int nx, int ny, int nz) {
  h3d_state *s = (h3d_state *)calloc(1, sizeof(h3d_state));
  s->n[0] = nx; s->n[1] = ny; s->n[2] = nz;
  s->sy = nx + 1 + 2 * H;
  s->sz = s->sy * (ny + 1 + 2 * H);
  for (int a = 0; a < 3; a++) s->d[a] = 1.0 / s->n[a];
  for (int f = 0; f < NF_H3D; f++)
    s->f[f] = (double *)calloc((size_t)(s->sz * (nz + 1 + 2 * H)), sizeof(double));
  return s;
}

void h3d_destroy(h3d_state *s) {
  for (int f = 0; f < NF_H3D; f++) free(s->f[f]);
  free(s);
}

double *h3d_field(h3d_state *s, int f) { return s->f[f]; }
long h3d_extent(h3d_state *s, int a) { return s->n[a] + 1 + 2 * H; }

void h3d_geometry(h3d_state *s) {
  const double dx = s->d[0], dy = s->d[1], dz = s->d[2];
  for (int k = -H; k < s->n[2] + H + 1; k++)
    for (int j = -H; j < s->n[1] + H + 1; j++)
      for (int i = -H; i < s->n[0] + H + 1; i++) {
        A3(s, VOL, i, j, k) = (dx * dy) * dz;
        A3(s, XAREA, i, j, k) = dy * dz;
        A3(s, YAREA, i, j, k) = dx * dz;
        A3(s, ZAREA, i, j, k) = dx * dy;
      }
}

/* dst(p) = sign * src(p + o) over a box: the reflective strip loop */
static void mirror(h3d_state *s, int fld, double sign, const int lo[3], const int hi[3], const int o[3]) {
#pragma omp parallel for
  for (int k = lo[2]; k < hi[2]; k++)
    for (int j = lo[1]; j < hi[1]; j++)
      for (int i = lo[0]; i < hi[0]; i++)
        A3(s, fld, i, j, k) = sign * A3(s, fld, i + o[0], j + o[1], k + o[2]);
}

/* reflection of a set of fields about the two walls of axis a, layer by layer:
 * cell-centred along a (cell -1-m <- m) or node-centred (node -m <- m);
 * other axes over [lo, hi) */
static void walls(h3d_state *s, int a, const int *flds, const double *sgn, int nf, int node, const int lo[3],
                  const int hi[3]) {
  const int n = s->n[a];
  for (int m = node ? 1 : 0; m < (node ? 3 : 2); m++) {
    int l[3], h[3], o[3] = {0, 0, 0};
    for (int b = 0; b < 3; b++) { l[b] = lo[b]; h[b] = hi[b]; }
    /* low wall */
    l[a] = node ? -m : -1 - m; h[a] = l[a] + 1; o[a] = node ? 2 * m : 2 * m + 1;
    for (int q = 0; q < nf; q++) mirror(s, flds[q], sgn[q], l, h, o);
    /* high wall */
    l[a] = n + m; h[a] = l[a] + 1; o[a] = node ? -2 * m : -2 * m - 1;
    for (int q = 0; q < nf; q++) mirror(s, flds[q], sgn[q], l, h, o);
  }
}

/* State halos at the start of a step: x walls over interior y, z; then y walls
 * over all x and interior z; then z walls over all x, y (so edges and corners
 * take every reflection).  Velocity normal to a wall is odd. */
static void bc_state(h3d_state *s) {
  const int nx = s->n[0], ny = s->n[1], nz = s->n[2];
  const int cells[2] = {RHO0, E0};
  const double even2[2] = {1.0, 1.0};
  const int vel[3] = {U0, V0, W0};
  for (int a = 0; a < 3; a++) {
    int lo[3] = {0, 0, 0}, hic[3] = {nx, ny, nz}, hin[3] = {nx + 1, ny + 1, nz + 1};
    for (int b = 0; b < a; b++) { lo[b] = -H; hic[b] = s->n[b] + H; hin[b] = s->n[b] + H + 1; }
    walls(s, a, cells, even2, 2, 0, lo, hic);
    double sg[3] = {1.0, 1.0, 1.0};
    sg[a] = -1.0;
    walls(s, a, vel, sg, 3, 1, lo, hin);
  }
}

static void eos(h3d_state *s, int rho, int ene, int with_cs, const int lo[3], const int hi[3]) {
#pragma omp parallel for
  for (int k = lo[2]; k < hi[2]; k++)
    for (int j = lo[1]; j < hi[1]; j++)
      for (int i = lo[0]; i < hi[0]; i++) {
        double r = A3(s, rho, i, j, k);
        double p = (GM1 * r) * A3(s, ene, i, j, k);
        A3(s, PRE, i, j, k) = p;
        if (with_cs) A3(s, CS, i, j, k) = sqrt((GAMMA * p) / r);
      }
}

/* sum of a node field over the 4 nodes of the face of cell (i,j,k) normal to
 * axis a at offset e (0 = lower face, 1 = upper face) */
static double face4(h3d_state *s, int fld, int a, int e, int i, int j, int k) {
  if (a == 0)
    return (A3(s, fld, i + e, j, k) + A3(s, fld, i + e, j + 1, k)) +
           (A3(s, fld, i + e, j, k + 1) + A3(s, fld, i + e, j + 1, k + 1));
  if (a == 1)
    return (A3(s, fld, i, j + e, k) + A3(s, fld, i + 1, j + e, k)) +
           (A3(s, fld, i, j + e, k + 1) + A3(s, fld, i + 1, j + e, k + 1));
  return (A3(s, fld, i, j, k + e) + A3(s, fld, i + 1, j, k + e)) +
         (A3(s, fld, i, j + 1, k + e) + A3(s, fld, i + 1, j + 1, k + e));
}

/* the same with the start-plus-end velocity of every node */
static double face4_2(h3d_state *s, int f0, int f1, int a, int e, int i, int j, int k) {
#define P2(ii, jj, kk) (A3(s, f0, ii, jj, kk) + A3(s, f1, ii, jj, kk))
  if (a == 0) return (P2(i + e, j, k) + P2(i + e, j + 1, k)) + (P2(i + e, j, k + 1) + P2(i + e, j + 1, k + 1));
  if (a == 1) return (P2(i, j + e, k) + P2(i + 1, j + e, k)) + (P2(i, j + e, k + 1) + P2(i + 1, j + e, k + 1));
  return (P2(i, j, k + e) + P2(i + 1, j, k + e)) + (P2(i, j + 1, k + e) + P2(i + 1, j + 1, k + e));
#undef P2
}

static const int VEL0[3] = {U0, V0, W0}, VEL1[3] = {U1, V1, W1};
static const int AREA[3] = {XAREA, YAREA, ZAREA}, VF[3] = {VFX, VFY, VFZ}, MF[3] = {MFX, MFY, MFZ};

static double jump(h3d_state *s, int a, int i, int j, int k) {
  return 0.25 * (face4(s, VEL0[a], a, 1, i, j, k) - face4(s, VEL0[a], a, 0, i, j, k));
}

static void viscosity(h3d_state *s, const int lo[3], const int hi[3]) {
#pragma omp parallel for
  for (int k = lo[2]; k < hi[2]; k++)
    for (int j = lo[1]; j < hi[1]; j++)
      for (int i = lo[0]; i < hi[0]; i++) {
        double d = (jump(s, 0, i, j, k) + jump(s, 1, i, j, k)) + jump(s, 2, i, j, k);
        double q = 0.0;
        if (d < 0.0) q = A3(s, RHO0, i, j, k) * ((CQ2 * d) * d - (CQ1 * A3(s, CS, i, j, k)) * d);
        A3(s, VISC, i, j, k) = q;
      }
}

/* PdV: fac = dt/8 (predictor: 4 start velocities over half a step;
 * corrector: 4 start + 4 end velocities over a full step) */
static void pdv(h3d_state *s, int corr, double dt, const int lo[3], const int hi[3]) {
  const double fac = 0.125 * dt;
#pragma omp parallel for
  for (int k = lo[2]; k < hi[2]; k++)
    for (int j = lo[1]; j < hi[1]; j++)
      for (int i = lo[0]; i < hi[0]; i++) {
        int off[3] = {0, 0, 0};
        double df[3];
        for (int a = 0; a < 3; a++) {
          double sl = corr ? face4_2(s, VEL0[a], VEL1[a], a, 0, i, j, k) : face4(s, VEL0[a], a, 0, i, j, k);
          double sh = corr ? face4_2(s, VEL0[a], VEL1[a], a, 1, i, j, k) : face4(s, VEL0[a], a, 1, i, j, k);
          off[a] = 1;
          double fl = (fac * A3(s, AREA[a], i, j, k)) * sl;
          double fh = (fac * A3(s, AREA[a], i + off[0], j + off[1], k + off[2])) * sh;
          off[a] = 0;
          df[a] = fh - fl;
        }
        double total = (df[0] + df[1]) + df[2];
        double vol = A3(s, VOL, i, j, k);
        double m = A3(s, RHO0, i, j, k) * vol;
        A3(s, RHO1, i, j, k) = m / (vol + total);
        A3(s, E1, i, j, k) = A3(s, E0, i, j, k) - ((A3(s, PRE, i, j, k) + A3(s, VISC, i, j, k)) * total) / m;
      }
}

/* node acceleration: force along a = 1/4 sum over the 4 faces normal to a
 * around the node of area x (P(lower cell) - P(upper cell)) */
static void accelerate(h3d_state *s, double dt, const int lo[3], const int hi[3]) {
#pragma omp parallel for
  for (int k = lo[2]; k < hi[2]; k++)
    for (int j = lo[1]; j < hi[1]; j++)
      for (int i = lo[0]; i < hi[0]; i++) {
        double P[2][2][2], M[2][2][2];
        for (int c = 0; c < 2; c++)
          for (int b = 0; b < 2; b++)
            for (int a = 0; a < 2; a++) {
              const int ci = i - 1 + a, cj = j - 1 + b, ck = k - 1 + c;
              P[c][b][a] = A3(s, PRE, ci, cj, ck) + A3(s, VISC, ci, cj, ck);
              M[c][b][a] = A3(s, RHO0, ci, cj, ck) * A3(s, VOL, ci, cj, ck);
            }
        const double mass = 0.125 * (((M[0][0][0] + M[0][0][1]) + (M[0][1][0] + M[0][1][1])) +
                                     ((M[1][0][0] + M[1][0][1]) + (M[1][1][0] + M[1][1][1])));
        const double fx = 0.25 * ((A3(s, XAREA, i, j - 1, k - 1) * (P[0][0][0] - P[0][0][1]) +
                                   A3(s, XAREA, i, j, k - 1) * (P[0][1][0] - P[0][1][1])) +
                                  (A3(s, XAREA, i, j - 1, k) * (P[1][0][0] - P[1][0][1]) +
                                   A3(s, XAREA, i, j, k) * (P[1][1][0] - P[1][1][1])));
        const double fy = 0.25 * ((A3(s, YAREA, i - 1, j, k - 1) * (P[0][0][0] - P[0][1][0]) +
                                   A3(s, YAREA, i, j, k - 1) * (P[0][0][1] - P[0][1][1])) +
                                  (A3(s, YAREA, i - 1, j, k) * (P[1][0][0] - P[1][1][0]) +
                                   A3(s, YAREA, i, j, k) * (P[1][0][1] - P[1][1][1])));
        const double fz = 0.25 * ((A3(s, ZAREA, i - 1, j - 1, k) * (P[0][0][0] - P[1][0][0]) +
                                   A3(s, ZAREA, i, j - 1, k) * (P[0][0][1] - P[1][0][1])) +
                                  (A3(s, ZAREA, i - 1, j, k) * (P[0][1][0] - P[1][1][0]) +
                                   A3(s, ZAREA, i, j, k) * (P[0][1][1] - P[1][1][1])));
        double u = A3(s, U0, i, j, k) + (dt * fx) / mass;
        double v = A3(s, V0, i, j, k) + (dt * fy) / mass;
        double w = A3(s, W0, i, j, k) + (dt * fz) / mass;
        if (i == 0 || i == s->n[0]) u = 0.0;
        if (j == 0 || j == s->n[1]) v = 0.0;
        if (k == 0 || k == s->n[2]) w = 0.0;
        A3(s, U1, i, j, k) = u;
        A3(s, V1, i, j, k) = v;
        A3(s, W1, i, j, k) = w;
      }
}

/* face volume flux along axis a (same expression as the PdV corrector) */
static void flux_calc(h3d_state *s, int a, double dt) {
  const double fac = 0.125 * dt;
  int lo[3] = {-1, -1, -1}, hi[3] = {s->n[0] + 1, s->n[1] + 1, s->n[2] + 1};
  hi[a] = s->n[a] + 2;
#pragma omp parallel for
  for (int k = lo[2]; k < hi[2]; k++)
    for (int j = lo[1]; j < hi[1]; j++)
      for (int i = lo[0]; i < hi[0]; i++)
        A3(s, VF[a], i, j, k) = (fac * A3(s, AREA[a], i, j, k)) * face4_2(s, VEL0[a], VEL1[a], a, 0, i, j, k);
}

/* ------------------------------------------------------------------- remap */
#define E(a, b) ((a) == (b) ? 1 : 0)

static double dflux(h3d_state *s, int a, int i, int j, int k) {
  return A3(s, VF[a], i + E(a, 0), j + E(a, 1), k + E(a, 2)) - A3(s, VF[a], i, j, k);
}

/* Volumes before and after sweep d over cells [-1, n+1)^3.  Directional
 * splitting x, y, z: before the x sweep the cell holds V + dVx + dVy + dVz,
 * after it V + dVy + dVz (as pre - dVx); the y sweep goes from V + dVy + dVz
 * to V + dVz; the z sweep from V + dVz back to V. */
static void adv_vol(h3d_state *s, int d) {
  const int nx = s->n[0], ny = s->n[1], nz = s->n[2];
#pragma omp parallel for
  for (int k = -1; k < nz + 1; k++)
    for (int j = -1; j < ny + 1; j++)
      for (int i = -1; i < nx + 1; i++) {
        const double vol = A3(s, VOL, i, j, k);
        if (d == 0) {
          const double dfx = dflux(s, 0, i, j, k);
          const double pre = vol + ((dfx + dflux(s, 1, i, j, k)) + dflux(s, 2, i, j, k));
          A3(s, W_PRE, i, j, k) = pre;
          A3(s, W_POST, i, j, k) = pre - dfx;
        } else if (d == 1) {
          const double dfz = dflux(s, 2, i, j, k);
          A3(s, W_PRE, i, j, k) = vol + (dflux(s, 1, i, j, k) + dfz);
          A3(s, W_POST, i, j, k) = vol + dfz;
        } else {
          A3(s, W_PRE, i, j, k) = vol + dflux(s, 2, i, j, k);
          A3(s, W_POST, i, j, k) = vol;
        }
      }
}

/* donor-cell mass and energy flux through the faces normal to d over the
 * given box: the upwind cell's density and energy times the volume flux */
static void adv_flux(h3d_state *s, int d, const int lo[3], const int hi[3]) {
#pragma omp parallel for
  for (int k = lo[2]; k < hi[2]; k++)
    for (int j = lo[1]; j < hi[1]; j++)
      for (int i = lo[0]; i < hi[0]; i++) {
        const double f = A3(s, VF[d], i, j, k);
        double mf = 0.0, ef = 0.0;
        if (f > 0.0) {
          mf = f * A3(s, RHO1, i - E(d, 0), j - E(d, 1), k - E(d, 2));
          ef = mf * A3(s, E1, i - E(d, 0), j - E(d, 1), k - E(d, 2));
        } else if (f < 0.0) {
          mf = f * A3(s, RHO1, i, j, k);
          ef = mf * A3(s, E1, i, j, k);
        }
        A3(s, MF[d], i, j, k) = mf;
        A3(s, W_EF, i, j, k) = ef;
      }
}

static void adv_cell(h3d_state *s, int d, const int lo[3], const int hi[3]) {
#pragma omp parallel for
  for (int k = lo[2]; k < hi[2]; k++)
    for (int j = lo[1]; j < hi[1]; j++)
      for (int i = lo[0]; i < hi[0]; i++) {
        const int i1 = i + E(d, 0), j1 = j + E(d, 1), k1 = k + E(d, 2);
        const double pm = A3(s, RHO1, i, j, k) * A3(s, W_PRE, i, j, k);
        const double post = pm + (A3(s, MF[d], i, j, k) - A3(s, MF[d], i1, j1, k1));
        const double pe = (A3(s, E1, i, j, k) * pm + (A3(s, W_EF, i, j, k) - A3(s, W_EF, i1, j1, k1))) / post;
        A3(s, RHO1, i, j, k) = post / A3(s, W_POST, i, j, k);
        A3(s, E1, i, j, k) = pe;
      }
}

/* dual-face mass flux of sweep d: an eighth of the 8 face mass fluxes (faces
 * p and p+e along d, the 4 cells around the node in the other two axes) */
static void nflux(h3d_state *s, int d, const int lo[3], const int hi[3]) {
  const int b = d == 0 ? 1 : 0, c = d == 2 ? 1 : 2;  /* the two other axes */
#pragma omp parallel for
  for (int k = lo[2]; k < hi[2]; k++)
    for (int j = lo[1]; j < hi[1]; j++)
      for (int i = lo[0]; i < hi[0]; i++) {
        double t[2];
        for (int e = 0; e < 2; e++) {
          int p[3] = {i, j, k};
          p[d] += e;
          double q[2][2];
          for (int y = 0; y < 2; y++)
            for (int x = 0; x < 2; x++) {
              int r[3] = {p[0], p[1], p[2]};
              r[b] -= 1 - x;
              r[c] -= 1 - y;
              q[y][x] = A3(s, MF[d], r[0], r[1], r[2]);
            }
          t[e] = (q[0][0] + q[0][1]) + (q[1][0] + q[1][1]);
        }
        A3(s, W_NF, i, j, k) = 0.125 * (t[0] + t[1]);
      }
}

static void nmass(h3d_state *s, int d) {
  const int nx = s->n[0], ny = s->n[1], nz = s->n[2];
#pragma omp parallel for
  for (int k = 0; k < nz + 1; k++)
    for (int j = 0; j < ny + 1; j++)
      for (int i = 0; i < nx + 1; i++) {
#define CM(a, b, c) (A3(s, RHO1, i - 1 + (a), j - 1 + (b), k - 1 + (c)) * A3(s, W_POST, i - 1 + (a), j - 1 + (b), k - 1 + (c)))
        const double post = 0.125 * (((CM(0, 0, 0) + CM(1, 0, 0)) + (CM(0, 1, 0) + CM(1, 1, 0))) +
                                     ((CM(0, 0, 1) + CM(1, 0, 1)) + (CM(0, 1, 1) + CM(1, 1, 1))));
#undef CM
        A3(s, W_NMPOST, i, j, k) = post;
        A3(s, W_NMPRE, i, j, k) = post + (A3(s, W_NF, i, j, k) - A3(s, W_NF, i - E(d, 0), j - E(d, 1), k - E(d, 2)));
      }
}

static void mom(h3d_state *s, int d, int vel, const int lo[3], const int hi[3]) {
  const int nx = s->n[0], ny = s->n[1], nz = s->n[2];
#pragma omp parallel for
  for (int k = lo[2]; k < hi[2]; k++)
    for (int j = lo[1]; j < hi[1]; j++)
      for (int i = lo[0]; i < hi[0]; i++) {
        const double f = A3(s, W_NF, i, j, k);
        double mf = 0.0;
        if (f > 0.0) mf = f * A3(s, vel, i, j, k);
        else if (f < 0.0) mf = f * A3(s, vel, i + E(d, 0), j + E(d, 1), k + E(d, 2));
        A3(s, W_MF, i, j, k) = mf;
      }
#pragma omp parallel for
  for (int k = 0; k < nz + 1; k++)
    for (int j = 0; j < ny + 1; j++)
      for (int i = 0; i < nx + 1; i++)
        A3(s, vel, i, j, k) = (A3(s, vel, i, j, k) * A3(s, W_NMPRE, i, j, k) +
                               (A3(s, W_MF, i - E(d, 0), j - E(d, 1), k - E(d, 2)) - A3(s, W_MF, i, j, k))) /
                              A3(s, W_NMPOST, i, j, k);
}

static double dt_cell(h3d_state *s, int i, int j, int k) {
  const double c2 = (GAMMA * GM1) * A3(s, E0, i, j, k);
  const double d = (jump(s, 0, i, j, k) + jump(s, 1, i, j, k)) + jump(s, 2, i, j, k);
  double qr = 0.0;
  if (d < 0.0) qr = (CQ2 * d) * d - (CQ1 * sqrt(c2)) * d;
  const double ce = sqrt(c2 + 2.0 * qr);
  double t = INFINITY;
  for (int a = 0; a < 3; a++) {
    const int v = VEL0[a];
#define AV(x, y, z) fabs(A3(s, v, i + (x), j + (y), k + (z)))
    const double m = fmax(fmax(fmax(AV(0, 0, 0), AV(1, 0, 0)), fmax(AV(0, 1, 0), AV(1, 1, 0))),
                          fmax(fmax(AV(0, 0, 1), AV(1, 0, 1)), fmax(AV(0, 1, 1), AV(1, 1, 1))));
#undef AV
    t = fmin(t, s->d[a] / (ce + m));
  }
  return CFL * t;
}

double h3d_dt(h3d_state *s) {
  double m = INFINITY;
#pragma omp parallel for reduction(min : m)
  for (int k = 0; k < s->n[2]; k++)
    for (int j = 0; j < s->n[1]; j++)
      for (int i = 0; i < s->n[0]; i++) {
        const double t = dt_cell(s, i, j, k);
        if (t < m) m = t;
      }
  return m;
}

void h3d_lagrangian(h3d_state *s, double dt) {
  const int *n = s->n;
  bc_state(s);
  const int cl[3] = {-H, -H, -H}, ch[3] = {n[0] + H, n[1] + H, n[2] + H};
  eos(s, RHO0, E0, 1, cl, ch);
  viscosity(s, cl, ch);
  pdv(s, 0, dt, cl, ch);
  eos(s, RHO1, E1, 0, cl, ch);
  const int nl[3] = {-1, -1, -1}, nh[3] = {n[0] + H, n[1] + H, n[2] + H};
  accelerate(s, dt, nl, nh);
  const int pl[3] = {-1, -1, -1}, ph[3] = {n[0] + 1, n[1] + 1, n[2] + 1};
  pdv(s, 1, dt, pl, ph);
}

/* strip of one field's halo layer on both walls of axis a over a box of the
 * other axes: low layer at index lo_idx <- lo_idx + o, high at hi_idx <- hi_idx - o */
static void halo_pair(h3d_state *s, int fld, double sign, int a, int lo_idx, int hi_idx, int o, const int lo[3],
                      const int hi[3]) {
  int l[3], h[3], off[3] = {0, 0, 0};
  for (int b = 0; b < 3; b++) { l[b] = lo[b]; h[b] = hi[b]; }
  l[a] = lo_idx; h[a] = lo_idx + 1; off[a] = o;
  mirror(s, fld, sign, l, h, off);
  l[a] = hi_idx; h[a] = hi_idx + 1; off[a] = -o;
  mirror(s, fld, sign, l, h, off);
}

double h3d_step(h3d_state *s, double dt) {
  const int *n = s->n;
  h3d_lagrangian(s, dt);
  for (int a = 0; a < 3; a++) flux_calc(s, a, dt);
  const int vel[3] = {U1, V1, W1};
  for (int d = 0; d < 3; d++) {
    adv_vol(s, d);
    /* faces normal to d: along d over [0, n+1); other axes over [-1, n+1) */
    int fl[3] = {-1, -1, -1}, fh[3] = {n[0] + 1, n[1] + 1, n[2] + 1};
    fl[d] = 0;
    adv_flux(s, d, fl, fh);
    int cl[3] = {-1, -1, -1}, ch[3] = {n[0] + 1, n[1] + 1, n[2] + 1};
    cl[d] = 0; ch[d] = n[d];
    adv_cell(s, d, cl, ch);
    /* density of the swept cells beyond the walls normal to d (the node
     * masses read it), and the mirror (odd) face mass flux beyond the walls.
     * Energy beyond a wall feeds only cells beyond the walls, so it is not
     * mirrored. */
    int bl[3] = {-1, -1, -1}, bh[3] = {n[0] + 1, n[1] + 1, n[2] + 1};
    halo_pair(s, RHO1, 1.0, d, -1, n[d], 1, bl, bh);
    halo_pair(s, MF[d], -1.0, d, -1, n[d] + 1, 2, bl, bh);
    int dl[3] = {0, 0, 0}, dh[3] = {n[0] + 1, n[1] + 1, n[2] + 1};
    dl[d] = -1; dh[d] = n[d] + 1;
    nflux(s, d, dl, dh);
    nmass(s, d);
    for (int v = 0; v < 3; v++) mom(s, d, vel[v], dl, dh);
    /* node velocities beyond the walls of the next sweep's axis */
    if (d < 2) {
      const int a = d + 1;
      int vl[3] = {0, 0, 0}, vh[3] = {n[0] + 1, n[1] + 1, n[2] + 1};
      for (int v = 0; v < 3; v++) halo_pair(s, vel[v], v == a ? -1.0 : 1.0, a, -1, n[a] + 1, 2, vl, vh);
    }
  }
  /* reset: the remapped state becomes the new state */
#pragma omp parallel for
  for (int k = 0; k < n[2]; k++)
    for (int j = 0; j < n[1]; j++)
      for (int i = 0; i < n[0]; i++) {
        A3(s, RHO0, i, j, k) = A3(s, RHO1, i, j, k);
        A3(s, E0, i, j, k) = A3(s, E1, i, j, k);
      }
#pragma omp parallel for
  for (int k = 0; k < n[2] + 1; k++)
    for (int j = 0; j < n[1] + 1; j++)
      for (int i = 0; i < n[0] + 1; i++) {
        A3(s, U0, i, j, k) = A3(s, U1, i, j, k);
        A3(s, V0, i, j, k) = A3(s, V1, i, j, k);
        A3(s, W0, i, j, k) = A3(s, W1, i, j, k);
      }
  return h3d_dt(s);
}

double h3d_sum_cells(h3d_state *s, int fld, int times_rho0) {
  double tot = 0.0;
  for (int k = 0; k < s->n[2]; k++)
    for (int j = 0; j < s->n[1]; j++) {
      double row = 0.0;
      for (int i = 0; i < s->n[0]; i++) {
        double v = A3(s, fld, i, j, k) * A3(s, VOL, i, j, k);
        if (times_rho0) v *= A3(s, RHO0, i, j, k);
        row += v;
      }
      tot += row;
    }
  return tot;
}
