// 2D hydro proxy kernels (FP64, gfx950).  One kernel per loop of the chain;
// 64 x 4 threads walking 4 rows each (the point loop of kernels_device.h), so
// each wavefront reads 64 consecutive x of a row.  The path is HBM-bound (well
// under 1 flop per byte), so there is no
// MFMA here.  Expression order matches the plain program exactly (compiled
// with -ffp-contract=off): tiled and untiled runs are bit-identical, and the
// CPU oracle agrees to rounding.
//
// Scheme: staggered-grid Lagrangian step (predictor-corrector PdV, node
// acceleration as the adjoint of the PdV volume change) and donor-cell remap
// sweeps x then y, as named for CloverLeaf 2D in the paper's Section 5.1.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels_device.h"
#include "ooc_internal.h"

namespace ooc {
namespace {

constexpr double kGamma = 1.4;
constexpr double kGm1 = 0.4;
constexpr double kCq2 = 1.0;  // quadratic viscosity coefficient
constexpr double kCq1 = 0.5;  // linear viscosity coefficient
constexpr double kCfl = 0.5;

// p = (g-1) rho e ; cs = sqrt(g p / rho)
OOC_KERNEL(k_eos) {
  ARGS
  POINT_BEGIN
  const double r = AT(0, 0, 0, 0);
  const double p = (kGm1 * r) * AT(1, 0, 0, 0);
  AT(2, 0, 0, 0) = p;
  AT(3, 0, 0, 0) = sqrt((kGamma * p) / r);
  POINT_END
}

OOC_KERNEL(k_eos_p) {
  ARGS
  POINT_BEGIN
  AT(2, 0, 0, 0) = (kGm1 * AT(0, 0, 0, 0)) * AT(1, 0, 0, 0);
  POINT_END
}

// q from the velocity jumps across the cell: compression d = du + dv < 0
OOC_KERNEL(k_visc) {
  ARGS
  POINT_BEGIN
  const double du = 0.5 * ((AT(2, 1, 0, 0) + AT(2, 1, 1, 0)) - (AT(2, 0, 0, 0) + AT(2, 0, 1, 0)));
  const double dv = 0.5 * ((AT(3, 0, 1, 0) + AT(3, 1, 1, 0)) - (AT(3, 0, 0, 0) + AT(3, 1, 0, 0)));
  const double d = du + dv;
  double q = 0.0;
  if (d < 0.0) q = AT(0, 0, 0, 0) * ((kCq2 * d) * d - (kCq1 * AT(1, 0, 0, 0)) * d);
  AT(4, 0, 0, 0) = q;
  POINT_END
}

// PdV: volume change from face fluxes (dt/4 times the summed node velocities of
// each face; the corrector sums start and end velocities), then density and
// energy update.  Argument indices of rho1/e1 depend on the phase.
template <bool kCorr>
OOC_KERNEL(k_pdv) {
  ARGS
  POINT_BEGIN
  const double fac = 0.25 * a.ds[0][0];
  double ul, ur, vb, vt;
  if (kCorr) {
    ul = (AT(7, 0, 0, 0) + AT(9, 0, 0, 0)) + (AT(7, 0, 1, 0) + AT(9, 0, 1, 0));
    ur = (AT(7, 1, 0, 0) + AT(9, 1, 0, 0)) + (AT(7, 1, 1, 0) + AT(9, 1, 1, 0));
    vb = (AT(8, 0, 0, 0) + AT(10, 0, 0, 0)) + (AT(8, 1, 0, 0) + AT(10, 1, 0, 0));
    vt = (AT(8, 0, 1, 0) + AT(10, 0, 1, 0)) + (AT(8, 1, 1, 0) + AT(10, 1, 1, 0));
  } else {
    ul = AT(7, 0, 0, 0) + AT(7, 0, 1, 0);
    ur = AT(7, 1, 0, 0) + AT(7, 1, 1, 0);
    vb = AT(8, 0, 0, 0) + AT(8, 1, 0, 0);
    vt = AT(8, 0, 1, 0) + AT(8, 1, 1, 0);
  }
  const double fl = (fac * AT(5, 0, 0, 0)) * ul;
  const double fr = (fac * AT(5, 1, 0, 0)) * ur;
  const double fb = (fac * AT(6, 0, 0, 0)) * vb;
  const double ft = (fac * AT(6, 0, 1, 0)) * vt;
  const double total = (fr - fl) + (ft - fb);
  const double vol = AT(4, 0, 0, 0);
  const double m = AT(0, 0, 0, 0) * vol;
  constexpr int R1 = kCorr ? 11 : 9, E1 = kCorr ? 12 : 10;
  AT(R1, 0, 0, 0) = m / (vol + total);
  AT(E1, 0, 0, 0) = AT(1, 0, 0, 0) - ((AT(2, 0, 0, 0) + AT(3, 0, 0, 0)) * total) / m;
  POINT_END
}

// Node acceleration from the pressure + viscosity of the four surrounding
// cells; wall-normal velocity of wall nodes held at zero.
OOC_KERNEL(k_accel) {
  ARGS
  POINT_BEGIN
  const double pbl = AT(2, -1, -1, 0) + AT(3, -1, -1, 0);
  const double pbr = AT(2, 0, -1, 0) + AT(3, 0, -1, 0);
  const double ptl = AT(2, -1, 0, 0) + AT(3, -1, 0, 0);
  const double ptr = AT(2, 0, 0, 0) + AT(3, 0, 0, 0);
  const double mass = 0.25 * ((AT(0, -1, -1, 0) * AT(1, -1, -1, 0) + AT(0, 0, -1, 0) * AT(1, 0, -1, 0)) +
                              (AT(0, -1, 0, 0) * AT(1, -1, 0, 0) + AT(0, 0, 0, 0) * AT(1, 0, 0, 0)));
  const double fx = 0.5 * (AT(4, 0, -1, 0) * (pbl - pbr) + AT(4, 0, 0, 0) * (ptl - ptr));
  const double fy = 0.5 * (AT(5, -1, 0, 0) * (pbl - ptl) + AT(5, 0, 0, 0) * (pbr - ptr));
  const double dt = a.ds[0][0];
  double u = AT(6, 0, 0, 0) + (dt * fx) / mass;
  double v = AT(7, 0, 0, 0) + (dt * fy) / mass;
  const int nx = (int)a.c[0], ny = (int)a.c[1];
  if (i == 0 || i == nx) u = 0.0;
  if (j == 0 || j == ny) v = 0.0;
  AT(8, 0, 0, 0) = u;
  AT(9, 0, 0, 0) = v;
  POINT_END
}

// face volume flux of the step; D = 0: x-faces (nodes j, j+1), D = 1: y-faces
template <int D>
OOC_KERNEL(k_flux) {
  ARGS
  POINT_BEGIN
  const int ex = D == 1, ey = D == 0;  // step to the face's second node
  const double fac = 0.25 * a.ds[0][0];
  AT(3, 0, 0, 0) = (fac * AT(0, 0, 0, 0)) * ((AT(1, 0, 0, 0) + AT(2, 0, 0, 0)) + (AT(1, ex, ey, 0) + AT(2, ex, ey, 0)));
  POINT_END
}

OOC_KERNEL(k_adv_vol_x) {
  ARGS
  POINT_BEGIN
  const double dfx = AT(1, 1, 0, 0) - AT(1, 0, 0, 0);
  const double pre = AT(0, 0, 0, 0) + (dfx + (AT(2, 0, 1, 0) - AT(2, 0, 0, 0)));
  AT(3, 0, 0, 0) = pre;
  AT(4, 0, 0, 0) = pre - dfx;
  POINT_END
}

OOC_KERNEL(k_adv_vol_y) {
  ARGS
  POINT_BEGIN
  AT(2, 0, 0, 0) = AT(0, 0, 0, 0) + (AT(1, 0, 1, 0) - AT(1, 0, 0, 0));
  AT(3, 0, 0, 0) = AT(0, 0, 0, 0);
  POINT_END
}

// donor-cell mass and energy flux through the face between cells p-e and p
template <int D>
OOC_KERNEL(k_adv_flux) {
  ARGS
  POINT_BEGIN
  const int ex = D == 0, ey = D == 1;
  const double f = AT(0, 0, 0, 0);
  double mf = 0.0, ef = 0.0;
  if (f > 0.0) {
    mf = f * AT(1, -ex, -ey, 0);
    ef = mf * AT(2, -ex, -ey, 0);
  } else if (f < 0.0) {
    mf = f * AT(1, 0, 0, 0);
    ef = mf * AT(2, 0, 0, 0);
  }
  AT(3, 0, 0, 0) = mf;
  AT(4, 0, 0, 0) = ef;
  POINT_END
}

template <int D>
OOC_KERNEL(k_adv_cell) {
  ARGS
  POINT_BEGIN
  const int ex = D == 0, ey = D == 1;
  const double pm = AT(0, 0, 0, 0) * AT(2, 0, 0, 0);
  const double post = pm + (AT(4, 0, 0, 0) - AT(4, ex, ey, 0));
  const double pe = (AT(1, 0, 0, 0) * pm + (AT(5, 0, 0, 0) - AT(5, ex, ey, 0))) / post;
  AT(0, 0, 0, 0) = post / AT(3, 0, 0, 0);
  AT(1, 0, 0, 0) = pe;
  POINT_END
}

// dual-face mass flux: mean of the four face mass fluxes around it
template <int D>
OOC_KERNEL(k_nflux) {
  ARGS
  POINT_BEGIN
  if (D == 0)
    AT(1, 0, 0, 0) = 0.25 * ((AT(0, 0, -1, 0) + AT(0, 0, 0, 0)) + (AT(0, 1, -1, 0) + AT(0, 1, 0, 0)));
  else
    AT(1, 0, 0, 0) = 0.25 * ((AT(0, -1, 0, 0) + AT(0, 0, 0, 0)) + (AT(0, -1, 1, 0) + AT(0, 0, 1, 0)));
  POINT_END
}

// node masses after the sweep (from the swept cells) and before it
template <int D>
OOC_KERNEL(k_nmass) {
  ARGS
  POINT_BEGIN
  const int ex = D == 0, ey = D == 1;
  const double post = 0.25 * ((AT(0, -1, -1, 0) * AT(1, -1, -1, 0) + AT(0, 0, -1, 0) * AT(1, 0, -1, 0)) +
                              (AT(0, -1, 0, 0) * AT(1, -1, 0, 0) + AT(0, 0, 0, 0) * AT(1, 0, 0, 0)));
  AT(3, 0, 0, 0) = post;
  AT(4, 0, 0, 0) = post + (AT(2, 0, 0, 0) - AT(2, -ex, -ey, 0));
  POINT_END
}

// donor-cell momentum flux through the dual face between nodes p and p+e
template <int D>
OOC_KERNEL(k_mflux) {
  ARGS
  POINT_BEGIN
  const int ex = D == 0, ey = D == 1;
  const double f = AT(0, 0, 0, 0);
  double mf = 0.0;
  if (f > 0.0) mf = f * AT(1, 0, 0, 0);
  else if (f < 0.0) mf = f * AT(1, ex, ey, 0);
  AT(2, 0, 0, 0) = mf;
  POINT_END
}

template <int D>
OOC_KERNEL(k_vel) {
  ARGS
  POINT_BEGIN
  const int ex = D == 0, ey = D == 1;
  AT(0, 0, 0, 0) = (AT(0, 0, 0, 0) * AT(1, 0, 0, 0) + (AT(3, -ex, -ey, 0) - AT(3, 0, 0, 0))) / AT(2, 0, 0, 0);
  POINT_END
}

// stable step of a cell, min-reduced: CFL * min over axes of spacing /
// (sqrt(c^2 + 2 q / rho) + largest node speed along the axis)
OOC_KERNEL(k_dt) {
  ARGS
  double t = INFINITY;  // smallest bound over this thread's points
  POINT_BEGIN
  {
    const double c2 = (kGamma * kGm1) * AT(0, 0, 0, 0);
    const double du = 0.5 * ((AT(1, 1, 0, 0) + AT(1, 1, 1, 0)) - (AT(1, 0, 0, 0) + AT(1, 0, 1, 0)));
    const double dv = 0.5 * ((AT(2, 0, 1, 0) + AT(2, 1, 1, 0)) - (AT(2, 0, 0, 0) + AT(2, 1, 0, 0)));
    const double d = du + dv;
    double qr = 0.0;
    if (d < 0.0) qr = (kCq2 * d) * d - (kCq1 * sqrt(c2)) * d;
    const double ce = sqrt(c2 + 2.0 * qr);
    const double um = fmax(fmax(fabs(AT(1, 0, 0, 0)), fabs(AT(1, 1, 0, 0))),
                           fmax(fabs(AT(1, 0, 1, 0)), fabs(AT(1, 1, 1, 0))));
    const double vm = fmax(fmax(fabs(AT(2, 0, 0, 0)), fabs(AT(2, 1, 0, 0))),
                           fmax(fabs(AT(2, 0, 1, 0)), fabs(AT(2, 1, 1, 0))));
    const double tx = a.c[0] / (ce + um);
    const double ty = a.c[1] / (ce + vm);
    t = fmin(t, kCfl * fmin(tx, ty));
  }
  POINT_END
  block_min_to(t, a.red[0]);
}

// Field summary of the state (the periodic diagnostic that reads many fields,
// Section 5.3): one block per row, each of the five sums in a fixed order
// (x stride 256 per thread, then a fixed tree), written to the row's partial
// slot of its SUM reduction -- volume (vol), mass (m = rho0 vol), internal
// energy (m e0), kinetic energy (m w / 2 with w the mean of u0^2 + v0^2 over
// the cell's four nodes) and pressure (p vol, p from the equation of state).
OOC_KERNEL(k_summary) {
  ARGS
  __shared__ double sm[5][256];
  const int j = a.lo[1] + blockIdx.y;
  const int k = 0;  // 2D: no plane term
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = a.lo[0] + threadIdx.x; i < a.hi[0]; i += 256) {
    const double vol = AT(0, 0, 0, 0);
    const double r = AT(1, 0, 0, 0), e = AT(2, 0, 0, 0);
    const double m = r * vol;
    const double u00 = AT(3, 0, 0, 0), u10 = AT(3, 1, 0, 0), u01 = AT(3, 0, 1, 0), u11 = AT(3, 1, 1, 0);
    const double v00 = AT(4, 0, 0, 0), v10 = AT(4, 1, 0, 0), v01 = AT(4, 0, 1, 0), v11 = AT(4, 1, 1, 0);
    const double w00 = u00 * u00 + v00 * v00, w10 = u10 * u10 + v10 * v10;
    const double w01 = u01 * u01 + v01 * v01, w11 = u11 * u11 + v11 * v11;
    const double wm = 0.25 * ((w00 + w10) + (w01 + w11));
    const double p = (kGm1 * r) * e;
    acc[0] += vol;
    acc[1] += m;
    acc[2] += m * e;
    acc[3] += m * (0.5 * wm);
    acc[4] += p * vol;
  }
  for (int q = 0; q < 5; q++) sm[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int q = 0; q < 5; q++) sm[q][threadIdx.x] += sm[q][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < 5) a.red[threadIdx.x][j + a.halo] = sm[threadIdx.x][0];
}

#define L(name, kern) \
  void name(const KArgs &a, const KArgs *d, int nd, void *s) { launch_point(kern, a, d, nd, s); }
L(l_eos, k_eos)
L(l_eos_p, k_eos_p)
L(l_visc, k_visc)
L(l_pdv_pred, k_pdv<false>)
L(l_pdv_corr, k_pdv<true>)
L(l_accel, k_accel)
L(l_flux_x, k_flux<0>)
L(l_flux_y, k_flux<1>)
L(l_adv_vol_x, k_adv_vol_x)
L(l_adv_vol_y, k_adv_vol_y)
L(l_adv_flux_x, k_adv_flux<0>)
L(l_adv_flux_y, k_adv_flux<1>)
L(l_adv_cell_x, k_adv_cell<0>)
L(l_adv_cell_y, k_adv_cell<1>)
L(l_nflux_x, k_nflux<0>)
L(l_nflux_y, k_nflux<1>)
L(l_nmass_x, k_nmass<0>)
L(l_nmass_y, k_nmass<1>)
L(l_mflux_x, k_mflux<0>)
L(l_mflux_y, k_mflux<1>)
L(l_vel_x, k_vel<0>)
L(l_vel_y, k_vel<1>)
L(l_dt, k_dt)
#undef L
void l_summary(const KArgs &a, const KArgs *d, int nd, void *s) { launch_rows(k_summary, a, d, nd, s); }

}  // namespace

void register_hydro2d_kernels(KernelInfo *t) {
  //                        name          dat  dat  const dev red
  t[OOC_K_H2D_EOS] = {"h2d_eos", 4, 4, 0, 0, 0, kPointGrid, l_eos};
  t[OOC_K_H2D_EOS_P] = {"h2d_eos_p", 3, 3, 0, 0, 0, kPointGrid, l_eos_p};
  t[OOC_K_H2D_VISC] = {"h2d_visc", 5, 5, 0, 0, 0, kPointGrid, l_visc};
  t[OOC_K_H2D_PDV_PRED] = {"h2d_pdv_pred", 11, 11, 0, 1, 0, kPointGrid, l_pdv_pred};
  t[OOC_K_H2D_PDV_CORR] = {"h2d_pdv_corr", 13, 13, 0, 1, 0, kPointGrid, l_pdv_corr};
  t[OOC_K_H2D_ACCEL] = {"h2d_accel", 10, 10, 2, 1, 0, kPointGrid, l_accel};
  t[OOC_K_H2D_FLUX_X] = {"h2d_flux_x", 4, 4, 0, 1, 0, kPointGrid, l_flux_x};
  t[OOC_K_H2D_FLUX_Y] = {"h2d_flux_y", 4, 4, 0, 1, 0, kPointGrid, l_flux_y};
  t[OOC_K_H2D_ADV_VOL_X] = {"h2d_adv_vol_x", 5, 5, 0, 0, 0, kPointGrid, l_adv_vol_x};
  t[OOC_K_H2D_ADV_VOL_Y] = {"h2d_adv_vol_y", 4, 4, 0, 0, 0, kPointGrid, l_adv_vol_y};
  t[OOC_K_H2D_ADV_FLUX_X] = {"h2d_adv_flux_x", 5, 5, 0, 0, 0, kPointGrid, l_adv_flux_x};
  t[OOC_K_H2D_ADV_FLUX_Y] = {"h2d_adv_flux_y", 5, 5, 0, 0, 0, kPointGrid, l_adv_flux_y};
  t[OOC_K_H2D_ADV_CELL_X] = {"h2d_adv_cell_x", 6, 6, 0, 0, 0, kPointGrid, l_adv_cell_x};
  t[OOC_K_H2D_ADV_CELL_Y] = {"h2d_adv_cell_y", 6, 6, 0, 0, 0, kPointGrid, l_adv_cell_y};
  t[OOC_K_H2D_NFLUX_X] = {"h2d_nflux_x", 2, 2, 0, 0, 0, kPointGrid, l_nflux_x};
  t[OOC_K_H2D_NFLUX_Y] = {"h2d_nflux_y", 2, 2, 0, 0, 0, kPointGrid, l_nflux_y};
  t[OOC_K_H2D_NMASS_X] = {"h2d_nmass_x", 5, 5, 0, 0, 0, kPointGrid, l_nmass_x};
  t[OOC_K_H2D_NMASS_Y] = {"h2d_nmass_y", 5, 5, 0, 0, 0, kPointGrid, l_nmass_y};
  t[OOC_K_H2D_MFLUX_X] = {"h2d_mflux_x", 3, 3, 0, 0, 0, kPointGrid, l_mflux_x};
  t[OOC_K_H2D_MFLUX_Y] = {"h2d_mflux_y", 3, 3, 0, 0, 0, kPointGrid, l_mflux_y};
  t[OOC_K_H2D_VEL_X] = {"h2d_vel_x", 4, 4, 0, 0, 0, kPointGrid, l_vel_x};
  t[OOC_K_H2D_VEL_Y] = {"h2d_vel_y", 4, 4, 0, 0, 0, kPointGrid, l_vel_y};
  t[OOC_K_H2D_DT] = {"h2d_dt", 3, 3, 2, 0, 1, kPointGrid, l_dt};
  t[OOC_K_H2D_SUMMARY] = {"h2d_summary", 5, 5, 0, 0, 5, kRowReduce, l_summary};
}

}  // namespace ooc
