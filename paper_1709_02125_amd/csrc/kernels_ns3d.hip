// 3D compressible Navier-Stokes proxy kernels (FP64, gfx950): primitives,
// stored first derivatives (4th-order central), and the residual with the
// 2N-storage Runge-Kutta update fused in (the OpenSBLI-style chain the paper
// tiles over several time steps, Section 5.1 and Section 5.3).  Expression
// order matches the plain program (compiled with -ffp-contract=off).
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels_device.h"
#include "ooc_internal.h"

namespace ooc {
namespace {

constexpr double kGamma = 1.4;
constexpr double kGm1 = kGamma - 1.0;

// argument slots of the residual kernel
enum { PR = 0, PU, PV, PW, PP, GUX, GTX = GUX + 9, QR = GUX + 12, DR = QR + 5 };

__device__ inline double deriv(double m2, double m1, double p1, double p2, double inv) {
  return (8.0 * (p1 - m1) - (p2 - m2)) * inv;
}

OOC_KERNEL(k_ns_init) {
  ARGS
  POINT_BEGIN
  const double r = AT(0, 0, 0, 0), u = AT(1, 0, 0, 0), v = AT(2, 0, 0, 0), w = AT(3, 0, 0, 0);
  const double p = AT(4, 0, 0, 0);
  AT(5, 0, 0, 0) = r;
  AT(6, 0, 0, 0) = r * u;
  AT(7, 0, 0, 0) = r * v;
  AT(8, 0, 0, 0) = r * w;
  AT(9, 0, 0, 0) = p / kGm1 + 0.5 * r * ((u * u + v * v) + w * w);
  POINT_END
}

OOC_KERNEL(k_ns_prims) {
  ARGS
  POINT_BEGIN
  const double r = AT(0, 0, 0, 0), ru = AT(1, 0, 0, 0), rv = AT(2, 0, 0, 0), rw = AT(3, 0, 0, 0);
  const double u = ru / r, v = rv / r, w = rw / r;
  AT(5, 0, 0, 0) = r;
  AT(6, 0, 0, 0) = u;
  AT(7, 0, 0, 0) = v;
  AT(8, 0, 0, 0) = w;
  AT(9, 0, 0, 0) = kGm1 * (AT(4, 0, 0, 0) - 0.5 * ((ru * u + rv * v) + rw * w));
  POINT_END
}

// T = gamma M^2 p / rho at an offset point
#define TEMP(di, dj, dk) ((gm2 * AT(4, di, dj, dk)) / AT(0, di, dj, dk))

OOC_KERNEL(k_ns_grads) {
  ARGS
  POINT_BEGIN
  const double inv = a.c[0], gm2 = a.c[1];
#pragma unroll
  for (int c = 0; c < 3; c++) {
    const int f = 1 + c;
    AT(5 + 3 * c, 0, 0, 0) = deriv(AT(f, -2, 0, 0), AT(f, -1, 0, 0), AT(f, 1, 0, 0), AT(f, 2, 0, 0), inv);
    AT(6 + 3 * c, 0, 0, 0) = deriv(AT(f, 0, -2, 0), AT(f, 0, -1, 0), AT(f, 0, 1, 0), AT(f, 0, 2, 0), inv);
    AT(7 + 3 * c, 0, 0, 0) = deriv(AT(f, 0, 0, -2), AT(f, 0, 0, -1), AT(f, 0, 0, 1), AT(f, 0, 0, 2), inv);
  }
  AT(14, 0, 0, 0) = deriv(TEMP(-2, 0, 0), TEMP(-1, 0, 0), TEMP(1, 0, 0), TEMP(2, 0, 0), inv);
  AT(15, 0, 0, 0) = deriv(TEMP(0, -2, 0), TEMP(0, -1, 0), TEMP(0, 1, 0), TEMP(0, 2, 0), inv);
  AT(16, 0, 0, 0) = deriv(TEMP(0, 0, -2), TEMP(0, 0, -1), TEMP(0, 0, 1), TEMP(0, 0, 2), inv);
  POINT_END
}
#undef TEMP

// total flux (convective minus viscous) along axis A at offset point (di,dj,dk)
template <int A>
__device__ inline void ns_flux(const KArgs &a, int i, int j, int k, int di, int dj, int dk, double mu,
                               double kappa, double out[5]) {
  const double r = AT(PR, di, dj, dk), p = AT(PP, di, dj, dk);
  const double u[3] = {AT(PU, di, dj, dk), AT(PV, di, dj, dk), AT(PW, di, dj, dk)};
  const double ua = u[A];
  double g[3][3];
#pragma unroll
  for (int c = 0; c < 3; c++)
#pragma unroll
    for (int b = 0; b < 3; b++) g[c][b] = AT(GUX + 3 * c + b, di, dj, dk);
  const double div = (g[0][0] + g[1][1]) + g[2][2];
  double tau[3];
#pragma unroll
  for (int c = 0; c < 3; c++) {
    double t = g[c][A] + g[A][c];
    if (c == A) t -= (2.0 / 3.0) * div;
    tau[c] = mu * t;
  }
  const double dT = AT(GTX + A, di, dj, dk);
  const double rE = p / kGm1 + 0.5 * r * ((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]);
  out[0] = r * ua;
#pragma unroll
  for (int c = 0; c < 3; c++) out[1 + c] = (r * u[c]) * ua + (c == A ? p : 0.0) - tau[c];
  out[4] = (rE + p) * ua - ((u[0] * tau[0] + u[1] * tau[1]) + u[2] * tau[2]) - kappa * dT;
}

template <int A>
__device__ inline void ns_axis(const KArgs &a, int i, int j, int k, double mu, double kappa, double inv,
                               double res[5]) {
  constexpr int ex = A == 0, ey = A == 1, ez = A == 2;
  double fm2[5], fm1[5], fp1[5], fp2[5];
  ns_flux<A>(a, i, j, k, -2 * ex, -2 * ey, -2 * ez, mu, kappa, fm2);
  ns_flux<A>(a, i, j, k, -ex, -ey, -ez, mu, kappa, fm1);
  ns_flux<A>(a, i, j, k, ex, ey, ez, mu, kappa, fp1);
  ns_flux<A>(a, i, j, k, 2 * ex, 2 * ey, 2 * ez, mu, kappa, fp2);
#pragma unroll
  for (int c = 0; c < 5; c++) res[c] -= deriv(fm2[c], fm1[c], fp1[c], fp2[c], inv);
}

template <bool kFirst>
OOC_KERNEL(k_ns_rhs) {
  ARGS
  POINT_BEGIN
  const double inv = a.c[0], mu = a.c[1], kappa = a.c[2], dt = a.c[3], A = a.c[4], B = a.c[5];
  double res[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  ns_axis<0>(a, i, j, k, mu, kappa, inv, res);
  ns_axis<1>(a, i, j, k, mu, kappa, inv, res);
  ns_axis<2>(a, i, j, k, mu, kappa, inv, res);
#pragma unroll
  for (int c = 0; c < 5; c++) {
    const double d = kFirst ? dt * res[c] : A * AT(DR + c, 0, 0, 0) + dt * res[c];
    AT(DR + c, 0, 0, 0) = d;
    AT(QR + c, 0, 0, 0) = AT(QR + c, 0, 0, 0) + B * d;
  }
  POINT_END
}

#define L(name, kern) \
  void name(const KArgs &a, const KArgs *d, int nd, void *s) { launch_point(kern, a, d, nd, s); }
L(l_init, k_ns_init)
L(l_prims, k_ns_prims)
L(l_grads, k_ns_grads)
L(l_rhs_first, k_ns_rhs<true>)
L(l_rhs, k_ns_rhs<false>)
#undef L

}  // namespace

void register_ns3d_kernels(KernelInfo *t) {
  t[OOC_K_NS_INIT] = {"ns_init", 10, 10, 0, 0, 0, kPointGrid, l_init};
  t[OOC_K_NS_PRIMS] = {"ns_prims", 10, 10, 0, 0, 0, kPointGrid, l_prims};
  t[OOC_K_NS_GRADS] = {"ns_grads", 17, 17, 2, 0, 0, kPointGrid, l_grads};
  t[OOC_K_NS_RHS_FIRST] = {"ns_rhs_first", 27, 27, 6, 0, 0, kPointGrid, l_rhs_first};
  t[OOC_K_NS_RHS] = {"ns_rhs", 27, 27, 6, 0, 0, kPointGrid, l_rhs};
}

}  // namespace ooc
