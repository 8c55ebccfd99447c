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

// Residual and RK update.  Each thread takes kZRows consecutive z-planes of
// one (i, j) column (z-coarsened point loop), so the z-neighbours a point
// reads (k-2..k+2) were mostly loaded for the thread's previous plane and hit
// in cache instead of HBM; the block's 4 wavefronts cover 4 adjacent rows for
// the y-neighbours.  Same arithmetic as a point-per-thread form.
constexpr int kZRows = 4;

template <bool kFirst>
__global__ void __launch_bounds__(256) k_ns_rhs(const KArgs *__restrict__ ap) {
  ARGS
  const int n_ = (int)(gridDim.x * gridDim.y * gridDim.z);
  const int l_ = xcd_block((int)(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)), n_);
  const int bx = l_ % (int)gridDim.x, by = (l_ / (int)gridDim.x) % (int)gridDim.y;
  const int bz = l_ / (int)(gridDim.x * gridDim.y);
  const int i = a.lo[0] + bx * 64 + (int)threadIdx.x;
  const int j = a.lo[1] + by * 4 + (int)threadIdx.y;
  if (i >= a.hi[0] || j >= a.hi[1]) return;
  const double inv = a.c[0], mu = a.c[1], kappa = a.c[2], dt = a.c[3], A = a.c[4], B = a.c[5];
  for (int r = 0; r < kZRows; r++) {
    const int k = a.lo[2] + bz * kZRows + r;
    if (k >= a.hi[2]) break;
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
  }
}

void launch_zrows(void (*kern)(const KArgs *), const KArgs &a, const KArgs *dev, int ndim, void *s) {
  const int nx = a.hi[0] - a.lo[0], ny = a.hi[1] - a.lo[1], nz = ndim == 3 ? a.hi[2] - a.lo[2] : 1;
  if (nx <= 0 || ny <= 0 || nz <= 0) return;
  const dim3 grid((nx + 63) / 64, (ny + 3) / 4, (nz + kZRows - 1) / kZRows);
  hipLaunchKernelGGL(kern, grid, dim3(64, 4, 1), 0, (hipStream_t)s, dev);
}

#define L(name, kern) \
  void name(const KArgs &a, const KArgs *d, int nd, void *s) { launch_point(kern, a, d, nd, s); }
L(l_init, k_ns_init)
L(l_prims, k_ns_prims)
L(l_grads, k_ns_grads)
void l_rhs_first(const KArgs &a, const KArgs *d, int nd, void *s) { launch_zrows(k_ns_rhs<true>, a, d, nd, s); }
void l_rhs(const KArgs &a, const KArgs *d, int nd, void *s) { launch_zrows(k_ns_rhs<false>, a, d, nd, s); }
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
