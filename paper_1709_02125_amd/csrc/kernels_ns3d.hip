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
  POINT_BEGIN_Z
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

// Residual and RK update.  A block of 64 x 4 threads owns a 64 x 4 (x, y)
// patch and walks kZRows consecutive z-planes.  Per plane, the x- and
// y-fluxes of every point the patch's differences need (the patch plus two
// columns / rows of halo each side) are evaluated once and staged in LDS, so
// the 4-point differences along x and y read LDS instead of re-evaluating
// neighbours' fluxes; the z-fluxes at k-2..k+2 are evaluated per point, their
// inputs mostly still in cache from the previous plane.  Each flux is the
// same function of the same inputs wherever it is evaluated, and the
// differences are taken in the same order (x, y, then z, subtracted from
// zero), so results equal a point-by-point evaluation exactly.
constexpr int kZRows = 4;

template <bool kFirst>
__global__ void __launch_bounds__(256) k_ns_rhs(const KArgs *__restrict__ ap) {
  ARGS
  __shared__ double sfx[5][4][68];  // x-flux, x = i0-2 .. i0+65, the patch's 4 rows
  __shared__ double sfy[5][8][64];  // y-flux, y = j0-2 .. j0+5, the patch's 64 columns
  const int n_ = (int)(gridDim.x * gridDim.y * gridDim.z);
  const int l_ = xcd_block((int)(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)), n_);
  const int bx = l_ % (int)gridDim.x, by = (l_ / (int)gridDim.x) % (int)gridDim.y;
  const int bz = l_ / (int)(gridDim.x * gridDim.y);
  const int tx = (int)threadIdx.x, ty = (int)threadIdx.y;
  const int i0 = a.lo[0] + bx * 64, j0 = a.lo[1] + by * 4;
  const int i = i0 + tx, j = j0 + ty;
  const bool xin = i < a.hi[0], yin = j < a.hi[1];
  // a flux is needed up to two points past the last point of the range
  const int xend = a.hi[0] + 2, yend = a.hi[1] + 2;
  // halo slots of this thread: x-halo column (tx < 4) and y-halo row (ty < 4)
  const int hm = tx < 2 ? tx : 64 + tx, hx = i0 - 2 + hm;
  const int hn = ty < 2 ? ty : 4 + ty, hy = j0 - 2 + hn;
  const double inv = a.c[0], mu = a.c[1], kappa = a.c[2], dt = a.c[3], A = a.c[4], B = a.c[5];
  for (int r = 0; r < kZRows; r++) {
    const int k = a.lo[2] + bz * kZRows + r;
    if (k >= a.hi[2]) break;  // the same for the whole block
    double f[5];
    if (yin && i < xend) {
      ns_flux<0>(a, i, j, k, 0, 0, 0, mu, kappa, f);
#pragma unroll
      for (int c = 0; c < 5; c++) sfx[c][ty][tx + 2] = f[c];
    }
    if (xin && j < yend) {
      ns_flux<1>(a, i, j, k, 0, 0, 0, mu, kappa, f);
#pragma unroll
      for (int c = 0; c < 5; c++) sfy[c][ty + 2][tx] = f[c];
    }
    if (tx < 4 && yin && hx < xend) {
      ns_flux<0>(a, hx, j, k, 0, 0, 0, mu, kappa, f);
#pragma unroll
      for (int c = 0; c < 5; c++) sfx[c][ty][hm] = f[c];
    }
    if (ty < 4 && xin && hy < yend) {
      ns_flux<1>(a, i, hy, k, 0, 0, 0, mu, kappa, f);
#pragma unroll
      for (int c = 0; c < 5; c++) sfy[c][hn][tx] = f[c];
    }
    __syncthreads();
    if (xin && yin) {
      double res[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int c = 0; c < 5; c++)
        res[c] -= deriv(sfx[c][ty][tx], sfx[c][ty][tx + 1], sfx[c][ty][tx + 3], sfx[c][ty][tx + 4], inv);
#pragma unroll
      for (int c = 0; c < 5; c++)
        res[c] -= deriv(sfy[c][ty][tx], sfy[c][ty + 1][tx], sfy[c][ty + 3][tx], sfy[c][ty + 4][tx], inv);
      ns_axis<2>(a, i, j, k, mu, kappa, inv, res);
#pragma unroll
      for (int c = 0; c < 5; c++) {
        const double d = kFirst ? dt * res[c] : A * AT(DR + c, 0, 0, 0) + dt * res[c];
        AT(DR + c, 0, 0, 0) = d;
        AT(QR + c, 0, 0, 0) = AT(QR + c, 0, 0, 0) + B * d;
      }
    }
    __syncthreads();  // the next plane overwrites the staged fluxes
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
void l_grads(const KArgs &a, const KArgs *d, int nd, void *s) { launch_point_z(k_ns_grads, a, d, nd, s); }
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
