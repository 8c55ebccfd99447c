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

// Launch shape of the z-marching kernels below: a block of 64 x PH threads
// owns a 64 x PH (x, y) patch of the range and walks a run of consecutive
// z-planes of it; grid.z cuts each patch's column into segments of at least
// kMinSegPlanes planes, as many as bring the launch to about kTargetThreads
// threads (every segment re-reads the 4 planes of stencil reach around it).
// Taller patches re-read fewer halo rows per point, but measured on 512^3 they
// were no faster (8 and 12 rows for the residual, 8 and 16 for the
// gradients: the residual is bound by the dependent load round trips of each
// plane, not by bytes), so both use 4.
constexpr int kRhsRows = 4;
constexpr int kGradRows = 4;
constexpr int kMinSegPlanes = 8;
constexpr int kTargetThreads = 2048 * 256;

template <int PH>
void launch_zmarch(void (*kern)(const KArgs *), const KArgs &a, const KArgs *dev, int ndim, void *s) {
  const int nx = a.hi[0] - x_origin(a.lo[0]), ny = a.hi[1] - a.lo[1], nz = ndim == 3 ? a.hi[2] - a.lo[2] : 1;
  if (a.hi[0] <= a.lo[0] || ny <= 0 || nz <= 0) return;
  const int gx = (nx + 63) / 64, gy = (ny + PH - 1) / PH;
  const int per = gx * gy * 64 * PH;
  const int want = (kTargetThreads + per - 1) / per;
  const int most = (nz + kMinSegPlanes - 1) / kMinSegPlanes;
  const int nseg = want < most ? want : most;
  hipLaunchKernelGGL(kern, dim3(gx, gy, nseg > 1 ? nseg : 1), dim3(64, PH, 1), 0, (hipStream_t)s, dev);
}

// Common prologue of the z-marching kernels (PH rows per patch): the block's
// patch origin (i0, j0), the thread's point (i, j), its z-segment [kb, ke),
// and which columns are needed: `own` (inside the two-point stencil reach of
// the range, so its values feed a neighbour's difference) and `out` (inside
// the range).  Block columns start at x_origin(lo), so threads left of the
// range idle.
#define ZMARCH_BEGIN(PH)                                                                         \
  const int n_ = (int)(gridDim.x * gridDim.y * gridDim.z);                                       \
  const int l_ = xcd_block((int)(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)), n_); \
  const int bx = l_ % (int)gridDim.x, by = (l_ / (int)gridDim.x) % (int)gridDim.y;               \
  const int bz = l_ / (int)(gridDim.x * gridDim.y);                                              \
  const int tx = (int)threadIdx.x, ty = (int)threadIdx.y;                                        \
  const int i0 = x_origin(a.lo[0]) + bx * 64, j0 = a.lo[1] + by * (PH);                          \
  const int i = i0 + tx, j = j0 + ty;                                                            \
  const int nz_ = a.hi[2] - a.lo[2], seg_ = (nz_ + (int)gridDim.z - 1) / (int)gridDim.z;         \
  const int kb = a.lo[2] + bz * seg_, ke = kb + seg_ < a.hi[2] ? kb + seg_ : a.hi[2];            \
  if (kb >= ke) return; /* the same for the whole block */                                       \
  const int xs = a.lo[0] - 2, xe = a.hi[0] + 2, ye = a.hi[1] + 2;                                \
  const bool own = i >= xs && i < xe && j < ye, out = i >= a.lo[0] && i < a.hi[0] && j < a.hi[1]; \
  const int64_t col = (int64_t)j * a.pitch + i;                                                  \
  /* halo slots: threads of rows ty < 4 load the y-halo rows j0-2, j0-1,     */                  \
  /* j0+PH, j0+PH+1 (LDS rows hn); threads tx < 4 of every row the x-halo    */                  \
  /* columns i0-2, i0-1, i0+64, i0+65 (LDS columns hm)                       */                  \
  const bool yhalo = ty < 4;                                                                     \
  const int hn = ty < 2 ? ty : (PH) + ty, hy = j0 - 2 + hn;                                      \
  const int hm = tx < 2 ? tx : 64 + tx, hx = i0 - 2 + hm;

// Stored first derivatives, marching along z.  Each thread keeps u, v, w and
// T = gamma M^2 p / rho of its own column for planes k-2 .. k+2 in registers,
// so every plane of the inputs is loaded once and T is evaluated once per
// point; the plane-k values of the patch plus two columns / rows of halo are
// staged in LDS for the x and y differences.  The values and the difference
// formula are those of a point-by-point evaluation, so results are identical.
template <int PH>
__global__ void __launch_bounds__(64 * PH) k_ns_grads(const KArgs *__restrict__ ap) {
  ARGS
  __shared__ double sv[4][PH + 4][68];  // u, v, w, T at plane k: y = j0-2 .. j0+PH+1, x = i0-2 .. i0+65
  ZMARCH_BEGIN(PH)
  const double inv = a.c[0], gm2 = a.c[1];
  auto load = [&](int64_t o, double v[4]) {
    v[0] = gp(a.p[1])[o];
    v[1] = gp(a.p[2])[o];
    v[2] = gp(a.p[3])[o];
    v[3] = (gm2 * gp(a.p[4])[o]) / gp(a.p[0])[o];
  };
  double rg[5][4];  // own column, planes k-2 .. k+2
  if (own)
#pragma unroll
    for (int q = 0; q < 4; q++) load((int64_t)(kb - 2 + q) * a.plane + col, rg[q]);
#pragma unroll 1
  for (int k = kb; k < ke; k++) {
    const int64_t pk = (int64_t)k * a.plane;
    if (own) {
      load(pk + 2 * a.plane + col, rg[4]);
#pragma unroll
      for (int f = 0; f < 4; f++) sv[f][ty + 2][tx + 2] = rg[2][f];
    }
    if (yhalo && i >= a.lo[0] && i < a.hi[0] && hy < ye) {
      double v[4];
      load(pk + (int64_t)hy * a.pitch + i, v);
#pragma unroll
      for (int f = 0; f < 4; f++) sv[f][hn][tx + 2] = v[f];
    }
    if (tx < 4 && j < a.hi[1] && hx >= xs && hx < xe) {
      double v[4];
      load(pk + (int64_t)j * a.pitch + hx, v);
#pragma unroll
      for (int f = 0; f < 4; f++) sv[f][ty + 2][hm] = v[f];
    }
    __syncthreads();
    if (out) {
      const int64_t o = pk + col;
#pragma unroll
      for (int c = 0; c < 3; c++) {
        gp(a.p[5 + 3 * c])[o] = deriv(sv[c][ty + 2][tx], sv[c][ty + 2][tx + 1], sv[c][ty + 2][tx + 3],
                                  sv[c][ty + 2][tx + 4], inv);
        gp(a.p[6 + 3 * c])[o] = deriv(sv[c][ty][tx + 2], sv[c][ty + 1][tx + 2], sv[c][ty + 3][tx + 2],
                                  sv[c][ty + 4][tx + 2], inv);
        gp(a.p[7 + 3 * c])[o] = deriv(rg[0][c], rg[1][c], rg[3][c], rg[4][c], inv);
      }
      gp(a.p[14])[o] = deriv(sv[3][ty + 2][tx], sv[3][ty + 2][tx + 1], sv[3][ty + 2][tx + 3], sv[3][ty + 2][tx + 4], inv);
      gp(a.p[15])[o] = deriv(sv[3][ty][tx + 2], sv[3][ty + 1][tx + 2], sv[3][ty + 3][tx + 2], sv[3][ty + 4][tx + 2], inv);
      gp(a.p[16])[o] = deriv(rg[0][3], rg[1][3], rg[3][3], rg[4][3], inv);
    }
    __syncthreads();  // the next plane overwrites the staged values
#pragma unroll
    for (int q = 0; q < 4; q++)
#pragma unroll
      for (int f = 0; f < 4; f++) rg[q][f] = rg[q + 1][f];
  }
}

// the 17 inputs of a flux at one point: rho, u, v, w, p, the 9 velocity
// gradients (u_x u_y u_z v_x ... w_z) and the 3 temperature gradients
__device__ inline void ns_load(const KArgs &a, int64_t o, double v[17]) {
#pragma unroll
  for (int f = 0; f < 17; f++) v[f] = gp(a.p[PR + f])[o];
}

// total flux (convective minus viscous) along axis A from a point's inputs
template <int A>
__device__ inline void ns_flux(const double v[17], double mu, double kappa, double out[5]) {
  const double r = v[PR], p = v[PP];
  const double u[3] = {v[PU], v[PV], v[PW]};
  const double ua = u[A];
  double g[3][3];
#pragma unroll
  for (int c = 0; c < 3; c++)
#pragma unroll
    for (int b = 0; b < 3; b++) g[c][b] = v[GUX + 3 * c + b];
  const double div = (g[0][0] + g[1][1]) + g[2][2];
  double tau[3];
#pragma unroll
  for (int c = 0; c < 3; c++) {
    double t = g[c][A] + g[A][c];
    if (c == A) t -= (2.0 / 3.0) * div;
    tau[c] = mu * t;
  }
  const double dT = v[GTX + A];
  const double rE = p / kGm1 + 0.5 * r * ((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]);
  out[0] = r * ua;
#pragma unroll
  for (int c = 0; c < 3; c++) out[1 + c] = (r * u[c]) * ua + (c == A ? p : 0.0) - tau[c];
  out[4] = (rE + p) * ua - ((u[0] * tau[0] + u[1] * tau[1]) + u[2] * tau[2]) - kappa * dT;
}

// Residual and RK update, marching along z.  Every flux is evaluated once, at
// the leading plane m = k + 2 of the march: the thread's own point gives its
// x-, y- and z-flux from one load of its 17 inputs; the x- and y-fluxes of the
// patch plus two columns / rows of halo are staged in LDS and differenced at
// once into the plane's x/y part of the residual, (0 - d/dx) - d/dy, which
// waits two planes in registers; the z-fluxes of planes k-2 .. k+2 wait in a
// register ring.  At plane k the z difference is subtracted and the
// low-storage Runge-Kutta update applied.  Each flux is the same function of
// the same inputs wherever it is evaluated and the differences are taken in
// the same order (x, y, then z, from zero), so results equal a point-by-point
// evaluation exactly.
template <bool kFirst, int PH>
__global__ void __launch_bounds__(64 * PH) k_ns_rhs(const KArgs *__restrict__ ap) {
  ARGS
  __shared__ double sfx[5][PH][68];      // x-flux at plane m, x = i0-2 .. i0+65, the patch's rows
  __shared__ double sfy[5][PH + 4][64];  // y-flux at plane m, y = j0-2 .. j0+PH+1, the patch's columns
  ZMARCH_BEGIN(PH)
  const double inv = a.c[0], mu = a.c[1], kappa = a.c[2], dt = a.c[3], A = a.c[4], B = a.c[5];
  double fz[5][5];   // own column's z-flux, planes k-2 .. k+2
  double rxy[3][5];  // own column's x/y residual part, planes k .. k+2
#pragma unroll 1
  for (int m = kb - 2; m < ke + 2; m++) {
    const int64_t pm = (int64_t)m * a.plane;
    const bool xy = m >= kb && m < ke;  // the same for the whole block
    if (own) {
      double v[17];
      ns_load(a, pm + col, v);
      ns_flux<2>(v, mu, kappa, fz[4]);
      if (xy) {
        double f[5];
        ns_flux<0>(v, mu, kappa, f);
#pragma unroll
        for (int c = 0; c < 5; c++) sfx[c][ty][tx + 2] = f[c];
        ns_flux<1>(v, mu, kappa, f);
#pragma unroll
        for (int c = 0; c < 5; c++) sfy[c][ty + 2][tx] = f[c];
      }
    }
    if (xy) {
      if (yhalo && i >= a.lo[0] && i < a.hi[0] && hy < ye) {
        double v[17], f[5];
        ns_load(a, pm + (int64_t)hy * a.pitch + i, v);
        ns_flux<1>(v, mu, kappa, f);
#pragma unroll
        for (int c = 0; c < 5; c++) sfy[c][hn][tx] = f[c];
      }
      if (tx < 4 && j < a.hi[1] && hx >= xs && hx < xe) {
        double v[17], f[5];
        ns_load(a, pm + (int64_t)j * a.pitch + hx, v);
        ns_flux<0>(v, mu, kappa, f);
#pragma unroll
        for (int c = 0; c < 5; c++) sfx[c][ty][hm] = f[c];
      }
      __syncthreads();
      if (out) {
#pragma unroll
        for (int c = 0; c < 5; c++) {
          double r = 0.0;
          r -= deriv(sfx[c][ty][tx], sfx[c][ty][tx + 1], sfx[c][ty][tx + 3], sfx[c][ty][tx + 4], inv);
          r -= deriv(sfy[c][ty][tx], sfy[c][ty + 1][tx], sfy[c][ty + 3][tx], sfy[c][ty + 4][tx], inv);
          rxy[2][c] = r;
        }
      }
      __syncthreads();  // the next plane overwrites the staged fluxes
    }
    if (m >= kb + 2 && out) {
      const int64_t o = pm - 2 * a.plane + col;  // plane k = m - 2
#pragma unroll
      for (int c = 0; c < 5; c++) {
        const double res = rxy[0][c] - deriv(fz[0][c], fz[1][c], fz[3][c], fz[4][c], inv);
        const double d = kFirst ? dt * res : A * gp(a.p[DR + c])[o] + dt * res;
        gp(a.p[DR + c])[o] = d;
        gp(a.p[QR + c])[o] = gp(a.p[QR + c])[o] + B * d;
      }
    }
#pragma unroll
    for (int c = 0; c < 5; c++) {
#pragma unroll
      for (int q = 0; q < 4; q++) fz[q][c] = fz[q + 1][c];
      rxy[0][c] = rxy[1][c];
      rxy[1][c] = rxy[2][c];
    }
  }
}

// Residual and RK update with the first derivatives evaluated on the fly from
// the primitives instead of read from stored gradient fields (so the chain
// keeps 15 fields instead of 27).  Same z-march as k_ns_rhs, with the fluxes
// of plane c evaluated when plane m = c + 2 of the primitives arrives and the
// update of plane k = c - 2 applied at the same step:
//  - each thread keeps u, v, w, T = gamma M^2 p / rho of its own column and of
//    one y-halo column (rows j0-2, j0-1, j0+4, j0+5) for planes c-2 .. c+2 in
//    registers (their z-derivatives), and rho, p for planes c .. c+2;
//  - u, v, w, T of plane c over the patch plus four columns / rows (a cross:
//    the x/y stencils of the patch and of its flux halo) are staged in LDS for
//    the x- and y-derivatives; the four x-halo flux columns load their
//    z-neighbours directly;
//  - fluxes, differences and the update then proceed as in k_ns_rhs.
// T, every derivative and every flux are the same expressions of the same
// values as in k_ns_grads and k_ns_rhs, so the results are bit-identical to
// the stored-gradient chain.
// Patches of 8 rows: a block of 512 threads (8 waves, the most that 2
// waves/SIMD at 244 VGPRs allow) and 89 KB of LDS; against 4 rows the y-halo
// columns' loads and primitives are shared by twice the points (conserved
// input, ns3d 512^3: in core 34.3 against 35.2 ms per step, out of core 43.3
// against 44.1 ms).
constexpr int kFusedRows = 8;
// planes of a fused z-segment at least: each segment re-reads 8 planes of
// primitives, so a tile's short z-range (36 planes at ns3d 512^3 with
// 4-step chains) runs as one segment (45.7 against 46.8 ms per step for
// the in-core chain cut into such tiles), while a whole 512-plane grid still
// splits in two for parallelism
constexpr int kFusedMinSegPlanes = 64;

// fused-residual argument slots: the stencil input (primitives, or with kQ
// the conserved variables), the conserved variables updated (with kQ: the
// other copy, written), the Runge-Kutta increments
enum { FPR = 0, FQR = 5, FDR = 10 };

// rho, u, v, w, p at storage offset o: the primitive fields, or (kQ) the
// same expressions of the conserved variables as k_ns_prims
template <bool kQ>
__device__ __forceinline__ void ns_prim5(const KArgs &a, int64_t o, double v[5]) {
  if (kQ) {
    const double r = gp(a.p[FPR])[o], ru = gp(a.p[FPR + 1])[o], rv = gp(a.p[FPR + 2])[o];
    const double rw = gp(a.p[FPR + 3])[o], e = gp(a.p[FPR + 4])[o];
    const double u = ru / r, vv = rv / r, w = rw / r;
    v[0] = r;
    v[1] = u;
    v[2] = vv;
    v[3] = w;
    v[4] = kGm1 * (e - 0.5 * ((ru * u + rv * vv) + rw * w));
  } else {
#pragma unroll
    for (int f = 0; f < 5; f++) v[f] = gp(a.p[FPR + f])[o];
  }
}

// u, v, w, T of the primitives at storage offset o
template <bool kQ>
__device__ __forceinline__ void ns_uvwt(const KArgs &a, int64_t o, double gm2, double out[4]) {
  if (kQ) {
    double v[5];
    ns_prim5<true>(a, o, v);
    out[0] = v[1];
    out[1] = v[2];
    out[2] = v[3];
    out[3] = (gm2 * v[4]) / v[0];
  } else {
    out[0] = gp(a.p[FPR + 1])[o];
    out[1] = gp(a.p[FPR + 2])[o];
    out[2] = gp(a.p[FPR + 3])[o];
    out[3] = (gm2 * gp(a.p[FPR + 4])[o]) / gp(a.p[FPR])[o];
  }
}

// the 17 flux inputs at one point from its rho, p, the staged plane (row
// sy, column sx of sv) and its z-column values zc[0..4] (planes c-2 .. c+2)
template <int R, int C>
__device__ __forceinline__ void ns_inputs(const double (&sv)[4][R][C], int sy, int sx, const double (&zc)[5][4],
                                          double rho, double p, double inv, double v[17]) {
  v[PR] = rho;
  v[PU] = zc[2][0];
  v[PV] = zc[2][1];
  v[PW] = zc[2][2];
  v[PP] = p;
#pragma unroll
  for (int c = 0; c < 3; c++) {
    v[GUX + 3 * c] = deriv(sv[c][sy][sx - 2], sv[c][sy][sx - 1], sv[c][sy][sx + 1], sv[c][sy][sx + 2], inv);
    v[GUX + 3 * c + 1] = deriv(sv[c][sy - 2][sx], sv[c][sy - 1][sx], sv[c][sy + 1][sx], sv[c][sy + 2][sx], inv);
    v[GUX + 3 * c + 2] = deriv(zc[0][c], zc[1][c], zc[3][c], zc[4][c], inv);
  }
  v[GTX] = deriv(sv[3][sy][sx - 2], sv[3][sy][sx - 1], sv[3][sy][sx + 1], sv[3][sy][sx + 2], inv);
  v[GTX + 1] = deriv(sv[3][sy - 2][sx], sv[3][sy - 1][sx], sv[3][sy + 1][sx], sv[3][sy + 2][sx], inv);
  v[GTX + 2] = deriv(zc[0][3], zc[1][3], zc[3][3], zc[4][3], inv);
}

template <bool kFirst, int PH, bool kQ>
__global__ void __launch_bounds__(64 * PH) k_ns_rhs_fused(const KArgs *__restrict__ ap) {
  ARGS
  // u, v, w, T at plane c: rows y = j0-4 .. j0+PH+3, columns x = i0-4 .. i0+67
  __shared__ double sv[4][PH + 8][72];
  __shared__ double sfx[5][PH][68];      // x-flux at plane c, x = i0-2 .. i0+65, the patch's rows
  __shared__ double sfy[5][PH + 4][64];  // y-flux at plane c, y = j0-2 .. j0+PH+1, the patch's columns
  ZMARCH_BEGIN(PH)
  const double inv = a.c[0], mu = a.c[1], kappa = a.c[2], dt = a.c[3], A = a.c[4], B = a.c[5], gm2 = a.c[6];
  // columns and rows whose primitives exist: the range plus 4 on each side
  const int xl = a.lo[0] - 4, xh = a.hi[0] + 4, yl = a.lo[1] - 4, yh = a.hi[1] + 4;
  const bool inx = i >= a.lo[0] && i < a.hi[0];
  // own column (i, j): flux point if `own`; loaded wherever it exists
  const bool own_ld = i >= xl && i < xh && j < yh;
  // y-halo column (i, hy): a flux point for the patch's y differences
  const bool yh_flux = yhalo && inx && hy < ye;
  const bool yh_ld = yhalo && i >= xl && i < xh && hy >= yl && hy < yh;
  // staged-only points of plane c: outer rows (i, oy); the y-halo rows' x
  // extension (hx, hy) for tx < 4; the patch rows' x extension (ox, j) for tx < 8
  const int orow = ty < 2 ? ty : PH + 4 + ty, oy = j0 - 4 + orow;
  const bool oy_ld = yhalo && inx && oy >= yl && oy < yh;
  const bool hxy_ld = yhalo && tx < 4 && hx >= xl && hx < xh && hy >= yl && hy < yh;
  const int om = tx < 4 ? tx : 64 + tx, ox = i0 - 4 + om;
  const bool ox_ld = tx < 8 && ox >= xl && ox < xh && j < yh;
  // x-halo flux columns i0-2, i0-1, i0+64, i0+65 (tx = 2 .. 5) in the patch's rows
  const bool xh_flux = tx >= 2 && tx < 6 && ox >= xs && ox < xe && j < a.hi[1];
  const int64_t ycol = (int64_t)hy * a.pitch + i;
  const int64_t ocol = (int64_t)oy * a.pitch + i, hcol = (int64_t)hy * a.pitch + hx;
  const int64_t xcol = (int64_t)j * a.pitch + ox;
  // own / y-halo column: u, v, w, T at planes c-2 .. c+2 (the newest plane
  // holds p until its T is formed), rho, p at planes c .. c+2
  double za[5][4], zb[5][4], ra[3][2], rb[3][2];
  double fz[5][5];   // own column's z-flux, planes k-2 .. k+2
  double rxy[3][5];  // own column's x/y residual part, planes k .. k+2
  // ring columns are loaded unconditionally, from a column clamped into the
  // primitives' extent where the thread's own one lies outside (its values
  // are then never used): no branch around the loads, so the wait for the
  // staging loads before them does not also wait for these
  const int64_t col_ld = own_ld ? col : (int64_t)(j < yh ? j : yh - 1) * a.pitch + (i < xl ? xl : (i < xh ? i : xh - 1));
  const int hyc = hy < yl ? yl : (hy < yh ? hy : yh - 1);
  const int64_t ycol_ld = yh_ld ? ycol : (int64_t)hyc * a.pitch + (i < xl ? xl : (i < xh ? i : xh - 1));
  // raw loads: u, v, w into z[0..2], rho, p into r[0..1] (kQ: rho u, rho v,
  // rho w and rho, E); form_t then completes the point after the loads have
  // arrived (kQ: the primitives first, as k_ns_prims evaluates them)
  auto load_raw = [&](int64_t o, double z[4], double r[2]) {
    z[0] = gp(a.p[FPR + 1])[o];
    z[1] = gp(a.p[FPR + 2])[o];
    z[2] = gp(a.p[FPR + 3])[o];
    r[0] = gp(a.p[FPR])[o];
    r[1] = gp(a.p[FPR + 4])[o];
  };
  auto form_t = [&](double z[4], double r[2]) {
    if (kQ) {
      const double ru = z[0], rv = z[1], rw = z[2];
      z[0] = ru / r[0];
      z[1] = rv / r[0];
      z[2] = rw / r[0];
      r[1] = kGm1 * (r[1] - 0.5 * ((ru * z[0] + rv * z[1]) + rw * z[2]));
    }
    z[3] = (gm2 * r[1]) / r[0];
  };
#pragma unroll
  for (int q = 0; q < 4; q++) {  // planes kb-4 .. kb-1
    const int64_t pq = (int64_t)(kb - 4 + q) * a.plane;
    double r[2], s2[2];
    load_raw(pq + col_ld, za[q], r);
    load_raw(pq + ycol_ld, zb[q], s2);
    form_t(za[q], r);
    form_t(zb[q], s2);
    if (q >= 2) {
      ra[q - 2][0] = r[0];
      ra[q - 2][1] = r[1];
      rb[q - 2][0] = s2[0];
      rb[q - 2][1] = s2[1];
    }
  }
#pragma unroll 1
  for (int c = kb - 2; c < ke + 2; c++) {
    const int64_t pc = (int64_t)c * a.plane;
    const bool xy = c >= kb && c < ke;  // the same for the whole block
    // ---- loads of plane c for the staging first, then the leading plane
    // m = c + 2 of the rings:
    // the staging waits only for the former, the rings' loads complete
    // behind it and are used after the barrier
    double ov[4], hxv[4], hv[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, zc[5][4];
    if (oy_ld) ns_uvwt<kQ>(a, pc + ocol, gm2, ov);
    if (hxy_ld) ns_uvwt<kQ>(a, pc + hcol, gm2, hxv);
    if (ox_ld) ns_prim5<kQ>(a, pc + xcol, hv);
    load_raw(pc + 2 * a.plane + col_ld, za[4], ra[2]);
    load_raw(pc + 2 * a.plane + ycol_ld, zb[4], rb[2]);
    // ---- stage plane c
#pragma unroll
    for (int f = 0; f < 4; f++) {
      if (own_ld) sv[f][ty + 4][tx + 4] = za[2][f];
      if (yh_ld) sv[f][hn + 2][tx + 4] = zb[2][f];
      if (oy_ld) sv[f][orow][tx + 4] = ov[f];
      if (hxy_ld) sv[f][hn + 2][hm + 2] = hxv[f];
    }
    if (ox_ld) {
      sv[0][ty + 4][om] = hv[1];
      sv[1][ty + 4][om] = hv[2];
      sv[2][ty + 4][om] = hv[3];
      sv[3][ty + 4][om] = (gm2 * hv[4]) / hv[0];
    }
    __syncthreads();
    // keep the scheduler from forming T (which waits for the rings' loads)
    // before the barrier
    __builtin_amdgcn_sched_barrier(0);
    form_t(za[4], ra[2]);
    form_t(zb[4], rb[2]);
    // ---- fluxes of plane c
    if (own) {
      double v[17];
      ns_inputs(sv, ty + 4, tx + 4, za, ra[0][0], ra[0][1], inv, v);
      ns_flux<2>(v, mu, kappa, fz[4]);
      if (xy) {
        double f[5];
        ns_flux<0>(v, mu, kappa, f);
#pragma unroll
        for (int q = 0; q < 5; q++) sfx[q][ty][tx + 2] = f[q];
        ns_flux<1>(v, mu, kappa, f);
#pragma unroll
        for (int q = 0; q < 5; q++) sfy[q][ty + 2][tx] = f[q];
      }
    }
    if (xy) {
      if (yh_flux) {
        double v[17], f[5];
        ns_inputs(sv, hn + 2, tx + 4, zb, rb[0][0], rb[0][1], inv, v);
        ns_flux<1>(v, mu, kappa, f);
#pragma unroll
        for (int q = 0; q < 5; q++) sfy[q][hn][tx] = f[q];
      }
      if (xh_flux) {
#pragma unroll
        for (int q = 0; q < 5; q++)
          if (q != 2) ns_uvwt<kQ>(a, pc + (int64_t)(q - 2) * a.plane + xcol, gm2, zc[q]);
        zc[2][0] = hv[1];
        zc[2][1] = hv[2];
        zc[2][2] = hv[3];
        zc[2][3] = 0.0;  // T at the point itself is not used by its derivatives
        double v[17], f[5];
        ns_inputs(sv, ty + 4, om, zc, hv[0], hv[4], inv, v);
        ns_flux<0>(v, mu, kappa, f);
#pragma unroll
        for (int q = 0; q < 5; q++) sfx[q][ty][om - 2] = f[q];
      }
      __syncthreads();
      if (out) {
#pragma unroll
        for (int q = 0; q < 5; q++) {
          double r = 0.0;
          r -= deriv(sfx[q][ty][tx], sfx[q][ty][tx + 1], sfx[q][ty][tx + 3], sfx[q][ty][tx + 4], inv);
          r -= deriv(sfy[q][ty][tx], sfy[q][ty + 1][tx], sfy[q][ty + 3][tx], sfy[q][ty + 4][tx], inv);
          rxy[2][q] = r;
        }
      }
    }
    __syncthreads();  // the next plane overwrites the staged values and fluxes
    if (c >= kb + 2 && out) {
      const int64_t o = pc - 2 * a.plane + col;  // plane k = c - 2
#pragma unroll
      for (int q = 0; q < 5; q++) {
        const double res = rxy[0][q] - deriv(fz[0][q], fz[1][q], fz[3][q], fz[4][q], inv);
        const double d = kFirst ? dt * res : A * gp(a.p[FDR + q])[o] + dt * res;
        gp(a.p[FDR + q])[o] = d;
        gp(a.p[FQR + q])[o] = gp(a.p[kQ ? FPR + q : FQR + q])[o] + B * d;
      }
    }
#pragma unroll
    for (int f = 0; f < 4; f++)
#pragma unroll
      for (int q = 0; q < 4; q++) {
        za[q][f] = za[q + 1][f];
        zb[q][f] = zb[q + 1][f];
      }
#pragma unroll
    for (int q = 0; q < 2; q++) {
      ra[q][0] = ra[q + 1][0];
      ra[q][1] = ra[q + 1][1];
      rb[q][0] = rb[q + 1][0];
      rb[q][1] = rb[q + 1][1];
    }
#pragma unroll
    for (int q = 0; q < 5; q++) {
#pragma unroll
      for (int r = 0; r < 4; r++) fz[r][q] = fz[r + 1][q];
      rxy[0][q] = rxy[1][q];
      rxy[1][q] = rxy[2][q];
    }
  }
}

template <int PH, int MINSEG>
void launch_zmarch_seg(void (*kern)(const KArgs *), const KArgs &a, const KArgs *dev, int ndim, void *s) {
  const int nx = a.hi[0] - x_origin(a.lo[0]), ny = a.hi[1] - a.lo[1], nz = ndim == 3 ? a.hi[2] - a.lo[2] : 1;
  if (a.hi[0] <= a.lo[0] || ny <= 0 || nz <= 0) return;
  const int gx = (nx + 63) / 64, gy = (ny + PH - 1) / PH;
  const int per = gx * gy * 64 * PH;
  const int want = (kTargetThreads + per - 1) / per;
  const int most = (nz + MINSEG - 1) / MINSEG;
  const int nseg = want < most ? want : most;
  hipLaunchKernelGGL(kern, dim3(gx, gy, nseg > 1 ? nseg : 1), dim3(64, PH, 1), 0, (hipStream_t)s, dev);
}

#define L(name, kern) \
  void name(const KArgs &a, const KArgs *d, int nd, void *s) { launch_point(kern, a, d, nd, s); }
L(l_init, k_ns_init)
L(l_prims, k_ns_prims)
void l_grads(const KArgs &a, const KArgs *d, int nd, void *s) {
  launch_zmarch<kGradRows>(k_ns_grads<kGradRows>, a, d, nd, s);
}
void l_rhs_first(const KArgs &a, const KArgs *d, int nd, void *s) {
  launch_zmarch<kRhsRows>(k_ns_rhs<true, kRhsRows>, a, d, nd, s);
}
void l_rhs(const KArgs &a, const KArgs *d, int nd, void *s) {
  launch_zmarch<kRhsRows>(k_ns_rhs<false, kRhsRows>, a, d, nd, s);
}
void l_rhs_fused_first(const KArgs &a, const KArgs *d, int nd, void *s) {
  launch_zmarch_seg<kFusedRows, kFusedMinSegPlanes>(k_ns_rhs_fused<true, kFusedRows, false>, a, d, nd, s);
}
void l_rhs_fused(const KArgs &a, const KArgs *d, int nd, void *s) {
  launch_zmarch_seg<kFusedRows, kFusedMinSegPlanes>(k_ns_rhs_fused<false, kFusedRows, false>, a, d, nd, s);
}
void l_rhs_fusedq_first(const KArgs &a, const KArgs *d, int nd, void *s) {
  launch_zmarch_seg<kFusedRows, kFusedMinSegPlanes>(k_ns_rhs_fused<true, kFusedRows, true>, a, d, nd, s);
}
void l_rhs_fusedq(const KArgs &a, const KArgs *d, int nd, void *s) {
  launch_zmarch_seg<kFusedRows, kFusedMinSegPlanes>(k_ns_rhs_fused<false, kFusedRows, true>, a, d, nd, s);
}
#undef L

}  // namespace

void register_ns3d_kernels(KernelInfo *t) {
  t[OOC_K_NS_INIT] = {"ns_init", 10, 10, 0, 0, 0, kPointGrid, l_init};
  t[OOC_K_NS_PRIMS] = {"ns_prims", 10, 10, 0, 0, 0, kPointGrid, l_prims};
  t[OOC_K_NS_GRADS] = {"ns_grads", 17, 17, 2, 0, 0, kPointGrid, l_grads};
  t[OOC_K_NS_RHS_FIRST] = {"ns_rhs_first", 27, 27, 6, 0, 0, kPointGrid, l_rhs_first};
  t[OOC_K_NS_RHS] = {"ns_rhs", 27, 27, 6, 0, 0, kPointGrid, l_rhs};
  t[OOC_K_NS_RHS_FUSED_FIRST] = {"ns_rhs_fused_first", 15, 15, 7, 0, 0, kPointGrid, l_rhs_fused_first};
  t[OOC_K_NS_RHS_FUSED] = {"ns_rhs_fused", 15, 15, 7, 0, 0, kPointGrid, l_rhs_fused};
  t[OOC_K_NS_RHS_FUSEDQ_FIRST] = {"ns_rhs_fusedq_first", 15, 15, 7, 0, 0, kPointGrid, l_rhs_fusedq_first};
  t[OOC_K_NS_RHS_FUSEDQ] = {"ns_rhs_fusedq", 15, 15, 7, 0, 0, kPointGrid, l_rhs_fusedq};
}

}  // namespace ooc
