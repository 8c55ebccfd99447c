// 3D hydro proxy kernels (FP64, gfx950): the three-dimensional form of the 2D
// proxy -- 8-node cell stencils and 8-cell node stencils, donor-cell remap
// sweeps x, y, z -- as the paper names CloverLeaf 3D (Section 5.1).  One kernel
// per loop over the z-walking point loop of kernels_device.h (one wavefront
// per 64 consecutive x of a row, the block's 4 wavefronts on 4 adjacent rows,
// each thread walking 4 consecutive z-planes, so both the j+1 and the k+1
// stencil reads mostly hit in cache).  The kernels with 8-point stencils
// (viscosity, PdV, acceleration, node mass, time step) keep what one plane
// loads for its upper z side in registers as the next plane's lower side.
// HBM-bound, no MFMA.
// Expression order follows the plain program exactly (built without FP
// contraction), so tiled and untiled runs are bit-identical.
//
// The equation of state kernels of the 2D proxy are point-wise and serve here
// unchanged.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels_device.h"
#include "ooc_internal.h"

namespace ooc {
namespace {

constexpr double kGamma = 1.4;
constexpr double kGm1 = 0.4;
constexpr double kCq2 = 1.0;
constexpr double kCq1 = 0.5;
constexpr double kCfl = 0.5;

// Sum over the 4 nodes of the face normal to axis AX, at offset e along AX
// (0 = the cell's lower face, 1 = its upper face), of start-plus-end values
// (node fields n0, n1)
template <int AX>
__device__ __forceinline__ double face4_2(const KArgs &a, int n0, int n1, int i, int j, int k, int e) {
#define P2(di, dj, dk) (AT(n0, di, dj, dk) + AT(n1, di, dj, dk))
  if (AX == 0) return (P2(e, 0, 0) + P2(e, 1, 0)) + (P2(e, 0, 1) + P2(e, 1, 1));
  if (AX == 1) return (P2(0, e, 0) + P2(1, e, 0)) + (P2(0, e, 1) + P2(1, e, 1));
  return (P2(0, 0, e) + P2(1, 0, e)) + (P2(0, 1, e) + P2(1, 1, e));
#undef P2
}

// The z-walk of the point loop with values carried from one plane to the
// next: the same block and thread mapping as POINT_BEGIN_Z (64 x 4 threads,
// each walking kPlanesPerThread consecutive z-planes of its (i, j) column),
// opened as a plain scope so a kernel can keep what plane k loaded for its
// upper half (k+1 side) and use it as plane k+1's lower half instead of
// loading it again.  The values are the same loads the point form makes, so
// the results are identical.
#define ZWALK_BEGIN                                                                               \
  const int n_ = (int)(gridDim.x * gridDim.y * gridDim.z);                                        \
  const int l_ = xcd_block((int)(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)), n_); \
  const int bx_ = l_ % (int)gridDim.x, by_ = (l_ / (int)gridDim.x) % (int)gridDim.y;              \
  const int i = x_origin(a.lo[0]) + bx_ * 64 + (int)threadIdx.x;                                  \
  const int j = a.lo[1] + by_ * 4 + (int)threadIdx.y;                                             \
  const int k0 = a.lo[2] + (l_ / (int)(gridDim.x * gridDim.y)) * kPlanesPerThread;                \
  const int k1 = k0 + kPlanesPerThread < a.hi[2] ? k0 + kPlanesPerThread : a.hi[2];               \
  if (i < a.lo[0] || i >= a.hi[0] || j >= a.hi[1] || k0 >= k1) return;

// Velocity jumps across a cell, walking z: each axis' jump is a quarter of
// (upper-face sum - lower-face sum) of the 4 face-node values, and the x- and
// y-face sums are split into node pairs at the cell's lower and upper z; the
// upper pairs and the upper z-face sum are the next plane's lower ones.
struct JumpCarry {
  double xl, xh, yl, yh, z;  // x pairs (lower / upper x face), y pairs, z-face sum, at one z
};

// node pairs and z sum at node plane k + dk of velocity fields nu, nv, nw
__device__ __forceinline__ JumpCarry jump_plane(const KArgs &a, int nu, int nv, int nw, int i, int j, int k,
                                                int dk) {
  JumpCarry c;
  c.xl = AT(nu, 0, 0, dk) + AT(nu, 0, 1, dk);
  c.xh = AT(nu, 1, 0, dk) + AT(nu, 1, 1, dk);
  c.yl = AT(nv, 0, 0, dk) + AT(nv, 1, 0, dk);
  c.yh = AT(nv, 0, 1, dk) + AT(nv, 1, 1, dk);
  c.z = (AT(nw, 0, 0, dk) + AT(nw, 1, 0, dk)) + (AT(nw, 0, 1, dk) + AT(nw, 1, 1, dk));
  return c;
}

// (jump x + jump y) + jump z of a cell from its lower (lo) and upper (hi) planes
__device__ __forceinline__ double jump_sum(const JumpCarry &lo, const JumpCarry &hi) {
  const double jx = 0.25 * ((lo.xh + hi.xh) - (lo.xl + hi.xl));
  const double jy = 0.25 * ((lo.yh + hi.yh) - (lo.yl + hi.yl));
  const double jz = 0.25 * (hi.z - lo.z);
  return (jx + jy) + jz;
}

// args: R rho0, R cs, R u0, R v0, R w0, W q
__global__ void __launch_bounds__(256) k_visc(const KArgs *__restrict__ ap) {
  ARGS
  int k;
  ZWALK_BEGIN
  k = k0;
  JumpCarry lo = jump_plane(a, 2, 3, 4, i, j, k, 0);
  for (; k < k1; k++) {
    const JumpCarry hi = jump_plane(a, 2, 3, 4, i, j, k, 1);
    const double d = jump_sum(lo, hi);
    double q = 0.0;
    if (d < 0.0) q = AT(0, 0, 0, 0) * ((kCq2 * d) * d - (kCq1 * AT(1, 0, 0, 0)) * d);
    AT(5, 0, 0, 0) = q;
    lo = hi;
  }
}

// PdV predictor / corrector.  args: 0 rho0, 1 e0, 2 p, 3 q, 4 vol, 5..7 x/y/z
// area, 8..10 u0 v0 w0, [corrector: 11..13 u1 v1 w1], then W rho1, W e1.
// Per cell, the volume change is the sum over axes of area x (sum of the 4
// face-node velocities) on the upper face minus the same on the lower face.
// Walking z, the x- and y-face sums split into their node pairs at the
// cell's lower and upper z (the upper pair is the next plane's lower pair),
// and the z-face sum and area of the upper face are the next plane's lower
// ones, so each plane loads only the nodes and areas of its upper z.
template <bool kCorr>
__global__ void __launch_bounds__(256) k_pdv(const KArgs *__restrict__ ap) {
  ARGS
  int k;
  ZWALK_BEGIN
  const double fac = 0.125 * a.ds[0][0];
  // node velocity along axis f at (i+di, j+dj, k+dk): start value, or start
  // plus end value for the corrector
  auto nv = [&](int f, int di, int dj, int dk) -> double {
    return kCorr ? AT(8 + f, di, dj, dk) + AT(11 + f, di, dj, dk) : AT(8 + f, di, dj, dk);
  };
  // x faces (e = lower / upper x): pair of nodes at one z; y faces likewise;
  // z face: the 4 nodes at one z
  auto xpair = [&](int e, int dk) { return nv(0, e, 0, dk) + nv(0, e, 1, dk); };
  auto ypair = [&](int e, int dk) { return nv(1, 0, e, dk) + nv(1, 1, e, dk); };
  auto zsum = [&](int dk) { return (nv(2, 0, 0, dk) + nv(2, 1, 0, dk)) + (nv(2, 0, 1, dk) + nv(2, 1, 1, dk)); };
  k = k0;
  double xl0 = xpair(0, 0), xh0 = xpair(1, 0), yl0 = ypair(0, 0), yh0 = ypair(1, 0);
  double zlo = zsum(0), azlo = AT(7, 0, 0, 0);
  constexpr int R1 = kCorr ? 14 : 11, E1 = kCorr ? 15 : 12;
  for (; k < k1; k++) {
    const double xl1 = xpair(0, 1), xh1 = xpair(1, 1), yl1 = ypair(0, 1), yh1 = ypair(1, 1);
    const double zhi = zsum(1), azhi = AT(7, 0, 0, 1);
    const double dfx = (fac * AT(5, 1, 0, 0)) * (xh0 + xh1) - (fac * AT(5, 0, 0, 0)) * (xl0 + xl1);
    const double dfy = (fac * AT(6, 0, 1, 0)) * (yh0 + yh1) - (fac * AT(6, 0, 0, 0)) * (yl0 + yl1);
    const double dfz = (fac * azhi) * zhi - (fac * azlo) * zlo;
    const double total = (dfx + dfy) + dfz;
    const double vol = AT(4, 0, 0, 0);
    const double m = AT(0, 0, 0, 0) * vol;
    AT(R1, 0, 0, 0) = m / (vol + total);
    AT(E1, 0, 0, 0) = AT(1, 0, 0, 0) - ((AT(2, 0, 0, 0) + AT(3, 0, 0, 0)) * total) / m;
    xl0 = xl1;
    xh0 = xh1;
    yl0 = yl1;
    yh0 = yh1;
    zlo = zhi;
    azlo = azhi;
  }
}

// Node acceleration: the force along each axis is a quarter of the sum, over
// the 4 faces normal to it around the node, of area x (P lower - P upper),
// the adjoint of the PdV volume change; node mass an eighth of its 8 cells.
// args: 0 rho0, 1 vol, 2 p, 3 q, 4..6 x/y/z area, 7..9 u0 v0 w0, 10..12 u1 v1
// w1; CONST nx, ny, nz; DEVSCALAR dt.  Walking z, a node's upper cells
// (pressure p + q, mass rho vol) and the x- and y-face areas at its upper z
// are the next node's lower ones and are carried, not loaded again.
__global__ void __launch_bounds__(256) k_accel(const KArgs *__restrict__ ap) {
  ARGS
  int k;
  ZWALK_BEGIN
  const double dt = a.ds[0][0];
  double P0[2][2], M0[2][2], ax0[2], ay0[2];  // cells below the node's plane: [b = y][e = x]
  k = k0;
#pragma unroll
  for (int b = 0; b < 2; b++) {
#pragma unroll
    for (int e = 0; e < 2; e++) {
      P0[b][e] = AT(2, e - 1, b - 1, -1) + AT(3, e - 1, b - 1, -1);
      M0[b][e] = AT(0, e - 1, b - 1, -1) * AT(1, e - 1, b - 1, -1);
    }
    ax0[b] = AT(4, 0, b - 1, -1);
    ay0[b] = AT(5, b - 1, 0, -1);
  }
  for (; k < k1; k++) {
    double P1[2][2], M1[2][2], ax1[2], ay1[2];
#pragma unroll
    for (int b = 0; b < 2; b++) {
#pragma unroll
      for (int e = 0; e < 2; e++) {
        P1[b][e] = AT(2, e - 1, b - 1, 0) + AT(3, e - 1, b - 1, 0);
        M1[b][e] = AT(0, e - 1, b - 1, 0) * AT(1, e - 1, b - 1, 0);
      }
      ax1[b] = AT(4, 0, b - 1, 0);
      ay1[b] = AT(5, b - 1, 0, 0);
    }
    const double mass = 0.125 * (((M0[0][0] + M0[0][1]) + (M0[1][0] + M0[1][1])) +
                                 ((M1[0][0] + M1[0][1]) + (M1[1][0] + M1[1][1])));
    const double fx = 0.25 * ((ax0[0] * (P0[0][0] - P0[0][1]) + ax0[1] * (P0[1][0] - P0[1][1])) +
                              (ax1[0] * (P1[0][0] - P1[0][1]) + ax1[1] * (P1[1][0] - P1[1][1])));
    const double fy = 0.25 * ((ay0[0] * (P0[0][0] - P0[1][0]) + ay0[1] * (P0[0][1] - P0[1][1])) +
                              (ay1[0] * (P1[0][0] - P1[1][0]) + ay1[1] * (P1[0][1] - P1[1][1])));
    const double fz = 0.25 * ((AT(6, -1, -1, 0) * (P0[0][0] - P1[0][0]) + AT(6, 0, -1, 0) * (P0[0][1] - P1[0][1])) +
                              (AT(6, -1, 0, 0) * (P0[1][0] - P1[1][0]) + AT(6, 0, 0, 0) * (P0[1][1] - P1[1][1])));
    double u = AT(7, 0, 0, 0) + (dt * fx) / mass;
    double v = AT(8, 0, 0, 0) + (dt * fy) / mass;
    double w = AT(9, 0, 0, 0) + (dt * fz) / mass;
    if (i == 0 || i == (int)a.c[0]) u = 0.0;
    if (j == 0 || j == (int)a.c[1]) v = 0.0;
    if (k == 0 || k == (int)a.c[2]) w = 0.0;
    AT(10, 0, 0, 0) = u;
    AT(11, 0, 0, 0) = v;
    AT(12, 0, 0, 0) = w;
#pragma unroll
    for (int b = 0; b < 2; b++) {
#pragma unroll
      for (int e = 0; e < 2; e++) {
        P0[b][e] = P1[b][e];
        M0[b][e] = M1[b][e];
      }
      ax0[b] = ax1[b];
      ay0[b] = ay1[b];
    }
  }
}

// face volume flux along D.  args: R area, R vel0, R vel1, W vf; DEVSCALAR dt
template <int D>
OOC_KERNEL(k_flux) {
  ARGS
  POINT_BEGIN_Z
  const double fac = 0.125 * a.ds[0][0];
  AT(3, 0, 0, 0) = (fac * AT(0, 0, 0, 0)) * face4_2<D>(a, 1, 2, i, j, k, 0);
  POINT_END
}

// volume change through the faces normal to axis AX of field n
template <int AX>
__device__ __forceinline__ double dflux(const KArgs &a, int n, int i, int j, int k) {
  return AT(n, AX == 0, AX == 1, AX == 2) - AT(n, 0, 0, 0);
}

// volumes before / after the x sweep.  args: R vol, R vfx, R vfy, R vfz, W pre, W post
OOC_KERNEL(k_adv_vol_x) {
  ARGS
  POINT_BEGIN_Z
  const double dfx = dflux<0>(a, 1, i, j, k);
  const double pre = AT(0, 0, 0, 0) + ((dfx + dflux<1>(a, 2, i, j, k)) + dflux<2>(a, 3, i, j, k));
  AT(4, 0, 0, 0) = pre;
  AT(5, 0, 0, 0) = pre - dfx;
  POINT_END
}

// y sweep.  args: R vol, R vfy, R vfz, W pre, W post
OOC_KERNEL(k_adv_vol_y) {
  ARGS
  POINT_BEGIN_Z
  const double vol = AT(0, 0, 0, 0);
  const double dfz = dflux<2>(a, 2, i, j, k);
  AT(3, 0, 0, 0) = vol + (dflux<1>(a, 1, i, j, k) + dfz);
  AT(4, 0, 0, 0) = vol + dfz;
  POINT_END
}

// z sweep.  args: R vol, R vfz, W pre, W post
OOC_KERNEL(k_adv_vol_z) {
  ARGS
  POINT_BEGIN_Z
  const double vol = AT(0, 0, 0, 0);
  AT(2, 0, 0, 0) = vol + dflux<2>(a, 1, i, j, k);
  AT(3, 0, 0, 0) = vol;
  POINT_END
}

// donor-cell mass / energy flux through the face between cells p - e_D and p.
// args: R vf, R rho1, R e1, W mf, W ef
template <int D>
OOC_KERNEL(k_adv_flux) {
  ARGS
  POINT_BEGIN_Z
  constexpr int ex = D == 0, ey = D == 1, ez = D == 2;
  const double f = AT(0, 0, 0, 0);
  double mf = 0.0, ef = 0.0;
  if (f > 0.0) {
    mf = f * AT(1, -ex, -ey, -ez);
    ef = mf * AT(2, -ex, -ey, -ez);
  } else if (f < 0.0) {
    mf = f * AT(1, 0, 0, 0);
    ef = mf * AT(2, 0, 0, 0);
  }
  AT(3, 0, 0, 0) = mf;
  AT(4, 0, 0, 0) = ef;
  POINT_END
}

// args: RW rho1, RW e1, R pre, R post, R mf, R ef
template <int D>
OOC_KERNEL(k_adv_cell) {
  ARGS
  POINT_BEGIN_Z
  constexpr int ex = D == 0, ey = D == 1, ez = D == 2;
  const double pm = AT(0, 0, 0, 0) * AT(2, 0, 0, 0);
  const double post = pm + (AT(4, 0, 0, 0) - AT(4, ex, ey, ez));
  const double pe = (AT(1, 0, 0, 0) * pm + (AT(5, 0, 0, 0) - AT(5, ex, ey, ez))) / post;
  AT(0, 0, 0, 0) = post / AT(3, 0, 0, 0);
  AT(1, 0, 0, 0) = pe;
  POINT_END
}

// Dual-face mass flux of sweep D: an eighth of the 8 face mass fluxes on the
// faces p and p + e_D, over the 4 cells around the node in the other two axes
// (B the first of them, C the second).  args: R mf, W nf
template <int D>
OOC_KERNEL(k_nflux) {
  ARGS
  POINT_BEGIN_Z
  constexpr int B = D == 0 ? 1 : 0, C = D == 2 ? 1 : 2;
  double t[2];
#pragma unroll
  for (int e = 0; e < 2; e++) {
    double q[2][2];
#pragma unroll
    for (int y = 0; y < 2; y++)
#pragma unroll
      for (int x = 0; x < 2; x++) {
        int o[3] = {0, 0, 0};
        o[D] = e;
        o[B] = -(1 - x);
        o[C] = -(1 - y);
        q[y][x] = AT(0, o[0], o[1], o[2]);
      }
    t[e] = (q[0][0] + q[0][1]) + (q[1][0] + q[1][1]);
  }
  AT(1, 0, 0, 0) = 0.125 * (t[0] + t[1]);
  POINT_END
}

// node masses after the sweep (from the swept cells) and before it.
// args: R rho1, R post, R nf, W nmpost, W nmpre.  Walking z, the summed
// masses of the 4 cells above a node are those below the next node.
template <int D>
__global__ void __launch_bounds__(256) k_nmass(const KArgs *__restrict__ ap) {
  ARGS
  int k;
  ZWALK_BEGIN
  constexpr int ex = D == 0, ey = D == 1, ez = D == 2;
  // the 4 cells around the node at cell plane k + dk - 1
#define CM(x, y, dk) (AT(0, (x) - 1, (y) - 1, (dk) - 1) * AT(1, (x) - 1, (y) - 1, (dk) - 1))
#define GROUP(dk) ((CM(0, 0, dk) + CM(1, 0, dk)) + (CM(0, 1, dk) + CM(1, 1, dk)))
  k = k0;
  double g0 = GROUP(0);
  for (; k < k1; k++) {
    const double g1 = GROUP(1);
    const double post = 0.125 * (g0 + g1);
    AT(3, 0, 0, 0) = post;
    AT(4, 0, 0, 0) = post + (AT(2, 0, 0, 0) - AT(2, -ex, -ey, -ez));
    g0 = g1;
  }
#undef GROUP
#undef CM
}

// donor-cell momentum flux through the dual face between nodes p and p + e_D.
// args: R nf, R vel, W mf
template <int D>
OOC_KERNEL(k_mflux) {
  ARGS
  POINT_BEGIN_Z
  constexpr int ex = D == 0, ey = D == 1, ez = D == 2;
  const double f = AT(0, 0, 0, 0);
  double mf = 0.0;
  if (f > 0.0) mf = f * AT(1, 0, 0, 0);
  else if (f < 0.0) mf = f * AT(1, ex, ey, ez);
  AT(2, 0, 0, 0) = mf;
  POINT_END
}

// args: RW vel, R nmpre, R nmpost, R mf
template <int D>
OOC_KERNEL(k_vel) {
  ARGS
  POINT_BEGIN_Z
  constexpr int ex = D == 0, ey = D == 1, ez = D == 2;
  AT(0, 0, 0, 0) = (AT(0, 0, 0, 0) * AT(1, 0, 0, 0) + (AT(3, -ex, -ey, -ez) - AT(3, 0, 0, 0))) / AT(2, 0, 0, 0);
  POINT_END
}

// largest |value| of node field n over the 4 nodes of the cell's face at z + dk
__device__ __forceinline__ double absmax4(const KArgs &a, int n, int i, int j, int k, int dk) {
  return fmax(fmax(fabs(AT(n, 0, 0, dk)), fabs(AT(n, 1, 0, dk))), fmax(fabs(AT(n, 0, 1, dk)), fabs(AT(n, 1, 1, dk))));
}

// stable step of a cell, min-reduced.  args: R e0, R u0, R v0, R w0; CONST dx,
// dy, dz; RED(MIN).  Walking z, the velocity jumps and the largest node speeds
// split into the cell's lower and upper node planes; the upper ones are the
// next cell's lower ones.  Every thread reaches the block reduction.
__global__ void __launch_bounds__(256) k_dt(const KArgs *__restrict__ ap) {
  ARGS
  double t = INFINITY;  // smallest bound over this thread's points
  const int n_ = (int)(gridDim.x * gridDim.y * gridDim.z);
  const int l_ = xcd_block((int)(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)), n_);
  const int bx_ = l_ % (int)gridDim.x, by_ = (l_ / (int)gridDim.x) % (int)gridDim.y;
  const int i = x_origin(a.lo[0]) + bx_ * 64 + (int)threadIdx.x;
  const int j = a.lo[1] + by_ * 4 + (int)threadIdx.y;
  const int k0 = a.lo[2] + (l_ / (int)(gridDim.x * gridDim.y)) * kPlanesPerThread;
  const int k1 = k0 + kPlanesPerThread < a.hi[2] ? k0 + kPlanesPerThread : a.hi[2];
  if (i >= a.lo[0] && i < a.hi[0] && j < a.hi[1] && k0 < k1) {
    int k = k0;
    JumpCarry lo = jump_plane(a, 1, 2, 3, i, j, k, 0);
    double mu = absmax4(a, 1, i, j, k, 0), mv = absmax4(a, 2, i, j, k, 0), mw = absmax4(a, 3, i, j, k, 0);
    for (; k < k1; k++) {
      const JumpCarry hi = jump_plane(a, 1, 2, 3, i, j, k, 1);
      const double hu = absmax4(a, 1, i, j, k, 1), hv = absmax4(a, 2, i, j, k, 1), hw = absmax4(a, 3, i, j, k, 1);
      const double c2 = (kGamma * kGm1) * AT(0, 0, 0, 0);
      const double d = jump_sum(lo, hi);
      double qr = 0.0;
      if (d < 0.0) qr = (kCq2 * d) * d - (kCq1 * sqrt(c2)) * d;
      const double ce = sqrt(c2 + 2.0 * qr);
      double tc = INFINITY;
      tc = fmin(tc, a.c[0] / (ce + fmax(mu, hu)));
      tc = fmin(tc, a.c[1] / (ce + fmax(mv, hv)));
      tc = fmin(tc, a.c[2] / (ce + fmax(mw, hw)));
      t = fmin(t, kCfl * tc);
      lo = hi;
      mu = hu;
      mv = hv;
      mw = hw;
    }
  }
  block_min_to(t, a.red[0]);
}

#define L(name, kern) \
  void name(const KArgs &a, const KArgs *d, int nd, void *s) { launch_point_z(kern, a, d, nd, s); }
L(l_visc, k_visc)
L(l_pdv_pred, k_pdv<false>)
L(l_pdv_corr, k_pdv<true>)
L(l_accel, k_accel)
L(l_flux_x, k_flux<0>)
L(l_flux_y, k_flux<1>)
L(l_flux_z, k_flux<2>)
L(l_adv_vol_x, k_adv_vol_x)
L(l_adv_vol_y, k_adv_vol_y)
L(l_adv_vol_z, k_adv_vol_z)
L(l_adv_flux_x, k_adv_flux<0>)
L(l_adv_flux_y, k_adv_flux<1>)
L(l_adv_flux_z, k_adv_flux<2>)
L(l_adv_cell_x, k_adv_cell<0>)
L(l_adv_cell_y, k_adv_cell<1>)
L(l_adv_cell_z, k_adv_cell<2>)
L(l_nflux_x, k_nflux<0>)
L(l_nflux_y, k_nflux<1>)
L(l_nflux_z, k_nflux<2>)
L(l_nmass_x, k_nmass<0>)
L(l_nmass_y, k_nmass<1>)
L(l_nmass_z, k_nmass<2>)
L(l_mflux_x, k_mflux<0>)
L(l_mflux_y, k_mflux<1>)
L(l_mflux_z, k_mflux<2>)
L(l_vel_x, k_vel<0>)
L(l_vel_y, k_vel<1>)
L(l_vel_z, k_vel<2>)
L(l_dt, k_dt)
#undef L

}  // namespace

void register_hydro3d_kernels(KernelInfo *t) {
  //                                   name            dat  dat const dev red
  t[OOC_K_H3D_VISC] = {"h3d_visc", 6, 6, 0, 0, 0, kPointGrid, l_visc};
  t[OOC_K_H3D_PDV_PRED] = {"h3d_pdv_pred", 13, 13, 0, 1, 0, kPointGrid, l_pdv_pred};
  t[OOC_K_H3D_PDV_CORR] = {"h3d_pdv_corr", 16, 16, 0, 1, 0, kPointGrid, l_pdv_corr};
  t[OOC_K_H3D_ACCEL] = {"h3d_accel", 13, 13, 3, 1, 0, kPointGrid, l_accel};
  t[OOC_K_H3D_FLUX_X] = {"h3d_flux_x", 4, 4, 0, 1, 0, kPointGrid, l_flux_x};
  t[OOC_K_H3D_FLUX_Y] = {"h3d_flux_y", 4, 4, 0, 1, 0, kPointGrid, l_flux_y};
  t[OOC_K_H3D_FLUX_Z] = {"h3d_flux_z", 4, 4, 0, 1, 0, kPointGrid, l_flux_z};
  t[OOC_K_H3D_ADV_VOL_X] = {"h3d_adv_vol_x", 6, 6, 0, 0, 0, kPointGrid, l_adv_vol_x};
  t[OOC_K_H3D_ADV_VOL_Y] = {"h3d_adv_vol_y", 5, 5, 0, 0, 0, kPointGrid, l_adv_vol_y};
  t[OOC_K_H3D_ADV_VOL_Z] = {"h3d_adv_vol_z", 4, 4, 0, 0, 0, kPointGrid, l_adv_vol_z};
  t[OOC_K_H3D_ADV_FLUX_X] = {"h3d_adv_flux_x", 5, 5, 0, 0, 0, kPointGrid, l_adv_flux_x};
  t[OOC_K_H3D_ADV_FLUX_Y] = {"h3d_adv_flux_y", 5, 5, 0, 0, 0, kPointGrid, l_adv_flux_y};
  t[OOC_K_H3D_ADV_FLUX_Z] = {"h3d_adv_flux_z", 5, 5, 0, 0, 0, kPointGrid, l_adv_flux_z};
  t[OOC_K_H3D_ADV_CELL_X] = {"h3d_adv_cell_x", 6, 6, 0, 0, 0, kPointGrid, l_adv_cell_x};
  t[OOC_K_H3D_ADV_CELL_Y] = {"h3d_adv_cell_y", 6, 6, 0, 0, 0, kPointGrid, l_adv_cell_y};
  t[OOC_K_H3D_ADV_CELL_Z] = {"h3d_adv_cell_z", 6, 6, 0, 0, 0, kPointGrid, l_adv_cell_z};
  t[OOC_K_H3D_NFLUX_X] = {"h3d_nflux_x", 2, 2, 0, 0, 0, kPointGrid, l_nflux_x};
  t[OOC_K_H3D_NFLUX_Y] = {"h3d_nflux_y", 2, 2, 0, 0, 0, kPointGrid, l_nflux_y};
  t[OOC_K_H3D_NFLUX_Z] = {"h3d_nflux_z", 2, 2, 0, 0, 0, kPointGrid, l_nflux_z};
  t[OOC_K_H3D_NMASS_X] = {"h3d_nmass_x", 5, 5, 0, 0, 0, kPointGrid, l_nmass_x};
  t[OOC_K_H3D_NMASS_Y] = {"h3d_nmass_y", 5, 5, 0, 0, 0, kPointGrid, l_nmass_y};
  t[OOC_K_H3D_NMASS_Z] = {"h3d_nmass_z", 5, 5, 0, 0, 0, kPointGrid, l_nmass_z};
  t[OOC_K_H3D_MFLUX_X] = {"h3d_mflux_x", 3, 3, 0, 0, 0, kPointGrid, l_mflux_x};
  t[OOC_K_H3D_MFLUX_Y] = {"h3d_mflux_y", 3, 3, 0, 0, 0, kPointGrid, l_mflux_y};
  t[OOC_K_H3D_MFLUX_Z] = {"h3d_mflux_z", 3, 3, 0, 0, 0, kPointGrid, l_mflux_z};
  t[OOC_K_H3D_VEL_X] = {"h3d_vel_x", 4, 4, 0, 0, 0, kPointGrid, l_vel_x};
  t[OOC_K_H3D_VEL_Y] = {"h3d_vel_y", 4, 4, 0, 0, 0, kPointGrid, l_vel_y};
  t[OOC_K_H3D_VEL_Z] = {"h3d_vel_z", 4, 4, 0, 0, 0, kPointGrid, l_vel_z};
  t[OOC_K_H3D_DT] = {"h3d_dt", 4, 4, 3, 0, 1, kPointGrid, l_dt};
}

}  // namespace ooc
