// Device-side helpers shared by the kernel translation units: point indexing
// over a launch range, field access through rebased pointers, and block-level
// reductions (wavefront = 64 lanes on gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include "ooc_internal.h"

namespace ooc {

// Every loop kernel reads its argument block from device memory (a per-chain
// table built once by the runtime): the launch itself carries one pointer.
#define OOC_KERNEL(name) __global__ void __launch_bounds__(256) name(const KArgs *__restrict__ ap)
#define ARGS const KArgs &a = *ap;

// Point kernels run 64 x 4 threads: one wavefront per row segment of 64
// x-points, so every load of a field row is a coalesced 512-byte access.  Each
// thread row walks kRowsPerThread rows 4 apart, so a block covers 64 x 16
// points and the row above a wavefront's row is read by its neighbour wave on
// the same CU at about the same time (the j+1 stencil reads hit L1/L2).
// Workgroup ids are handed to the 8 XCDs round-robin; the block order is
// remapped so each XCD gets a contiguous run of blocks, keeping the lines
// that neighbouring blocks share in one L2.
constexpr int kRowsPerThread = 4;
constexpr int kBlockRows = 4 * kRowsPerThread;
constexpr int kXcds = 8;
// consecutive z-planes one thread of the z-walking point loop covers (8 and
// 16 were measured to read more from HBM on 640^3, not less)
constexpr int kPlanesPerThread = 4;

// x of a launch's first block column: the range start rounded down to a
// multiple of 16 points.  With x = 0 stored on a 128-byte boundary, every
// 64-point row segment a wavefront touches is then four whole 128-byte lines
// (threads left of the range start idle).
__host__ __device__ inline int x_origin(int lo) { return lo & ~15; }

// bijection of [0, n): workgroup id -> logical block, contiguous per XCD
__device__ __forceinline__ int xcd_block(int pid, int n) {
  const int q = n / kXcds, r = n % kXcds, x = pid % kXcds, s = pid / kXcds;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + s;
}

// Opens the per-point loop: i, j, k are the point's indices inside it.
#define POINT_BEGIN                                                                        \
  {                                                                                        \
    const int n_ = (int)(gridDim.x * gridDim.y * gridDim.z);                               \
    const int l_ = xcd_block((int)(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)), n_); \
    const int bx_ = l_ % (int)gridDim.x, by_ = (l_ / (int)gridDim.x) % (int)gridDim.y;      \
    const int i = x_origin(a.lo[0]) + bx_ * 64 + (int)threadIdx.x;                         \
    const int k = a.lo[2] + l_ / (int)(gridDim.x * gridDim.y);                              \
    const int j0_ = a.lo[1] + by_ * kBlockRows + (int)threadIdx.y;                           \
    if (i >= a.lo[0] && i < a.hi[0])                                                       \
      for (int r_ = 0; r_ < kRowsPerThread; r_++) {                                        \
        const int j = j0_ + 4 * r_;                                                        \
        if (j >= a.hi[1]) break;
#define POINT_END \
  }               \
  }

// The same point loop walking kPlanesPerThread consecutive z-planes instead of
// rows (for stencils that reach along z: a thread's z-neighbours were mostly
// loaded for its previous plane); launched with point_grid_z.
#define POINT_BEGIN_Z                                                                      \
  {                                                                                        \
    const int n_ = (int)(gridDim.x * gridDim.y * gridDim.z);                               \
    const int l_ = xcd_block((int)(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)), n_); \
    const int bx_ = l_ % (int)gridDim.x, by_ = (l_ / (int)gridDim.x) % (int)gridDim.y;      \
    const int i = x_origin(a.lo[0]) + bx_ * 64 + (int)threadIdx.x;                         \
    const int j = a.lo[1] + by_ * 4 + (int)threadIdx.y;                                    \
    const int k0_ = a.lo[2] + (l_ / (int)(gridDim.x * gridDim.y)) * kPlanesPerThread;       \
    if (i >= a.lo[0] && i < a.hi[0] && j < a.hi[1])                                        \
      for (int r_ = 0; r_ < kPlanesPerThread; r_++) {                                      \
        const int k = k0_ + r_;                                                            \
        if (k >= a.hi[2]) break;

// Field storage is device global memory, but its pointers come from the
// argument table in memory, so the compiler cannot tell and would emit flat
// accesses -- which share the LDS wait counter, making every wait for an LDS
// result also wait for all outstanding HBM loads.  Accesses go through gp().
typedef __attribute__((address_space(1))) double gdouble;
__device__ __forceinline__ gdouble *gp(double *p) { return (gdouble *)p; }

// element (i+di, j+dj, k+dk) of DAT argument n
#define AT(n, di, dj, dk) \
  gp(a.p[n])[(int64_t)(k + (dk)) * a.plane + (int64_t)(j + (dj)) * a.pitch + (i + (di))]

inline dim3 point_grid_z(const KArgs &a) {
  const int nx = a.hi[0] - x_origin(a.lo[0]), ny = a.hi[1] - a.lo[1], nz = a.hi[2] - a.lo[2];
  if (a.hi[0] <= a.lo[0] || ny <= 0 || nz <= 0) return dim3(0, 0, 0);
  return dim3((nx + 63) / 64, (ny + 3) / 4, (nz + kPlanesPerThread - 1) / kPlanesPerThread);
}

inline dim3 point_grid(const KArgs &a, int ndim) {
  const int nx = a.hi[0] - x_origin(a.lo[0]), ny = a.hi[1] - a.lo[1];
  const int nz = ndim == 3 ? a.hi[2] - a.lo[2] : 1;
  if (a.hi[0] <= a.lo[0] || ny <= 0 || nz <= 0) return dim3(0, 0, 0);
  return dim3((nx + 63) / 64, (ny + kBlockRows - 1) / kBlockRows, nz);
}

__device__ inline double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// min / max are exact in any order, so one compare-and-swap loop per block
// suffices for a tiling-independent result.
__device__ inline void atomic_min_f64(double *addr, double v) {
  if (v != v) return;
  unsigned long long *p = (unsigned long long *)addr;
  unsigned long long old = __atomic_load_n(p, __ATOMIC_RELAXED);
  while (!(__longlong_as_double(old) <= v)) {
    unsigned long long prev = atomicCAS(p, old, (unsigned long long)__double_as_longlong(v));
    if (prev == old) break;
    old = prev;
  }
}
__device__ inline void atomic_max_f64(double *addr, double v) {
  if (v != v) return;
  unsigned long long *p = (unsigned long long *)addr;
  unsigned long long old = __atomic_load_n(p, __ATOMIC_RELAXED);
  while (!(__longlong_as_double(old) >= v)) {
    unsigned long long prev = atomicCAS(p, old, (unsigned long long)__double_as_longlong(v));
    if (prev == old) break;
    old = prev;
  }
}

// 64 x 4 block: wave w = threadIdx.y
__device__ inline void block_min_to(double v, double *out) {
  __shared__ double sm[4];
  v = wave_min(v);
  if (threadIdx.x == 0) sm[threadIdx.y] = v;
  __syncthreads();
  if (threadIdx.x == 0 && threadIdx.y == 0)
    atomic_min_f64(out, fmin(fmin(sm[0], sm[1]), fmin(sm[2], sm[3])));
}
__device__ inline void block_max_to(double v, double *out) {
  __shared__ double sm[4];
  v = wave_max(v);
  if (threadIdx.x == 0) sm[threadIdx.y] = v;
  __syncthreads();
  if (threadIdx.x == 0 && threadIdx.y == 0)
    atomic_max_f64(out, fmax(fmax(sm[0], sm[1]), fmax(sm[2], sm[3])));
}

// 256-thread 1D block: fixed pairwise tree, deterministic
__device__ inline double block_sum_fixed(double v) {
  __shared__ double sm[256];
  sm[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] += sm[threadIdx.x + s];
    __syncthreads();
  }
  return sm[0];
}

void launch_point(void (*k)(const KArgs *), const KArgs &a, const KArgs *dev, int ndim, void *s);
void launch_point_z(void (*k)(const KArgs *), const KArgs &a, const KArgs *dev, int ndim, void *s);
void launch_rows(void (*k)(const KArgs *), const KArgs &a, const KArgs *dev, int ndim, void *s);

}  // namespace ooc
