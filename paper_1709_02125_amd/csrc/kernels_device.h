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

// Point kernels run 64 x 4 blocks: one wavefront per row segment of 64 x-points,
// so every load of a field row is a coalesced 512-byte access.
#define POINT_INDEX_OR_RETURN                                     \
  const int i = a.lo[0] + (int)(blockIdx.x * 64 + threadIdx.x);   \
  const int j = a.lo[1] + (int)(blockIdx.y * 4 + threadIdx.y);    \
  const int k = a.lo[2] + (int)blockIdx.z;                        \
  if (i >= a.hi[0] || j >= a.hi[1]) return;

#define POINT_INDEX_ACTIVE                                        \
  const int i = a.lo[0] + (int)(blockIdx.x * 64 + threadIdx.x);   \
  const int j = a.lo[1] + (int)(blockIdx.y * 4 + threadIdx.y);    \
  const int k = a.lo[2] + (int)blockIdx.z;                        \
  const bool active = i < a.hi[0] && j < a.hi[1];

// element (i+di, j+dj, k+dk) of DAT argument n
#define AT(n, di, dj, dk) \
  a.p[n][(int64_t)(k + (dk)) * a.plane + (int64_t)(j + (dj)) * a.pitch + (i + (di))]

inline dim3 point_grid(const KArgs &a, int ndim) {
  const int nx = a.hi[0] - a.lo[0], ny = a.hi[1] - a.lo[1];
  const int nz = ndim == 3 ? a.hi[2] - a.lo[2] : 1;
  if (nx <= 0 || ny <= 0 || nz <= 0) return dim3(0, 0, 0);
  return dim3((nx + 63) / 64, (ny + 3) / 4, nz);
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
void launch_rows(void (*k)(const KArgs *), const KArgs &a, const KArgs *dev, int ndim, void *s);

}  // namespace ooc
