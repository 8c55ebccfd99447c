// Generic kernels of the loop-chain library for gfx950: mirror / copy strips,
// fills, order-fixed sums, min/max reductions, the batched slot-to-slot edge
// copy, and float32 <-> float64 conversion of streamed rows.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels_device.h"
#include "ooc_internal.h"

namespace ooc {

KernelInfo *kernel_table() {
  static KernelInfo t[OOC_K_MAX_ID];
  return t;
}

// ---------------------------------------------------------------- generic
// dst_q(p) = sign_q * src_q(p + o_q) for each of the n pairs.
__device__ inline void mirror_point(const KArgs &a, int i, int j, int k) {
  const int n = a.ndat / 2;
  for (int q = 0; q < n; q++) {
    const int32_t *o = a.off[2 * q + 1];
    AT(2 * q, 0, 0, 0) = a.c[q] * AT(2 * q + 1, o[0], o[1], o[2]);
  }
}

// Strip loops are often a wall layer one or a few points wide in x: their
// points are numbered x-fastest and handed out 256 per block, so every lane
// has work whatever the shape of the box (a 64-wide row mapping would leave
// most lanes of a one-point-wide strip idle).
__device__ inline void mirror_flat(const KArgs &a, int64_t e) {
  const int64_t nx = a.hi[0] - a.lo[0], ny = a.hi[1] - a.lo[1];
  const int64_t t = e / nx;
  mirror_point(a, a.lo[0] + (int)(e - t * nx), a.lo[1] + (int)(t % ny), a.lo[2] + (int)(t / ny));
}

inline int64_t box_points(const KArgs &a, int ndim) {
  const int64_t nx = a.hi[0] - a.lo[0], ny = a.hi[1] - a.lo[1];
  const int64_t nz = ndim == 3 ? a.hi[2] - a.lo[2] : 1;
  return nx > 0 && ny > 0 && nz > 0 ? nx * ny * nz : 0;
}

__global__ void __launch_bounds__(256) k_mirror(const KArgs *__restrict__ ap, int64_t npts) {
  ARGS
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < npts) mirror_flat(a, e);
}

static void l_mirror(const KArgs &a, const KArgs *d, int nd, void *s) {
  const int64_t npts = box_points(a, nd);
  if (npts) hipLaunchKernelGGL(k_mirror, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, (hipStream_t)s, d, npts);
}

// Several independent mirror loops of one tile in a single launch: block b
// belongs to the loop whose block range holds it (prefix sums in blk0), and
// runs exactly the single-loop body there.
struct MirrorBatch {
  const KArgs *args[32];
  int64_t npts[32];
  int32_t blk0[33];
  int32_t n;
};

__global__ void __launch_bounds__(256) k_mirror_batch(MirrorBatch mb) {
  const int b = blockIdx.x;
  int s = 0;
  while (s + 1 < mb.n && b >= mb.blk0[s + 1]) s++;
  const int64_t e = (int64_t)(b - mb.blk0[s]) * 256 + threadIdx.x;
  if (e < mb.npts[s]) mirror_flat(*mb.args[s], e);
}

void launch_mirror_batch(const KArgs *const *host_args, const KArgs *const *dev_args, int n, int ndim,
                         void *stream) {
  for (int s0 = 0; s0 < n; s0 += 32) {
    MirrorBatch mb{};
    mb.n = n - s0 < 32 ? n - s0 : 32;
    int blocks = 0;
    for (int q = 0; q < mb.n; q++) {
      mb.args[q] = dev_args[s0 + q];
      mb.npts[q] = box_points(*host_args[s0 + q], ndim);
      mb.blk0[q] = blocks;
      blocks += (int)((mb.npts[q] + 255) / 256);
    }
    mb.blk0[mb.n] = blocks;
    if (blocks) hipLaunchKernelGGL(k_mirror_batch, dim3(blocks), dim3(256), 0, (hipStream_t)stream, mb);
  }
}

OOC_KERNEL(k_fill_pt) {
  ARGS
  POINT_BEGIN
  AT(0, 0, 0, 0) = a.c[0];
  POINT_END
}

// out = c0 * (sum over the stencil of in) / npts + c1, stencil summed in order
OOC_KERNEL(k_avg) {
  ARGS
  POINT_BEGIN
  double s = 0.0;
  for (int q = 0; q < a.nst; q++) s += AT(1, a.st[q][0], a.st[q][1], a.st[q][2]);
  AT(0, 0, 0, 0) = a.c[0] * (s / (double)a.nst) + a.c[1];
  POINT_END
}

OOC_KERNEL(k_inc_add) {
  ARGS
  POINT_BEGIN
  AT(0, 0, 0, 0) = AT(0, 0, 0, 0) + a.c[0] * AT(1, 0, 0, 0);
  POINT_END
}

OOC_KERNEL(k_minmax) {
  ARGS
  double v = INFINITY, w = -INFINITY;  // over this thread's points
  POINT_BEGIN
  v = fmin(v, AT(0, 0, 0, 0));
  w = fmax(w, AT(0, 0, 0, 0));
  POINT_END
  block_min_to(v, a.red[0]);
  block_max_to(w, a.red[1]);
}

// One block per row (y, z): the row's product sum in a fixed order, written to
// the row's partial slot.  Independent of tiling because a row is always
// summed by one block in the same order.
OOC_KERNEL(k_sum_prod) {
  ARGS
  const int j = a.lo[1] + blockIdx.y;
  const int k = a.lo[2] + blockIdx.z;
  double s = 0.0;
  for (int i = a.lo[0] + threadIdx.x; i < a.hi[0]; i += 256) {
    double v = AT(0, 0, 0, 0);
    if (a.ndat > 1) v *= AT(1, 0, 0, 0);
    if (a.ndat > 2) v *= AT(2, 0, 0, 0);
    s += v;
  }
  s = block_sum_fixed(s);
  if (threadIdx.x == 0) {
    const int64_t row = (int64_t)(k + a.halo) * a.red_rows + (j + a.halo);
    a.red[0][a.plane ? row : (j + a.halo)] = s;
  }
}

void launch_point(void (*k)(const KArgs *), const KArgs &a, const KArgs *dev, int ndim, void *s) {
  dim3 grid = point_grid(a, ndim);
  if (grid.x && grid.y && grid.z) hipLaunchKernelGGL(k, grid, dim3(64, 4, 1), 0, (hipStream_t)s, dev);
}

void launch_point_z(void (*k)(const KArgs *), const KArgs &a, const KArgs *dev, int ndim, void *s) {
  if (ndim != 3) return launch_point(k, a, dev, ndim, s);
  dim3 grid = point_grid_z(a);
  if (grid.x && grid.y && grid.z) hipLaunchKernelGGL(k, grid, dim3(64, 4, 1), 0, (hipStream_t)s, dev);
}

void launch_rows(void (*k)(const KArgs *), const KArgs &a, const KArgs *dev, int ndim, void *s) {
  dim3 grid(1, a.hi[1] - a.lo[1], ndim == 3 ? a.hi[2] - a.lo[2] : 1);
  if (grid.y && grid.z && a.hi[0] > a.lo[0]) hipLaunchKernelGGL(k, grid, dim3(256, 1, 1), 0, (hipStream_t)s, dev);
}

#define POINT_LAUNCHER(name, kern) \
  static void name(const KArgs &a, const KArgs *d, int nd, void *s) { launch_point(kern, a, d, nd, s); }
POINT_LAUNCHER(l_fill, k_fill_pt)
POINT_LAUNCHER(l_avg, k_avg)
POINT_LAUNCHER(l_inc_add, k_inc_add)
POINT_LAUNCHER(l_minmax, k_minmax)
static void l_sum_prod(const KArgs &a, const KArgs *d, int nd, void *s) { launch_rows(k_sum_prod, a, d, nd, s); }

void register_common_kernels(KernelInfo *t) {
  t[OOC_K_MIRROR] = {"mirror", 2, 12, -1, 0, 0, kPointGrid, l_mirror};
  t[OOC_K_FILL] = {"fill", 1, 1, 1, 0, 0, kPointGrid, l_fill};
  t[OOC_K_SUM_PROD] = {"sum_prod", 1, 3, 0, 0, 1, kRowReduce, l_sum_prod};
  t[OOC_K_AVG] = {"avg", 2, 2, 2, 0, 0, kPointGrid, l_avg};
  t[OOC_K_INC_ADD] = {"inc_add", 2, 2, 1, 0, 0, kPointGrid, l_inc_add};
  t[OOC_K_MINMAX] = {"minmax", 1, 1, 0, 0, 2, kPointGrid, l_minmax};
}

// --------------------------------------------------------- runtime helpers
// Batched copy of up to 32 contiguous segments (the slot-to-slot edge copy),
// each a multiple of 2 doubles and 16-byte aligned (rows are 256-byte multiples).
struct SegTable {
  const double *src[32];
  double *dst[32];
  int64_t n[32];
  int64_t blk0[33];
  int nseg;
};
constexpr int64_t kSegChunk = 4096;  // doubles per block

__global__ void __launch_bounds__(256) k_copy_segs(SegTable t) {
  const int64_t b = blockIdx.x;
  int s = 0;
  while (s + 1 < t.nseg && b >= t.blk0[s + 1]) s++;
  const int64_t base = (b - t.blk0[s]) * kSegChunk;
  const int64_t end = base + kSegChunk < t.n[s] ? base + kSegChunk : t.n[s];
  const double2 *src = (const double2 *)t.src[s];
  double2 *dst = (double2 *)t.dst[s];
  for (int64_t e = base / 2 + threadIdx.x; e < end / 2; e += 256) dst[e] = src[e];
}

void launch_copy_segments(const CopySeg *segs, int nseg, void *stream) {
  for (int s0 = 0; s0 < nseg; s0 += 32) {
    SegTable t{};
    t.nseg = nseg - s0 < 32 ? nseg - s0 : 32;
    int64_t blocks = 0;
    for (int q = 0; q < t.nseg; q++) {
      t.src[q] = segs[s0 + q].src;
      t.dst[q] = segs[s0 + q].dst;
      t.n[q] = segs[s0 + q].n;
      t.blk0[q] = blocks;
      blocks += (t.n[q] + kSegChunk - 1) / kSegChunk;
    }
    t.blk0[t.nseg] = blocks;
    if (blocks) hipLaunchKernelGGL(k_copy_segs, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, t);
  }
}

__global__ void __launch_bounds__(256) k_fill(double *d, int64_t n, double v) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) d[e] = v;
}

void launch_fill(double *dst, int64_t n, double value, void *stream) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, dst, n, value);
}

__global__ void k_set1(double *d, double v) {
  if (threadIdx.x == 0) d[0] = v;
}
__global__ void k_copy1(const double *s, double *d) {
  if (threadIdx.x == 0) d[0] = s[0];
}

void launch_red_init(double *acc, double value, void *stream) {
  hipLaunchKernelGGL(k_set1, dim3(1), dim3(64), 0, (hipStream_t)stream, acc, value);
}

void launch_red_commit(const double *acc, double *committed, void *stream) {
  hipLaunchKernelGGL(k_copy1, dim3(1), dim3(64), 0, (hipStream_t)stream, acc, committed);
}

// Fixed-order combination of the per-row partials: thread t sums rows
// t, t+256, ... in order, then a fixed tree.
__global__ void __launch_bounds__(256) k_sum_finalize(const double *p, int64_t n, double *out) {
  double s = 0.0;
  for (int64_t e = threadIdx.x; e < n; e += 256) s += p[e];
  s = block_sum_fixed(s);
  if (threadIdx.x == 0) out[0] = s;
}

void launch_sum_finalize(const double *partials, int64_t n, double *committed, void *stream) {
  hipLaunchKernelGGL(k_sum_finalize, dim3(1), dim3(256), 0, (hipStream_t)stream, partials, n, committed);
}

__global__ void __launch_bounds__(256) k_f32_to_f64(const float *s, double *d, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
    d[e] = (double)s[e];
}

__global__ void __launch_bounds__(256) k_f64_to_f32(const double *s, float *d, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
    d[e] = (float)s[e];  // round to nearest even
}

void launch_f32_to_f64(const float *src, double *dst, int64_t n, void *stream) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_f32_to_f64, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, src, dst, n);
}

void launch_f64_to_f32(const double *src, float *dst, int64_t n, void *stream) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_f64_to_f32, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, src, dst, n);
}

}  // namespace ooc

namespace ooc {

// Host-link transfers done by a kernel that reads or writes the pinned host
// arrays directly through their device mapping: one launch per tile for all
// of its runs, with the float32 <-> float64 conversion done in flight.
struct XferTable {
  const void *src[32];
  void *dst[32];
  int64_t n[32];  // elements (mode 0: 16-byte units)
  int32_t mode[32];
  int64_t blk0[33];
  int32_t nseg;
};
constexpr int64_t kXferChunk = 4096;  // elements per block

// four float64 values read as two 16-byte loads
struct Double4 {
  double2 lo, hi;
};

// A small grid strides over the chunks.  The copy is bound by the host link.
// Its stores to host memory hold up other kernels' memory requests while they
// sit in the queues towards the link (measured: a strip loop beside a
// 64-block device-to-host copy took 0.6 ms instead of 8 us), so the writing
// direction runs only a few wavefronts, each with several loads in flight
// before its stores; the reading direction needs more wavefronts to cover
// the link's read latency.  When the uploads bound the pipeline, the writing
// direction narrows further (its stores in flight also slow the concurrent
// DMA uploads).
constexpr int kXferWriteBlocks = 8;
constexpr int kXferWriteBlocksNarrow = 2;
constexpr int kXferReadBlocks = 64;
constexpr int kXferUnroll = 4;

template <class S, class D, class F>
__device__ __forceinline__ void xfer_range(const S *src, D *dst, int64_t e0, int64_t end, F conv) {
  for (int64_t e = e0 + threadIdx.x; e < end; e += kXferUnroll * 256) {
    S v[kXferUnroll];
#pragma unroll
    for (int u = 0; u < kXferUnroll; u++)
      if (e + u * 256 < end) v[u] = src[e + u * 256];
#pragma unroll
    for (int u = 0; u < kXferUnroll; u++)
      if (e + u * 256 < end) dst[e + u * 256] = conv(v[u]);
  }
}

__device__ void xfer_chunk(const XferTable &t, int64_t b) {
  int s = 0;
  while (s + 1 < t.nseg && b >= t.blk0[s + 1]) s++;
  const int64_t base = (b - t.blk0[s]) * kXferChunk;
  const int64_t end = base + kXferChunk < t.n[s] ? base + kXferChunk : t.n[s];
  if (t.mode[s] == 0) {
    xfer_range((const double2 *)t.src[s], (double2 *)t.dst[s], base, end, [](double2 v) { return v; });
  } else if (t.mode[s] == 1) {  // float32 -> float64, 2 elements per lane step
    xfer_range((const float2 *)t.src[s], (double2 *)t.dst[s], base / 2, end / 2,
               [](float2 v) { return make_double2((double)v.x, (double)v.y); });
  } else if (t.mode[s] == 2) {  // float64 -> float32 (round to nearest even), 8-byte stores
    xfer_range((const double2 *)t.src[s], (float2 *)t.dst[s], base / 2, end / 2,
               [](double2 v) { return make_float2((float)v.x, (float)v.y); });
  } else {  // the same, 4 elements per lane step: 16-byte stores like the float64 copy's
    xfer_range((const Double4 *)t.src[s], (float4 *)t.dst[s], base / 4, end / 4, [](Double4 v) {
      return make_float4((float)v.lo.x, (float)v.lo.y, (float)v.hi.x, (float)v.hi.y);
    });
  }
}

__global__ void __launch_bounds__(256) k_xfer(XferTable t) {
  for (int64_t b = blockIdx.x; b < t.blk0[t.nseg]; b += gridDim.x) xfer_chunk(t, b);
}

void launch_xfer_segments(const XferSeg *segs, int nseg, bool to_host, bool narrow, void *stream) {
  for (int s0 = 0; s0 < nseg; s0 += 32) {
    XferTable t{};
    t.nseg = nseg - s0 < 32 ? nseg - s0 : 32;
    int64_t blocks = 0;
    for (int q = 0; q < t.nseg; q++) {
      const XferSeg &g = segs[s0 + q];
      t.src[q] = g.src;
      t.dst[q] = g.dst;
      t.n[q] = g.n;
      t.mode[q] = g.mode;
      t.blk0[q] = blocks;
      blocks += (g.n + kXferChunk - 1) / kXferChunk;
    }
    t.blk0[t.nseg] = blocks;
    const int64_t cap = to_host ? (narrow ? kXferWriteBlocksNarrow : kXferWriteBlocks) : kXferReadBlocks;
    const int64_t grid = blocks < cap ? blocks : cap;
    if (blocks) hipLaunchKernelGGL(k_xfer, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream, t);
  }
}

}  // namespace ooc
