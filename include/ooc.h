/*
 * ooc.h -- C ABI of the out-of-core tiled stencil loop-chain library (gfx950).
 *
 * The interface follows the structured-mesh abstraction of the paper's
 * Section 3: a block (the grid, ooc_create), datasets on it (ooc_decl_field),
 * stencils (per-argument offset lists) and parallel loops over an iteration
 * range with read / write / read-write access (ooc_par_loop).  Data is only
 * reachable through opaque handles, and only calls that return data to the
 * caller (ooc_reduce, ooc_fetch_field, ooc_execute) end the lazily queued
 * loop chain (Section 3).  Execution of a chain follows the explicitly managed
 * tiling of Section 4 (Algorithm 1, with the optimisations of Section 4.1).
 *
 * Conventions shared by every call:
 *  - Every function returns int: OOC_OK (0) or a negative OOC_E_* code.  No
 *    C++ exception crosses this boundary.  The message of the last failure is
 *    available from ooc_last_error().
 *  - After an OOC_E_DEVICE failure the context is failed: every later call
 *    except ooc_destroy / ooc_last_error returns OOC_E_FAILED.
 *  - Pointers passed in (names, offsets, initial data) are copied before the
 *    call returns; the caller keeps ownership.
 *  - Grid indices are logical: an axis of n interior cells with halo depth h
 *    has valid indices [-h, n + h + delta) where delta (0 or 1) is the field's
 *    size increment on that axis (nodes and faces have one more point).
 *  - The tiled axis is the last grid axis (y in 2D, z in 3D).
 *  - Host field data is row-major with x fastest, laid out over the field's
 *    full logical extent (halo included), as float64.
 */
#ifndef OOC_H
#define OOC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ooc_ctx ooc_ctx;
typedef int32_t ooc_field;
typedef int32_t ooc_red;

/* return codes */
enum {
  OOC_OK = 0,
  OOC_E_ARG = -1,     /* invalid argument: bad handle, range, stencil or kernel signature */
  OOC_E_BUDGET = -2,  /* no tile schedule fits the device byte budget */
  OOC_E_DEVICE = -3,  /* a HIP runtime call failed; the context is now failed */
  OOC_E_STATE = -4,   /* call not valid in the current state (e.g. before bind) */
  OOC_E_FAILED = -5,  /* the context failed earlier */
  OOC_E_STALE = -6,   /* fetch of a temporary whose host copy was skipped (Cyclic) */
  OOC_E_NOMEM = -7    /* host allocation (pinned memory) failed */
};

/* dataset access modes (Section 3: read / write / both; INC is a point-wise
 * read-modify-write, analysed as read-write) */
enum { OOC_READ = 1, OOC_WRITE = 2, OOC_RW = 3, OOC_INC = 4 };

/* reduction operators */
enum { OOC_RED_MIN = 1, OOC_RED_MAX = 2, OOC_RED_SUM = 3 };

/* kinds of loop argument */
enum {
  OOC_ARG_DAT = 0,       /* a field accessed through a stencil */
  OOC_ARG_RED = 1,       /* a reduction the loop contributes to */
  OOC_ARG_CONST = 2,     /* a double passed by value */
  OOC_ARG_DEVSCALAR = 3  /* the last committed value of a reduction, read on the device */
};

/* context flags */
enum {
  OOC_FLAG_CYCLIC = 1,        /* Section 4.1 opt (2): do not download write-first datasets */
  OOC_FLAG_PREFETCH = 2,      /* Section 4.1 opt (3): start the next chain's first tile early */
  OOC_FLAG_FP32_STREAM = 4,   /* store streamed fields on the host as float32 (transfers halved) */
  OOC_FLAG_INCORE = 8,        /* keep every field resident on the device (no streaming) */
  OOC_FLAG_GRAPH = 16,        /* replay each chain's tile pipeline from a captured hipGraph.
                                * Switched off in this version: ooc_create and ooc_set_flags
                                * reject it with OOC_E_ARG. */
  OOC_FLAG_FUSE = 32,         /* launch independent strip (mirror) loops of a tile together */
  OOC_FLAG_DEBUG_POISON = 64, /* fill every slot with NaN before use (finds missing uploads) */
  OOC_FLAG_DEBUG_SYNC = 128,  /* serialise the three streams (separates races from plan bugs) */
  OOC_FLAG_PLAN_ONLY = 256,   /* no host or device storage: for ooc_debug_plan only (schedule search) */
  OOC_FLAG_KERNEL_COPY = 512, /* uploads too by a copy kernel on the pinned arrays' device mapping
                                 (one launch per tile; FP32 converted in flight) instead of runtime
                                 memcpy calls.  Downloads go by copy kernel when the host arrays
                                 are device-mapped (pinned by ooc_bind_device), unless
                                 OOC_FLAG_MEMCPY_DOWNLOAD is set */
  OOC_FLAG_RING = 1024,       /* ring slabs instead of slots: each streamed field lives in one ring
                                 of device memory mapped twice at consecutive virtual addresses
                                 (HIP virtual memory API), so the rows two tiles share stay in
                                 place -- no edge copy -- and a ring only holds the rows of the S
                                 tiles in flight.  The rings are allocated by the library within
                                 the budget (the arena given to ooc_bind_device then only needs
                                 the reductions and resident fields, or may be NULL with 0 bytes:
                                 the library allocates that too).  A chain's first tiles wait
                                 only for the downloads of the previous chain's tiles whose ring
                                 positions they take.  Fixed at creation; OOC_E_ARG at the first
                                 flush if the device lacks the API. */
  OOC_FLAG_MEMCPY_DOWNLOAD = 2048 /* downloads by runtime memcpy calls (FP32 rounded into a staging
                                 area first) instead of the copy kernel, also when the host arrays
                                 are device-mapped: for chains bound by their kernels, which the
                                 copy kernel's host stores slow down more than the runtime's
                                 copies do (ns3d 512^3 on rings: 59 against 73 ms per step); the
                                 copy kernel stays faster for chains bound by the link (hydro2d
                                 15360^2, hydro3d 640^3).  Ignored with OOC_FLAG_KERNEL_COPY. */
};

/* per-field flags for ooc_decl_field */
enum {
  OOC_FIELD_RESIDENT = 1  /* keep this field on the device for the context's lifetime */
};

typedef struct {
  int32_t kind;            /* OOC_ARG_* */
  int32_t handle;          /* field (DAT) or reduction (RED, DEVSCALAR) handle */
  int32_t access;          /* DAT only: OOC_READ / OOC_WRITE / OOC_RW / OOC_INC */
  int32_t npts;            /* DAT only: number of stencil points (1 .. 256) */
  const int32_t *offsets;  /* DAT only: npts * ndim offsets, point-major */
  double value;            /* CONST only */
} ooc_arg;

typedef struct {
  uint64_t chains, tiles, launches;
  uint64_t bytes_h2d, bytes_d2h, bytes_edge;   /* cumulative transfer bytes */
  uint64_t bytes_hbm_alg;                      /* cumulative algorithmic loop bytes (Section 5.1 rule) */
  uint64_t last_bytes_h2d, last_bytes_d2h;     /* of the last flush */
  int64_t tile_rows;                           /* tile height of the last planned chain */
  int32_t ntiles_last;                         /* tiles of the last planned chain */
  int32_t slots;                               /* buffer depth in use */
  uint64_t slot_bytes;                         /* bytes of one slot of the last plan */
  double last_flush_ms;                        /* device time of the last flush */
  double last_kernel_ms;                       /* summed kernel time of the last flush (if timed) */
  double last_issue_ms;                        /* host time spent issuing the last flush's chains */
  double max_call_ms;                          /* longest single runtime call while issuing chains,
                                                  since creation or the last ooc_set_timing call */
  uint64_t host_pinned_bytes, host_pageable_bytes; /* host field storage pinned / left pageable
                                                     (pinning failed): transfers of pageable rows
                                                     are synchronous with the host */
  int32_t max_call_kind;                       /* that call: 0 upload copy, 1 download, 2 kernel
                                                  launch, 3 stream wait, 4 event record, 5 other */
  int32_t max_call_chain;                      /* chains issued before it (0 = in the first chain) */
} ooc_stats;

/* Create a context for a grid of ndim (2 or 3) axes with dims[a] interior cells
 * per axis and halo depth `halo` (Section 3: a block).  device_budget_bytes
 * caps the device memory the context may use for data: tile slots, resident
 * fields and reduction buffers (the kernels' launch-argument table, a few MB,
 * is allocated apart from it).  Nothing is allocated on the device here. */
int ooc_create(ooc_ctx **out, int ndim, const int64_t dims[3], int halo,
               size_t device_budget_bytes, uint32_t flags);

/* Hand the context its device arena (at least the budget, 256-byte aligned)
 * and its three streams: host-to-device, compute, device-to-host (Section 4:
 * streams 1, 0 and 2 of Algorithm 1).  Streams are hipStream_t values; the
 * arena and the streams stay owned by the caller and must outlive the
 * context.  If never called, the first flush allocates its own.  With
 * OOC_FLAG_RING the arena may be NULL with arena_bytes 0 (see the flag). */
int ooc_bind_device(ooc_ctx *ctx, void *arena, size_t arena_bytes,
                    void *stream_h2d, void *stream_compute, void *stream_d2h);

/* Declare a float64 field (Section 3: a dataset).  size_delta[a] in {0,1}
 * adds one point on axis a (node / face centring).  init_host, if not NULL,
 * holds the full logical extent (halo included, x fastest); NULL means zeros.
 * The library keeps the field in pinned host memory it owns. */
int ooc_decl_field(ooc_ctx *ctx, const char *name, const int32_t size_delta[3],
                   const double *init_host, uint32_t field_flags, ooc_field *out);

/* Declare a reduction (MIN / MAX / SUM).  A SUM is order-fixed: per-row
 * partials in x order, combined in a fixed order, so its value does not
 * depend on the tiling. */
int ooc_decl_reduction(ooc_ctx *ctx, int op, ooc_red *out);

/* Set the committed value of a reduction (what DEVSCALAR arguments read). */
int ooc_set_reduction(ooc_ctx *ctx, ooc_red red, double value);

/* Queue a parallel loop (Section 3; Figure 1): kernel_id from ooc_kernels.h,
 * range[2a], range[2a+1] the half-open iteration range on axis a.  Nothing
 * executes (lazy execution, Section 3).  Checked at the call:
 *  - the kernel's signature (argument kinds and counts);
 *  - every DAT access stays inside its field's extent;
 *  - WRITE / RW / INC arguments access only offset 0 (points are order-free);
 *  - a loop that writes a field reads it at non-zero offsets only where the
 *    shifted range is disjoint from the written range. */
int ooc_par_loop(ooc_ctx *ctx, int kernel_id, const int64_t range[6], int nargs,
                 const ooc_arg *args);

/* Drop everything queued without executing it (after ooc_debug_plan, for
 * schedule search). */
int ooc_discard_queue(ooc_ctx *ctx);

/* Mark a step boundary in the queue; with ooc_set_schedule(chain_steps = k)
 * a chain ends after every k marks. */
int ooc_mark_step(ooc_ctx *ctx);

/* Flush: analyse and execute everything queued, then wait for the device. */
int ooc_execute(ooc_ctx *ctx);

/* Analyse and issue the queued chains without waiting for the device: they
 * run asynchronously on the context's streams while the caller queues more
 * loops.  With a chain length set (ooc_set_schedule), a trailing chain that
 * has not yet reached its step marks stays queued.  The next ooc_execute or
 * data-returning call issues the rest and waits. */
int ooc_submit(ooc_ctx *ctx);

/* Flush, then return the committed value of a reduction (Section 3: getting
 * the result of a reduction ends the chain). */
int ooc_reduce(ooc_ctx *ctx, ooc_red red, double *out);

/* Flush, then copy the field's full logical extent (float64, x fastest) into
 * dst (bytes must equal the extent size).  OOC_E_STALE if the field is a
 * temporary whose download was skipped under OOC_FLAG_CYCLIC. */
int ooc_fetch_field(ooc_ctx *ctx, ooc_field f, double *dst, size_t bytes);

/* Replace a field's host data (full logical extent, float64). */
int ooc_set_field(ooc_ctx *ctx, ooc_field f, const double *src, size_t bytes);

/* Set / clear context flags, e.g. OOC_FLAG_CYCLIC once the cyclic part of an
 * application begins (Section 4.1). */
int ooc_set_flags(ooc_ctx *ctx, uint32_t set, uint32_t clear);

/* Schedule: tile height in rows of the tiled axis (0 = largest that fits the
 * budget; on ring slabs the tallest, down to 3/5 of it, whose chain
 * boundaries stay clear), chain length in step marks (0 = whole flush), slot
 * count (0 = 3, the paper's three slots; 2..8 allowed).  When the tile height
 * does not divide the tiled range, the first tile takes the remainder. */
int ooc_set_schedule(ooc_ctx *ctx, int64_t tile_rows, int chain_steps, int slots);

int ooc_get_stats(ooc_ctx *ctx, ooc_stats *out);

/* Storage layout shared by every field of the context (host and device
 * copies alike): element (i, j, k) of a field (logical indices, the field's
 * lower bound being -halo on every axis) lies at
 * (k + halo) * plane + (j + halo) * pitch + (i + x_origin) elements from the
 * start of its storage; in 2D the k term is absent and plane is 0.  x_origin
 * (16) puts x = 0 on a 128-byte boundary of every row.  Returns OOC_E_ARG on a
 * null pointer. */
int ooc_get_layout(ooc_ctx *ctx, int64_t *pitch, int64_t *plane, int64_t *x_origin);

/* Enable per-launch timing with hipEvents (adds a little overhead); read the
 * summed kernel time of the last flush from ooc_stats.last_kernel_ms.
 * on = 1 times every loop launch; on = 2 + k times only launches of kernel
 * id k (one kernel's figures with few events in flight); 0 turns it off.
 * Every call clears the accumulated per-kernel figures and the longest-call
 * record of ooc_stats (max_call_ms, max_call_kind, max_call_chain). */
int ooc_set_timing(ooc_ctx *ctx, int on);

/* Per-tile stage timing (hipEvents on the three streams), from the next
 * flush on while on != 0: for every tile, the begin and end of its upload
 * stage (upload stream, after the wait for its slot), of its loops and of its
 * edge copy (compute stream, after the wait for its uploads) and of its
 * download stage (download stream, after the wait for its compute).  Times
 * are microseconds from the first tile's upload begin of the collected
 * period: the tiles issued since the previous waiting flush. */
typedef struct {
  int64_t tile;                       /* global tile index */
  float h2d_begin_us, h2d_end_us;     /* upload stage */
  float comp_begin_us, comp_end_us;   /* loops of the tile */
  float edge_end_us;                  /* edge copy to the next slot, from comp_end_us */
  float d2h_begin_us, d2h_end_us;     /* download stage */
} ooc_tile_time;
int ooc_set_tile_timing(ooc_ctx *ctx, int on);

/* The records of the last collected period (see ooc_set_tile_timing): *count
 * receives their number; min(capacity, count) records are copied to out (out
 * may be NULL to query the count).  Returns OOC_E_ARG if count is NULL. */
int ooc_tile_times(ooc_ctx *ctx, ooc_tile_time *out, int capacity, int *count);

/* Accumulated timing of one kernel id over the flushes since timing was
 * enabled: summed launch time (ms, hipEvents on the compute stream), launch
 * count and algorithmic bytes (Section 5.1 rule: 1x per read or written
 * dataset point, 2x for read-write). */
int ooc_kernel_stats(ooc_ctx *ctx, int kernel_id, double *ms, uint64_t *launches, uint64_t *bytes);

/* Message of the last failing call on ctx (owned by the context, valid until
 * its next call; empty if nothing failed yet); "null context" for NULL. */
const char *ooc_last_error(ooc_ctx *ctx);

/* Failure injection for tests of the error path: from now on, the n-th
 * runtime call the context checks (copies, launches, event and stream calls
 * while it issues chains) is reported as failed right after it was issued
 * successfully; n = 0 turns injection off.  The device sees no fault; the
 * context becomes failed exactly as after a real OOC_E_DEVICE (the failing
 * call returns OOC_E_DEVICE, later calls OOC_E_FAILED, ooc_destroy still
 * waits for the issued work and frees everything).  OOC_E_ARG for n < 0. */
int ooc_debug_fail_after(ooc_ctx *ctx, int64_t n);

/* Waits for the context's device work on its three streams (also after a
 * failure: errors of that wait are ignored), then frees its events, pinned
 * host arrays, argument tables, streams and arena where the library created
 * them, and the context itself.  OOC_E_ARG for NULL. */
int ooc_destroy(ooc_ctx *ctx);

/* ------------------------------------------------------------ inspection */
/* Plan the chain that the next flush would execute first, without running it,
 * and expose the plan (owned by the context, valid until the next call that
 * plans or flushes).  Used by host-side tests of the tiling analysis. */
typedef struct {
  int32_t ntiles, nloops, nfields, slots;
  int64_t tile_rows;
  uint64_t slot_bytes;
  const int64_t *loop_rows;   /* [nloops][ntiles][2]: tiled-axis rows of loop i in tile t */
  const int64_t *resident;    /* [nfields][ntiles][2]: rows held in the slot during tile t */
  int32_t nup, ndown, nedge;  /* counts of transfer runs */
  const int64_t *up;          /* [nup][4]: field, tile, row_lo, row_hi (uploaded before tile) */
  const int64_t *down;        /* [ndown][4]: field, tile, row_lo, row_hi (downloaded after tile) */
  const int64_t *edge;        /* [nedge][4]: field, tile, row_lo, row_hi (copied tile-1 -> tile) */
  const int32_t *temporary;   /* [nfields]: 1 if no element is read before written in the chain */
  int32_t ring;               /* 1 with OOC_FLAG_RING: then no edge copies are made, and ... */
  const int64_t *ring_rows;   /* [nfields]: ... rows of each field's ring (0 if not streamed) */
} ooc_plan_info;

int ooc_debug_plan(ooc_ctx *ctx, ooc_plan_info *out);

/* Field geometry: logical lower bound and extent per axis (the storage
 * layout is given by ooc_get_layout). */
int ooc_field_shape(ooc_ctx *ctx, ooc_field f, int64_t lo[3], int64_t n[3]);

/* ------------------------------------------------------- schedule cost model
 * A small multilayer perceptron (inputs -> H tanh -> H tanh -> 1 linear, FP64,
 * mean-squared-error loss) trained on the device by the library's own forward,
 * backward and Adam kernels.  It learns log time per cell-step of a schedule
 * (tile height, chain length, buffer depth) from features of the plan, and
 * proposes schedules; the exhaustive sweep is its fallback and yardstick.  This is
 * an extension, not part of the paper.  X is row-major N x n_inputs (host);
 * all buffers are the caller's and copied.  Every call returns 0, OOC_E_ARG
 * for a NULL or out-of-range argument (n_inputs 1..256, n_hidden 1..1024,
 * n >= 1), or OOC_E_DEVICE when a device call fails. */
typedef struct ooc_mlp ooc_mlp;
int ooc_mlp_create(ooc_mlp **out, int n_inputs, int n_hidden, uint64_t seed);
int ooc_mlp_num_params(ooc_mlp *m);
/* parameter vector layout: W0[H][D], b0[H], W1[H][H], b1[H], W2[H], b2 */
int ooc_mlp_get_params(ooc_mlp *m, double *out);
int ooc_mlp_set_params(ooc_mlp *m, const double *in);  /* also resets Adam state */
int ooc_mlp_predict(ooc_mlp *m, const double *X, int n, double *out);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same prediction
 * as ooc_mlp_predict, bit for bit (same kernels), but it allocates nothing.
 * Its inputs, hidden activations and outputs live in one static device array
 * of OOC_MLP_SCRATCH_DOUBLES doubles (4 MiB), held by every device the
 * library runs on until the process ends.  A batch needs
 * pad(n*n_inputs) + 2*pad(n*n_hidden) + pad(n) doubles, pad() rounding up to
 * a multiple of 32; a larger batch is refused with OOC_E_ARG before any
 * device work.  X (n x n_inputs, row-major) and out (n) are host memory owned
 * by the caller.  The call runs on the network's device and stream and waits
 * for its result.  All calls on one device share the array: calls that
 * overlap in time on one device (from several threads) race.  OOC_E_ARG for a
 * NULL pointer or n < 1, OOC_E_DEVICE when a device call fails. */
#define OOC_MLP_SCRATCH_DOUBLES 524288
int ooc_mlp_predict_noalloc(ooc_mlp *m, const double *X, int n, double *out);
/* gradient of the loss with respect to every parameter (same layout) */
int ooc_mlp_gradient(ooc_mlp *m, const double *X, const double *y, int n, double *grad, double *loss);
/* full-batch Adam (beta 0.9 / 0.999, eps 1e-8); loss after the last epoch */
int ooc_mlp_train(ooc_mlp *m, const double *X, const double *y, int n, int epochs, double lr, double *loss);
int ooc_mlp_destroy(ooc_mlp *m);

#ifdef __cplusplus
}
#endif
#endif /* OOC_H */
