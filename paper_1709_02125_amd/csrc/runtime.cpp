// C ABI of the out-of-core stencil loop-chain library: context, validation,
// lazy loop queue, chain splitting, device memory manager and the three-stream
// tile pipeline (the paper's Algorithm 1 with the optimisations of Section 4.1).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <stdexcept>
#include <thread>

#include "ooc_internal.h"

using namespace ooc;

namespace {

struct DeviceError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct ArgError : std::runtime_error {
  int code;
  ArgError(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

// failure injection (ooc_debug_fail_after): called after every checked call
void after_hip_call();

#define HIPCHK(x)                                                                  \
  do {                                                                             \
    hipError_t e_ = (x);                                                           \
    if (e_ != hipSuccess)                                                          \
      throw DeviceError(std::string(#x) + ": " + hipGetErrorString(e_));           \
    after_hip_call();                                                              \
  } while (0)

uint64_t align256(uint64_t x) { return (x + 255) / 256 * 256; }

struct KStat {
  double ms = 0;
  uint64_t launches = 0, bytes = 0;
};

struct TimedLaunch {
  int kid;
  uint64_t bytes;
  hipEvent_t a, b;
};

// parallel fill / copy of large host buffers
void par_memcpy(void *dst, const void *src, size_t n) {
  const size_t chunk = 256ull << 20;
  if (n < 2 * chunk) {
    if (src) std::memcpy(dst, src, n);
    else std::memset(dst, 0, n);
    return;
  }
  int nt = (int)std::min<size_t>(16, (n + chunk - 1) / chunk);
  std::vector<std::thread> th;
  size_t per = (n + nt - 1) / nt;
  for (int k = 0; k < nt; k++) {
    size_t o = k * per, m = std::min(per, n - std::min(n, o));
    if (!m) continue;
    th.emplace_back([=] {
      if (src) std::memcpy((char *)dst + o, (const char *)src + o, m);
      else std::memset((char *)dst + o, 0, m);
    });
  }
  for (auto &t : th) t.join();
}

}  // namespace

struct ooc_ctx {
  int ndim = 2, tax = 1, halo = 2;
  int64_t dims[3] = {1, 1, 1};
  size_t budget = 0;
  uint32_t flags = 0;
  int64_t pitch = 0, plane = 0;
  std::vector<Field> fields;
  std::vector<char> pinned;  // per field: host array is pinned
  std::vector<Reduction> reds;
  std::vector<LoopRec> queue;
  int marks = 0;
  int64_t tile_rows = 0;
  int chain_steps = 0;
  int slots = 3;
  // device
  bool bound = false, own_arena = false, own_streams = false, ready = false, failed = false;
  char *arena = nullptr;
  size_t arena_bytes = 0;
  hipStream_t s_up = nullptr, s_comp = nullptr, s_down = nullptr;
  char *slot_base = nullptr;
  uint64_t slot_stride = 0;
  // ring slabs (OOC_FLAG_RING): per field one ring of device memory mapped
  // twice at consecutive virtual addresses, and the staging areas of the S
  // tiles in flight
  struct Ring {
    char *va = nullptr;
    uint64_t bytes = 0;
    hipMemGenericAllocationHandle_t h{};
    bool created = false;
    int maps = 0;
  };
  std::vector<Ring> rings;
  // where each ring holds the current chain's rows (bytes; row r at
  // (r * row bytes + origin) mod ring bytes), and the previous chain's held
  // rows and origins, from which the next chain's origins are chosen
  std::vector<uint64_t> ring_origin;
  bool ring_prev_valid = false;
  int64_t ring_prev_g0 = 0;
  int ring_prev_T = 0;
  std::vector<int64_t> ring_prev_resA, ring_prev_resB;
  std::vector<uint64_t> ring_prev_origin;
  char *stage_base = nullptr;
  uint64_t stage_stride = 0, stage_alloc = 0;
  uint64_t ring_granule = kRingGranule;
  int device = 0;
  // tiles and events
  int64_t gtile = 0, gbase = 0, gsynced = -1;
  int64_t prev_last_tile = -1;   // last tile of the previously issued chain
  int64_t prev2_last_tile = -1;  // last tile of the chain issued before that one
  std::vector<hipEvent_t> ev_up, ev_comp, ev_down;  // indexed by g - gbase
  std::map<std::string, Plan> plans;
  Plan dbg;
  std::vector<int64_t> dbg_loop_rows, dbg_res, dbg_up, dbg_down, dbg_edge, dbg_ring;
  ooc_stats st{};
  bool timing = false;
  int timing_kid = -1;  // with timing: only this kernel id (-1: every loop)
  std::vector<TimedLaunch> timed;
  std::vector<hipEvent_t> tev_pool;
  size_t tev_next = 0;
  std::map<int, KStat> kstats;
  // per-tile stage events (ooc_set_tile_timing): 7 per tile, pooled
  bool tile_timing = false;
  struct TileEv {
    int64_t g;
    hipEvent_t e[7];  // h2d begin/end, compute begin/end, edge end, d2h begin/end
  };
  std::vector<TileEv> tile_ev;
  std::vector<hipEvent_t> tile_pool;
  size_t tile_pool_next = 0;
  std::vector<ooc_tile_time> tile_times;
  // per-chain launch-argument tables: device copy read by the kernels, pinned
  // host mirror it is uploaded from, cache keyed by chain and slot phase
  KArgs *argtab_dev = nullptr, *argtab_host = nullptr;
  size_t argtab_cap = 0, argtab_used = 0;
  std::map<std::string, size_t> argtab_cache;
  // captured chain pipelines (OOC_FLAG_GRAPH), keyed like the argument table
  struct ChainGraph {
    hipGraphExec_t exec;
    uint64_t launches;
  };
  std::map<std::string, ChainGraph> graphs;
  int64_t capture_g0 = -1;  // first tile of the chain being captured, -1 if none
  hipEvent_t ev_fork = nullptr, ev_join_c = nullptr, ev_join_d = nullptr, ev_pre = nullptr, ev_post = nullptr;
  int64_t fail_after = 0;  // ooc_debug_fail_after: checked calls left until the injected failure
  std::string err;
};

namespace {

// context whose ABI call is running on this thread (set by guarded())
thread_local ooc_ctx *t_ctx = nullptr;

void after_hip_call() {
  ooc_ctx *c = t_ctx;
  if (c && c->fail_after > 0 && --c->fail_after == 0)
    throw DeviceError("injected failure of a runtime call (ooc_debug_fail_after)");
}

KernelInfo *g_table = nullptr;

KernelInfo *table() {
  if (!g_table) {
    g_table = kernel_table();
    register_common_kernels(g_table);
    register_hydro2d_kernels(g_table);
    register_ns3d_kernels(g_table);
    register_hydro3d_kernels(g_table);
  }
  return g_table;
}

hipEvent_t &evref(std::vector<hipEvent_t> &v, ooc_ctx *c, int64_t g) {
  size_t k = (size_t)(g - c->gbase);
  while (v.size() <= k) {
    hipEvent_t e;
    HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    v.push_back(e);
  }
  return v[k];
}

// Host-side issue profile (OOC_PROFILE_HOST=1 prints it per flush): time spent
// in each kind of runtime call while issuing.
enum { kCallH2D, kCallD2H, kCallLaunch, kCallWait, kCallRecord, kCallOther, kCallN };
double g_call_ms[kCallN];
int g_call_n[kCallN];
double g_call_max[kCallN];

template <class Fn>
void timed_call(ooc_ctx *c, Fn fn, int kind = kCallH2D) {
  auto a = std::chrono::steady_clock::now();
  fn();
  double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - a).count();
  if (ms > c->st.max_call_ms) {
    c->st.max_call_ms = ms;
    c->st.max_call_kind = kind;
    c->st.max_call_chain = (int32_t)c->st.chains;
  }
  g_call_ms[kind] += ms;
  g_call_n[kind]++;
  g_call_max[kind] = std::max(g_call_max[kind], ms);
}

void wait_tile(ooc_ctx *c, hipStream_t s, std::vector<hipEvent_t> &v, int64_t g) {
  if (g <= c->gsynced || g < c->gbase) return;
  if (c->capture_g0 >= 0 && g < c->capture_g0) return;  // ordered before the graph instead
  hipEvent_t e = evref(v, c, g);
  timed_call(c, [&] { HIPCHK(hipStreamWaitEvent(s, e, 0)); }, kCallWait);
}

// record stage k of the tile being issued (tile timing on)
void tile_mark(ooc_ctx *c, int k, hipStream_t s) {
  if (c->tile_ev.empty()) return;
  hipEvent_t &e = c->tile_ev.back().e[k];
  timed_call(c, [&] { HIPCHK(hipEventRecord(e, s)); }, kCallRecord);
}

void tile_begin(ooc_ctx *c, int64_t g) {
  ooc_ctx::TileEv t;
  t.g = g;
  for (hipEvent_t &e : t.e) {
    if (c->tile_pool_next == c->tile_pool.size()) {
      hipEvent_t x;
      HIPCHK(hipEventCreate(&x));
      c->tile_pool.push_back(x);
    }
    e = c->tile_pool[c->tile_pool_next++];
  }
  c->tile_ev.push_back(t);
}

// turn the stage events of the tiles issued since the last collection into
// microseconds from the first tile's upload begin (after a device sync)
void collect_tile_times(ooc_ctx *c) {
  if (c->tile_ev.empty()) return;
  c->tile_times.clear();
  const hipEvent_t base = c->tile_ev[0].e[0];
  for (const ooc_ctx::TileEv &t : c->tile_ev) {
    float us[7];
    for (int k = 0; k < 7; k++) {
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, base, t.e[k]));
      us[k] = ms * 1e3f;
    }
    c->tile_times.push_back({t.g, us[0], us[1], us[2], us[3], us[4], us[5], us[6]});
  }
  c->tile_ev.clear();
  c->tile_pool_next = 0;
}

hipEvent_t timing_event(ooc_ctx *c) {
  if (c->tev_next == c->tev_pool.size()) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    c->tev_pool.push_back(e);
  }
  return c->tev_pool[c->tev_next++];
}

void *alloc_host(ooc_ctx *c, size_t bytes, bool &pinned) {
  void *p = nullptr;
  pinned = false;
  if (c->bound && bytes) {
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) == hipSuccess) {
      pinned = true;
      return p;
    }
    (void)hipGetLastError();
  }
  p = std::aligned_alloc(4096, std::max<size_t>(4096, (bytes + 4095) / 4096 * 4096));
  return p;
}

// device address of a pinned host array (kernel-copy transfers)
void map_host(Field &f) {
  void *d = nullptr;
  if (f.host && hipHostGetDevicePointer(&d, f.host, 0) == hipSuccess) f.host_dev = d;
  else (void)hipGetLastError();
}

void free_host(void *p, bool pinned) {
  if (!p) return;
  if (pinned) (void)hipHostFree(p);
  else std::free(p);
}

// Storage layout of a field: every field shares the row pitch (x) and, in 3D,
// the plane size (x * y), so kernels index all fields alike.  Within a row, x
// = 0 is element kXOrigin (a 128-byte boundary when the row starts on one):
// a 64-point row segment starting at a multiple of 16 is four whole lines.
void layout_field(ooc_ctx *c, Field &f) {
  for (int a = 0; a < 3; a++) {
    if (a < c->ndim) {
      f.lo[a] = -c->halo;
      f.n[a] = c->dims[a] + 2 * c->halo + f.delta[a];
    } else {
      f.lo[a] = 0;
      f.n[a] = 1;
    }
  }
  f.nrows = f.n[c->tax];
  f.row_elems = c->ndim == 2 ? c->pitch : c->plane;
}

// host <-> logical extent copy (field storage is padded to the shared pitch)
void copy_extent(ooc_ctx *c, Field &f, double *dst, const double *src, bool to_user) {
  const int64_t nx = f.n[0];
  const int64_t ny = c->ndim == 3 ? f.n[1] : f.n[1];
  const int64_t nz = c->ndim == 3 ? f.n[2] : 1;
  for (int64_t k = 0; k < nz; k++)
    for (int64_t j = 0; j < ny; j++) {
      int64_t so = (c->ndim == 3 ? k * c->plane + j * c->pitch : j * c->pitch) + kXOrigin + f.lo[0];
      int64_t uo = (k * ny + j) * nx;
      if (f.fp32) {
        float *h = (float *)f.host + so;
        if (to_user) for (int64_t i = 0; i < nx; i++) dst[uo + i] = (double)h[i];
        else for (int64_t i = 0; i < nx; i++) h[i] = (float)src[uo + i];
      } else {
        double *h = (double *)f.host + so;
        if (to_user) std::memcpy(dst + uo, h, nx * 8);
        else std::memcpy(h, src + uo, nx * 8);
      }
    }
}

int fail(ooc_ctx *c, int code, const std::string &m) {
  c->err = m;
  return code;
}

#define GUARD(c)                                                   \
  if (!(c)) return OOC_E_ARG;                                      \
  if ((c)->failed) return OOC_E_FAILED;

template <class Fn>
int guarded(ooc_ctx *c, Fn fn) {
  struct Cur {
    ooc_ctx *prev;
    explicit Cur(ooc_ctx *x) : prev(t_ctx) { t_ctx = x; }
    ~Cur() { t_ctx = prev; }
  } cur(c);
  try {
    return fn();
  } catch (const DeviceError &e) {
    c->failed = true;
    c->err = e.what();
    return OOC_E_DEVICE;
  } catch (const ArgError &e) {
    c->err = e.what();
    return e.code;
  } catch (const std::bad_alloc &) {
    c->err = "host allocation failed";
    return OOC_E_NOMEM;
  }
}

void drop_graphs(ooc_ctx *c) {
  if (c->graphs.empty()) return;
  HIPCHK(hipStreamSynchronize(c->s_up));
  for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.second.exec);
  c->graphs.clear();
}

// The launch-argument table is metadata, not field data: it lives in its own
// small device allocation (outside the field budget), grown only at a point
// where no kernel can be reading it.
void grow_argtab(ooc_ctx *c, size_t entries) {
  if (entries <= c->argtab_cap) return;
  drop_graphs(c);
  if (c->argtab_dev) {
    HIPCHK(hipStreamSynchronize(c->s_comp));
    HIPCHK(hipFree(c->argtab_dev));
    free_host(c->argtab_host, true);
    c->argtab_dev = nullptr;
    c->argtab_host = nullptr;
  }
  HIPCHK(hipMalloc((void **)&c->argtab_dev, entries * sizeof(KArgs)));
  bool pin = false;
  c->argtab_host = (KArgs *)alloc_host(c, entries * sizeof(KArgs), pin);
  if (!pin) throw DeviceError("pinned allocation of the argument table failed");
  c->argtab_cap = entries;
  c->argtab_used = 0;
  c->argtab_cache.clear();
}

// ------------------------------------------------------------- device setup
int64_t sum_partials(const ooc_ctx *c) {
  return c->ndim == 2 ? c->dims[1] + 2 * c->halo + 1
                      : (c->dims[2] + 2 * c->halo + 1) * (c->dims[1] + 2 * c->halo + 1);
}

// Device bytes taken ahead of the slots: reduction buffers and resident fields.
constexpr size_t kArgTableBytes = 32u << 20;     // initial size of the launch-argument table
constexpr size_t kArgTableMaxBytes = 256u << 20;  // it grows while full up to this size

uint64_t reserved_bytes(const ooc_ctx *c) {
  uint64_t used = 0;
  for (const Reduction &r : c->reds) used += 256 + (r.op == OOC_RED_SUM ? align256(sum_partials(c) * 8) : 0);
  for (const Field &f : c->fields)
    if (f.resident) used += align256((uint64_t)f.nrows * f.row_elems * 8);
  return used;
}

// Ring slabs: device bytes available to the rings and the staging areas.
uint64_t ring_capacity(const ooc_ctx *c) {
  const uint64_t used = reserved_bytes(c);
  return c->budget > used ? c->budget - used : 0;
}

void free_rings(ooc_ctx *c) {
  for (ooc_ctx::Ring &r : c->rings) {
    if (r.maps > 1) (void)hipMemUnmap(r.va + r.bytes, r.bytes);
    if (r.maps > 0) (void)hipMemUnmap(r.va, r.bytes);
    if (r.va) (void)hipMemAddressFree(r.va, 2 * r.bytes);
    if (r.created) (void)hipMemRelease(r.h);
    r = ooc_ctx::Ring();
  }
  if (c->stage_base) (void)hipFree(c->stage_base);
  c->stage_base = nullptr;
  c->stage_alloc = 0;
}

// Give every field of the plan a ring at least as large as the plan needs.
// When one is short, all rings are released, once the device is done with
// them, and allocated afresh at the plan's sizes (which fit the budget):
// data does not live in the rings between chains.  Launch arguments cached
// for earlier chains point into the old rings and are dropped.
void ensure_rings(ooc_ctx *c, const Plan &P) {
  // the staging areas are laid out at the stride they were allocated with:
  // that stride must hold this plan's staging, and the allocation one area
  // per slot at that stride (the slot count may have grown since)
  bool ok = c->stage_stride >= P.stage_bytes && c->stage_alloc >= (uint64_t)c->slots * c->stage_stride;
  for (int f : P.slot_fields) ok = ok && c->rings[f].bytes >= P.ring_bytes[f];
  if (ok) return;
  for (hipStream_t st : {c->s_up, c->s_comp, c->s_down}) HIPCHK(hipStreamSynchronize(st));
  drop_graphs(c);
  c->argtab_cache.clear();
  c->argtab_used = 0;
  free_rings(c);
  c->ring_prev_valid = false;  // the device is done with every earlier chain
  std::fill(c->ring_origin.begin(), c->ring_origin.end(), 0);
  hipMemAllocationProp prop = {};
  prop.type = hipMemAllocationTypePinned;
  prop.location.type = hipMemLocationTypeDevice;
  prop.location.id = c->device;
  hipMemAccessDesc acc = {};
  acc.location = prop.location;
  acc.flags = hipMemAccessFlagsProtReadWrite;
  for (int f : P.slot_fields) {
    ooc_ctx::Ring &r = c->rings[f];
    if (!P.ring_bytes[f]) continue;
    r.bytes = P.ring_bytes[f];
    HIPCHK(hipMemCreate(&r.h, r.bytes, &prop, 0));
    r.created = true;
    void *va = nullptr;
    HIPCHK(hipMemAddressReserve(&va, 2 * r.bytes, c->ring_granule, nullptr, 0));
    r.va = (char *)va;
    HIPCHK(hipMemMap(r.va, r.bytes, 0, r.h, 0));
    r.maps = 1;
    HIPCHK(hipMemMap(r.va + r.bytes, r.bytes, 0, r.h, 0));
    r.maps = 2;
    HIPCHK(hipMemSetAccess(r.va, 2 * r.bytes, &acc, 1));
  }
  c->stage_stride = P.stage_bytes;
  if (P.stage_bytes) {
    HIPCHK(hipMalloc((void **)&c->stage_base, (uint64_t)c->slots * P.stage_bytes));
    c->stage_alloc = (uint64_t)c->slots * P.stage_bytes;
  }
}

// Device address of stored row `row` of field f in tile t: in the tile's
// slot, or in the field's ring (row r at byte (r * row bytes + the chain's
// origin) mod ring bytes of the first mapping, the window of the tile
// contiguous from there on).
char *row_ptr(ooc_ctx *c, const Plan &P, int f, int t, char *slot, int64_t row) {
  const Field &fd = c->fields[f];
  const int64_t A = P.resA[(size_t)f * P.T + t];
  if (P.ring) {
    const ooc_ctx::Ring &r = c->rings[f];
    if (!r.bytes) return r.va;  // not held in this chain
    return r.va + ((uint64_t)A * fd.row_bytes_dev() + c->ring_origin[f]) % r.bytes + (row - A) * fd.row_bytes_dev();
  }
  return slot + P.slab_off[f] + (row - A) * fd.row_bytes_dev();
}

void setup_device(ooc_ctx *c) {
  if (c->ready) return;
  if (!c->bound) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) throw DeviceError("no HIP device available");
    if (!(c->flags & OOC_FLAG_RING)) {  // ring slabs allocate their own memory below
      HIPCHK(hipMalloc((void **)&c->arena, c->budget));
      c->arena_bytes = c->budget;
      c->own_arena = true;
    }
    HIPCHK(hipStreamCreateWithFlags(&c->s_up, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&c->s_comp, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&c->s_down, hipStreamNonBlocking));
    c->own_streams = true;
    c->bound = true;
  }
  HIPCHK(hipGetDevice(&c->device));
  if (c->flags & OOC_FLAG_RING) {
    int vmm = 0;
    HIPCHK(hipDeviceGetAttribute(&vmm, hipDeviceAttributeVirtualMemoryManagementSupported, c->device));
    if (!vmm) throw ArgError(OOC_E_ARG, "ring slabs need the HIP virtual memory API, which this device lacks");
    hipMemAllocationProp prop = {};
    prop.type = hipMemAllocationTypePinned;
    prop.location.type = hipMemLocationTypeDevice;
    prop.location.id = c->device;
    size_t g = 0;
    HIPCHK(hipMemGetAllocationGranularity(&g, &prop, hipMemAllocationGranularityMinimum));
    if (g > 0) c->ring_granule = (kRingGranule + g - 1) / g * g;
    c->rings.assign(c->fields.size(), ooc_ctx::Ring());
    c->ring_origin.assign(c->fields.size(), 0);
    if (!c->arena) {  // bound without an arena: reductions and resident fields get their own
      const uint64_t need = std::max<uint64_t>(reserved_bytes(c), 256);
      HIPCHK(hipMalloc((void **)&c->arena, need));
      c->arena_bytes = need;
      c->own_arena = true;
    }
  }
  // pin host arrays declared before the device was bound
  for (size_t k = 0; k < c->fields.size(); k++) {
    Field &f = c->fields[k];
    if (c->pinned[k]) continue;
    bool pin = false;
    void *p = alloc_host(c, f.host_bytes(), pin);
    par_memcpy(p, f.host, f.host_bytes());
    free_host(f.host, false);
    f.host = p;
    c->pinned[k] = pin;
    if (pin) map_host(f);
  }
  c->st.host_pinned_bytes = c->st.host_pageable_bytes = 0;
  for (size_t k = 0; k < c->fields.size(); k++)
    (c->pinned[k] ? c->st.host_pinned_bytes : c->st.host_pageable_bytes) += c->fields[k].host_bytes();
  const size_t budget = std::min(c->budget, c->arena_bytes);
  uint64_t off = 0;
  grow_argtab(c, kArgTableBytes / sizeof(KArgs));
  for (Reduction &r : c->reds) {
    r.acc = (double *)(c->arena + off);
    r.committed = (double *)(c->arena + off + 8);
    off += 256;
    if (r.op == OOC_RED_SUM) {
      r.npartials = sum_partials(c);
      r.partials = (double *)(c->arena + off);
      off += align256(r.npartials * 8);
    }
  }
  for (Field &f : c->fields) {
    if (!f.resident) continue;
    f.dev_res = (double *)(c->arena + off);
    off += align256((uint64_t)f.nrows * f.row_elems * 8);
  }
  if (off > budget)
    throw ArgError(OOC_E_BUDGET, "resident fields and reductions need " + std::to_string(off) +
                                     " bytes, more than the budget of " + std::to_string(budget));
  c->slot_base = c->arena + off;
  c->slot_stride = (c->flags & OOC_FLAG_RING) ? ring_capacity(c) : (budget - off) / c->slots / 256 * 256;
  // initial device state: reductions, resident fields
  for (Reduction &r : c->reds) {
    double v = r.host_set ? r.host_value : 0.0;
    HIPCHK(hipMemcpyAsync(r.committed, &v, 8, hipMemcpyHostToDevice, c->s_comp));
  }
  for (Field &f : c->fields) {
    if (!f.resident) continue;
    HIPCHK(hipMemcpyAsync(f.dev_res, f.host, (size_t)f.nrows * f.row_elems * 8, hipMemcpyHostToDevice,
                          c->s_comp));
    f.dev_valid = true;
    f.host_valid = true;
  }
  HIPCHK(hipStreamSynchronize(c->s_comp));
  c->ready = true;
}

// ------------------------------------------------------------ chain running
std::string plan_key(ooc_ctx *c, const LoopRec *L, int n) {
  std::string k;
  auto put = [&](const void *p, size_t b) { k.append((const char *)p, b); };
  int hdr[4] = {(c->flags & OOC_FLAG_CYCLIC) ? 1 : 0, c->slots, n, 0};
  put(hdr, sizeof hdr);
  put(&c->tile_rows, 8);
  put(&c->slot_stride, 8);
  for (int i = 0; i < n; i++) {
    put(&L[i].kid, 4);
    put(L[i].lo, 24);
    put(L[i].hi, 24);
    for (const ArgRec &a : L[i].args) {
      int h[3] = {a.kind, a.handle, a.access};
      put(h, sizeof h);
      if (a.kind == OOC_ARG_DAT) {
        int np = a.npts();
        put(&np, 4);
        put(a.offs.data(), a.offs.size() * 4);
      }
    }
  }
  return k;
}

const Plan &get_plan(ooc_ctx *c, const LoopRec *L, int n) {
  std::string key = plan_key(c, L, n);
  auto it = c->plans.find(key);
  if (it != c->plans.end()) return it->second;
  PlanInput in;
  in.ndim = c->ndim;
  in.tax = c->tax;
  in.halo = c->halo;
  in.fields = &c->fields;
  in.loops = L;
  in.nloops = n;
  in.cyclic = (c->flags & OOC_FLAG_CYCLIC) != 0;
  in.S = c->slots;
  in.forced_h = c->tile_rows;
  in.ring = (c->flags & OOC_FLAG_RING) != 0;
  in.ring_granule = c->ring_granule;
  in.slot_capacity = c->ready ? c->slot_stride : UINT64_MAX;
  if (in.ring) {
    in.slot_capacity = ring_capacity(c);
  } else if (!c->ready) {
    // planning before the device exists (inspection): use the budget minus
    // what resident fields and reductions will take
    const uint64_t used = reserved_bytes(c);
    in.slot_capacity = c->budget > used ? (c->budget - used) / c->slots / 256 * 256 : 0;
  }
  Plan p;
  std::string err;
  int rc = make_plan(in, p, err);
  if (rc != OOC_OK) throw ArgError(rc, err);
  if (c->plans.size() > 64) c->plans.clear();
  return c->plans.emplace(key, std::move(p)).first->second;
}

double *field_ptr(ooc_ctx *c, int f, const Plan &P, int t, char *slot) {
  Field &fd = c->fields[f];
  char *base;
  int64_t A;
  if (fd.resident) {
    base = (char *)fd.dev_res;
    A = 0;
  } else {
    A = P.resA[(size_t)f * P.T + t];
    base = row_ptr(c, P, f, t, slot, A);
  }
  int64_t shift = -A * fd.row_elems + kXOrigin - fd.lo[1] * c->pitch;
  if (c->ndim == 3) shift -= fd.lo[2] * c->plane;
  return (double *)(base + shift * 8);
}

KArgs make_kargs(ooc_ctx *c, const LoopRec &L, const Plan &P, int i, int t, char *slot, uint64_t *bytes_out) {
  KArgs a;
  std::memset(&a, 0, sizeof a);
  for (int d = 0; d < 3; d++) {
    a.lo[d] = (int32_t)L.lo[d];
    a.hi[d] = (int32_t)L.hi[d];
  }
  a.lo[c->tax] = (int32_t)P.s(i, t);
  a.hi[c->tax] = (int32_t)P.en(i, t);
  a.pitch = c->pitch;
  a.plane = c->plane;
  a.halo = c->halo;
  a.red_rows = c->dims[1] + 2 * c->halo + 1;
  int nd = 0, nc = 0, ndv = 0, nr = 0;
  uint64_t bytes = 0;
  int64_t pts = 1;
  for (int d = 0; d < c->ndim; d++) pts *= (a.hi[d] - a.lo[d]);
  for (const ArgRec &g : L.args) {
    switch (g.kind) {
      case OOC_ARG_DAT:
        a.p[nd] = field_ptr(c, g.handle, P, t, slot);
        for (int q = 0; q < 3; q++) a.off[nd][q] = g.offs[q];
        if (nd == 1) {
          a.nst = std::min(g.npts(), kMaxStencil);
          for (int s = 0; s < a.nst; s++)
            for (int q = 0; q < 3; q++) a.st[s][q] = g.offs[3 * s + q];
        }
        bytes += (uint64_t)pts * 8 * (g.access == OOC_RW || g.access == OOC_INC ? 2 : 1);
        nd++;
        break;
      case OOC_ARG_CONST: a.c[nc++] = g.value; break;
      case OOC_ARG_DEVSCALAR: a.ds[ndv++] = c->reds[g.handle].committed; break;
      case OOC_ARG_RED: {
        Reduction &r = c->reds[g.handle];
        a.red[nr++] = r.op == OOC_RED_SUM ? r.partials : r.acc;
      } break;
    }
  }
  a.ndat = nd;
  *bytes_out = bytes;
  return a;
}

void launch_loop(ooc_ctx *c, int kid, const KArgs &a, const KArgs *dev, uint64_t bytes) {
  const KernelInfo &ki = table()[kid];
  if (c->timing && (c->timing_kid < 0 || c->timing_kid == kid)) {
    TimedLaunch tl{kid, bytes, timing_event(c), timing_event(c)};
    HIPCHK(hipEventRecord(tl.a, c->s_comp));
    ki.launch(a, dev, c->ndim, c->s_comp);
    HIPCHK(hipGetLastError());
    HIPCHK(hipEventRecord(tl.b, c->s_comp));
    c->timed.push_back(tl);
  } else {
    timed_call(c, [&] { ki.launch(a, dev, c->ndim, c->s_comp); }, kCallLaunch);
    HIPCHK(hipGetLastError());
  }
  c->st.launches++;
}

// Can loops a and b (a before b) run in one launch?  Only if neither writes a
// point the other reads or writes: every write box is tested against every
// access box of the other loop on the same field.
bool loops_independent(const LoopRec &a, const LoopRec &b, int ndim) {
  auto box_meet = [&](const LoopRec &x, const int32_t *ox, const LoopRec &y, const int32_t *oy) {
    for (int d = 0; d < ndim; d++)
      if (x.lo[d] + ox[d] >= y.hi[d] + oy[d] || y.lo[d] + oy[d] >= x.hi[d] + ox[d]) return false;
    return true;
  };
  static const int32_t zero[3] = {0, 0, 0};
  for (int pass = 0; pass < 2; pass++) {
    const LoopRec &w = pass ? b : a, &o = pass ? a : b;
    for (const ArgRec &gw : w.args) {
      if (gw.kind != OOC_ARG_DAT || !writes_access(gw.access)) continue;
      for (const ArgRec &go : o.args) {
        if (go.kind != OOC_ARG_DAT || go.handle != gw.handle) continue;
        for (int p = 0; p < go.npts(); p++)
          if (box_meet(w, zero, o, &go.offs[3 * p])) return false;
      }
    }
  }
  return true;
}

bool loop_nonempty(const LoopRec &L, int ndim) {
  for (int d = 0; d < ndim; d++)
    if (L.hi[d] <= L.lo[d]) return false;
  return true;
}

void run_chain(ooc_ctx *c, const LoopRec *L, int n, int64_t prev_last_tile) {
  auto issue0 = std::chrono::steady_clock::now();
  const Plan &P = get_plan(c, L, n);
  if ((uint64_t)P.slot_bytes > c->slot_stride)
    throw ArgError(OOC_E_BUDGET, P.ring ? "plan does not fit the ring capacity" : "plan does not fit its slot");
  if (P.ring) ensure_rings(c, P);
  const int T = P.T, S = c->slots;
  const bool dbg_sync = (c->flags & OOC_FLAG_DEBUG_SYNC) != 0;
  // reductions written in this chain: start from the operator's identity
  std::vector<int> wreds;
  for (int i = 0; i < n; i++)
    for (const ArgRec &g : L[i].args)
      if (g.kind == OOC_ARG_RED && std::find(wreds.begin(), wreds.end(), g.handle) == wreds.end())
        wreds.push_back(g.handle);
  // index transfer runs by tile
  std::vector<std::vector<const Run *>> up(T), down(T), edge(T);
  for (const Run &r : P.up) up[r.t].push_back(&r);
  for (const Run &r : P.down) down[r.t].push_back(&r);
  for (const Run &r : P.edge) edge[r.t].push_back(&r);
  const int64_t g0 = c->gtile;
  // ring slabs: each ring's origin for this chain, and for its first S tiles
  // the previous chain's tile whose download must end first (-1: none)
  std::vector<int64_t> ring_wait(S, -1);
  if (P.ring) {
    const int64_t prev_end = c->ring_prev_g0 + c->ring_prev_T;
    if (!c->ring_prev_valid || prev_end != g0 || prev_end - 1 <= c->gsynced) {
      std::fill(c->ring_origin.begin(), c->ring_origin.end(), 0);  // the device is done with the previous chain
    } else {
      const int nf = (int)c->fields.size();
      std::vector<uint64_t> rbytes(nf), rowb(nf);
      for (int f = 0; f < nf; f++) {
        rbytes[f] = c->rings[f].bytes;
        rowb[f] = c->fields[f].row_bytes_dev();
      }
      RingChain pv, nx;
      pv.T = c->ring_prev_T;
      pv.resA = c->ring_prev_resA.data();
      pv.resB = c->ring_prev_resB.data();
      pv.origin = c->ring_prev_origin.data();
      nx.T = T;
      nx.resA = P.resA.data();
      nx.resB = P.resB.data();
      std::vector<int64_t> w(S);
      choose_ring_origins(nf, rbytes.data(), rowb.data(), pv, nx, S, c->ring_origin.data(), w.data());
      for (int t = 0; t < S; t++)
        if (w[t] >= 0) ring_wait[t] = c->ring_prev_g0 + w[t];
    }
  }
  // launch arguments of the whole chain, built and uploaded once per distinct
  // (chain, slot phase) and reused by every later identical chain
  struct Launch {
    int kid;
    uint64_t bytes;
  };
  std::vector<Launch> launches;
  std::vector<KArgs> hostargs;
  // a tile's slot (ring slabs: its staging area)
  auto slot_of = [&](int64_t g) {
    return P.ring ? c->stage_base + (uint64_t)(g % S) * c->stage_stride : c->slot_base + (uint64_t)(g % S) * c->slot_stride;
  };
  if (P.ring && P.stage_bytes &&
      (c->stage_stride < P.stage_bytes || (uint64_t)S * c->stage_stride > c->stage_alloc))
    throw ArgError(OOC_E_STATE, "ring staging areas do not cover the plan");
  for (int t = 0; t < T; t++) {
    char *slot = slot_of(g0 + t);
    for (int i = 0; i < n; i++)
      if (P.s(i, t) < P.en(i, t) && loop_nonempty(L[i], c->ndim)) {
        uint64_t b = 0;
        hostargs.push_back(make_kargs(c, L[i], P, i, t, slot, &b));
        launches.push_back({L[i].kid, b});
      }
  }
  std::string akey = plan_key(c, L, n);
  for (int i = 0; i < n; i++)
    for (const ArgRec &g : L[i].args)
      if (g.kind == OOC_ARG_CONST) akey.append((const char *)&g.value, 8);
  const int64_t phase = g0 % S;
  akey.append((const char *)&phase, 8);
  if (P.ring) akey.append((const char *)c->ring_origin.data(), c->ring_origin.size() * sizeof(uint64_t));
  size_t abase;
  auto hit = c->argtab_cache.find(akey);
  if (hit != c->argtab_cache.end()) {
    abase = hit->second;
  } else {
    if (hostargs.size() > c->argtab_cap) grow_argtab(c, 2 * hostargs.size());
    if (c->argtab_used + hostargs.size() > c->argtab_cap) {
      // table full: a larger one up to a limit (chains that differ only in
      // their slot phase or ring origins each have entries of their own),
      // else wait until no kernel reads it and start over
      if (c->argtab_cap * sizeof(KArgs) < kArgTableMaxBytes) {
        grow_argtab(c, 2 * c->argtab_cap);
      } else {
        drop_graphs(c);
        HIPCHK(hipStreamSynchronize(c->s_comp));
        c->argtab_cache.clear();
        c->argtab_used = 0;
      }
    }
    abase = c->argtab_used;
    std::memcpy(c->argtab_host + abase, hostargs.data(), hostargs.size() * sizeof(KArgs));
    timed_call(c, [&] {
      HIPCHK(hipMemcpyAsync(c->argtab_dev + abase, c->argtab_host + abase, hostargs.size() * sizeof(KArgs),
                            hipMemcpyHostToDevice, c->s_comp));
    }, kCallOther);
    c->argtab_used += hostargs.size();
    c->argtab_cache.emplace(akey, abase);
  }
  // transfer byte counts (known from the plan)
  uint64_t chain_up = 0, chain_down = 0;
  for (const Run &r : P.up) {
    const uint64_t nb = (uint64_t)(r.hi - r.lo) * c->fields[r.f].row_bytes_host();
    c->st.bytes_h2d += nb;
    c->st.last_bytes_h2d += nb;
    chain_up += nb;
  }
  for (const Run &r : P.down) {
    const uint64_t nb = (uint64_t)(r.hi - r.lo) * c->fields[r.f].row_bytes_host();
    c->st.bytes_d2h += nb;
    c->st.last_bytes_d2h += nb;
    chain_down += nb;
  }
  // A chain that moves at most 60 % as much down as up is bound by its
  // uploads; its download kernel then runs on a narrow grid, since host
  // stores in flight slow the concurrent DMA uploads (measured on C2: 2
  // blocks 239 ms per step, 8 blocks 270 ms).  Otherwise the wider grid
  // finishes each download sooner (C4: 8 blocks 111 ms, 2 blocks 121 ms).
  const bool narrow_down = chain_down * 5 <= chain_up * 3;
  // Float32 downloads round on the way out.  A chain whose kernels move more
  // than 60 times its link bytes through HBM is bound by its kernels: its
  // downloads keep 8-byte host stores, which slow the stencils beside them
  // less (ns3d 512^3 FP32: 82-85 against 90-91 ms per step with 16-byte
  // stores); otherwise 16-byte stores move the rows faster (hydro2d 15360^2
  // FP32 with resident geometry: 102 against 122 ms).
  const int f32_down_mode = P.alg_bytes > 60 * (chain_up + chain_down) ? 2 : 3;
  if (!P.ring)  // in rings the rows two tiles share stay in place
    for (const Run &r : P.edge) c->st.bytes_edge += (uint64_t)(r.hi - r.lo) * c->fields[r.f].row_elems * 8;
  const uint64_t launches0 = c->st.launches;

  auto body = [&]() {
  for (int h : wreds) {
    Reduction &r = c->reds[h];
    if (r.op == OOC_RED_SUM) launch_fill(r.partials, r.npartials, 0.0, c->s_comp);
    else launch_red_init(r.acc, r.op == OOC_RED_MIN ? INFINITY : -INFINITY, c->s_comp);
  }
  size_t li = 0;
  for (int t = 0; t < T; t++) {
    const int64_t g = c->gtile++;
    char *slot = slot_of(g);
    // ---- upload: the rows of the tile's footprint that the previous tile
    // does not hand over (Algorithm 1's upload stage)
    wait_tile(c, c->s_up, c->ev_down, g - S);  // slot free again
    if (t == 0 && prev_last_tile >= 0 && !(c->flags & OOC_FLAG_PREFETCH))
      wait_tile(c, c->s_up, c->ev_comp, prev_last_tile);  // no early start of the next chain
    // ring slabs: the first tiles may take ring positions of the previous
    // chain's last tiles; then they start once those are downloaded
    if (P.ring && t < S && ring_wait[t] >= 0) wait_tile(c, c->s_up, c->ev_down, ring_wait[t]);
    if (P.ring && (c->flags & OOC_FLAG_DEBUG_POISON)) {
      // poison the rows the tile brings into its rings (before the uploads)
      for (int f : P.slot_fields) {
        const int64_t A = P.resA[(size_t)f * T + t], B = P.resB[(size_t)f * T + t];
        if (B <= A) continue;
        const bool prev = t > 0 && P.resB[(size_t)f * T + t - 1] > P.resA[(size_t)f * T + t - 1];
        const int64_t new0 = prev ? std::max(A, P.resB[(size_t)f * T + t - 1]) : A;
        if (new0 < B)
          launch_fill((double *)row_ptr(c, P, f, t, slot, new0), (B - new0) * c->fields[f].row_elems, NAN, c->s_up);
      }
    } else if (c->flags & OOC_FLAG_DEBUG_POISON) {
      // a slot with an incoming edge was poisoned on the compute stream just
      // before that edge copy (see below); order this tile's uploads after it
      if (t == 0) launch_fill((double *)slot, P.slot_bytes / 8, NAN, c->s_up);
      else wait_tile(c, c->s_up, c->ev_comp, g - 1);
    }
    if (c->tile_timing && c->capture_g0 < 0) {
      tile_begin(c, g);
      tile_mark(c, 0, c->s_up);
    }
    int64_t waited = -1;
    uint64_t stage_up = 0, stage_down = 0;
    const bool kcopy = (c->flags & OOC_FLAG_KERNEL_COPY) != 0;
    std::vector<XferSeg> xup;
    for (const Run *r : up[t]) {
      Field &f = c->fields[r->f];
      int64_t dep = -1;
      for (int64_t q = r->lo; q < r->hi; q++) dep = std::max(dep, f.last_down[q]);
      if (dep > waited && dep > c->gsynced) {
        wait_tile(c, c->s_up, c->ev_down, dep);
        waited = dep;
      }
      char *dst = row_ptr(c, P, r->f, t, slot, r->lo);
      const size_t nb = (size_t)(r->hi - r->lo) * f.row_bytes_host();
      const char *src = (const char *)f.host + r->lo * f.row_bytes_host();
      if (kcopy) {
        if (!f.host_dev) throw DeviceError("kernel copy needs device-mapped pinned host arrays");
        const char *hsrc = (const char *)f.host_dev + r->lo * f.row_bytes_host();
        const int64_t elems = (r->hi - r->lo) * f.row_elems;
        xup.push_back(f.fp32 ? XferSeg{hsrc, dst, elems, 1} : XferSeg{hsrc, dst, (int64_t)nb / 16, 0});
        continue;
      }
      if (f.fp32) {  // float32 rows land in staging, widened into the slab
        char *stage = slot + P.stage_up_off + stage_up;
        timed_call(c, [&] { HIPCHK(hipMemcpyAsync(stage, src, nb, hipMemcpyHostToDevice, c->s_up)); });
        launch_f32_to_f64((const float *)stage, (double *)dst, (r->hi - r->lo) * f.row_elems, c->s_up);
        stage_up += align256(nb);
      } else {
        timed_call(c, [&] { HIPCHK(hipMemcpyAsync(dst, src, nb, hipMemcpyHostToDevice, c->s_up)); });
      }
    }
    if (!xup.empty()) {
      timed_call(c, [&] { launch_xfer_segments(xup.data(), (int)xup.size(), false, false, c->s_up); }, kCallH2D);
      HIPCHK(hipGetLastError());
    }
    if (c->tile_timing && c->capture_g0 < 0) tile_mark(c, 1, c->s_up);
    timed_call(c, [&] { HIPCHK(hipEventRecord(evref(c->ev_up, c, g), c->s_up)); }, kCallRecord);
    if (dbg_sync) HIPCHK(hipStreamSynchronize(c->s_up));
    // ---- execute every loop of the chain over its rows of this tile
    timed_call(c, [&] { HIPCHK(hipStreamWaitEvent(c->s_comp, evref(c->ev_up, c, g), 0)); }, kCallWait);
    if (c->tile_timing && c->capture_g0 < 0) tile_mark(c, 2, c->s_comp);
    // fused strip loops cannot be timed one by one: fusion stays on unless
    // the mirror loops themselves are being timed
    const bool fuse = (c->flags & OOC_FLAG_FUSE) &&
                      !(c->timing && (c->timing_kid < 0 || c->timing_kid == OOC_K_MIRROR));
    std::vector<const KArgs *> bh, bd;  // pending batch of independent mirror loops
    std::vector<int> bl;
    auto flush_batch = [&] {
      if (bh.size() == 1) {
        launch_loop(c, OOC_K_MIRROR, *bh[0], bd[0], 0);
      } else if (!bh.empty()) {
        timed_call(c, [&] { launch_mirror_batch(bh.data(), bd.data(), (int)bh.size(), c->ndim, c->s_comp); },
                   kCallLaunch);
        HIPCHK(hipGetLastError());
        c->st.launches++;
      }
      bh.clear();
      bd.clear();
      bl.clear();
    };
    for (int i = 0; i < n; i++)
      if (P.s(i, t) < P.en(i, t) && loop_nonempty(L[i], c->ndim)) {
        if (fuse && L[i].kid == OOC_K_MIRROR) {
          bool ok = true;
          for (int q : bl) ok = ok && loops_independent(L[q], L[i], c->ndim);
          if (!ok) flush_batch();
          bh.push_back(&hostargs[li]);
          bd.push_back(c->argtab_dev + abase + li);
          bl.push_back(i);
        } else {
          flush_batch();
          launch_loop(c, launches[li].kid, hostargs[li], c->argtab_dev + abase + li, launches[li].bytes);
        }
        li++;
      }
    flush_batch();
    if (c->tile_timing && c->capture_g0 < 0) tile_mark(c, 3, c->s_comp);
    // ---- hand the right edge to the next tile's slot (on the compute stream)
    const bool poison = (c->flags & OOC_FLAG_DEBUG_POISON) != 0;
    if (!P.ring && t + 1 < T && (poison || !edge[t + 1].empty())) {
      wait_tile(c, c->s_comp, c->ev_down, g + 1 - S);  // next slot free again
      char *nslot = c->slot_base + (uint64_t)((g + 1) % S) * c->slot_stride;
      if (poison) launch_fill((double *)nslot, P.slot_bytes / 8, NAN, c->s_comp);
      std::vector<CopySeg> segs;
      for (const Run *r : edge[t + 1]) {
        Field &f = c->fields[r->f];
        const int64_t A0 = P.resA[(size_t)r->f * T + t], A1 = P.resA[(size_t)r->f * T + t + 1];
        CopySeg s;
        s.src = (const double *)(slot + P.slab_off[r->f] + (r->lo - A0) * f.row_bytes_dev());
        s.dst = (double *)(nslot + P.slab_off[r->f] + (r->lo - A1) * f.row_bytes_dev());
        s.n = (r->hi - r->lo) * f.row_elems;
        segs.push_back(s);
      }
      launch_copy_segments(segs.data(), (int)segs.size(), c->s_comp);
      HIPCHK(hipGetLastError());
    }
    if (t == T - 1) {
      for (int h : wreds) {
        Reduction &r = c->reds[h];
        if (r.op == OOC_RED_SUM) launch_sum_finalize(r.partials, r.npartials, r.committed, c->s_comp);
        else launch_red_commit(r.acc, r.committed, c->s_comp);
      }
    }
    if (c->tile_timing && c->capture_g0 < 0) tile_mark(c, 4, c->s_comp);
    timed_call(c, [&] { HIPCHK(hipEventRecord(evref(c->ev_comp, c, g), c->s_comp)); }, kCallRecord);
    if (dbg_sync) HIPCHK(hipStreamSynchronize(c->s_comp));
    // ---- download: the written rows this tile holds that the next tile
    // does not take over (Algorithm 1's download stage)
    timed_call(c, [&] { HIPCHK(hipStreamWaitEvent(c->s_down, evref(c->ev_comp, c, g), 0)); }, kCallWait);
    if (c->tile_timing && c->capture_g0 < 0) tile_mark(c, 5, c->s_down);
    std::vector<XferSeg> xdown;
    for (const Run *r : down[t]) {
      Field &f = c->fields[r->f];
      const char *src = row_ptr(c, P, r->f, t, slot, r->lo);
      const size_t nb = (size_t)(r->hi - r->lo) * f.row_bytes_host();
      char *dst = (char *)f.host + r->lo * f.row_bytes_host();
      // Downloads go by copy kernel into the device-mapped host rows unless
      // the context asks for runtime memcpy calls.  On link-bound chains the
      // kernel keeps the higher rate (hydro2d 15360^2: 240 against 261 ms
      // per step in FP64, 100 against 173 ms in FP32; hydro3d 640^3 FP32:
      // 172 against 248 ms); on kernel-bound ones its host stores slow the
      // stencils beside them more than the runtime's copies do (ns3d 512^3
      // on rings: 59 against 73 ms per step).
      if (kcopy || (f.host_dev && !(c->flags & OOC_FLAG_MEMCPY_DOWNLOAD))) {
        if (!f.host_dev) throw DeviceError("kernel copy needs device-mapped pinned host arrays");
        char *hdst = (char *)f.host_dev + r->lo * f.row_bytes_host();
        const int64_t elems = (r->hi - r->lo) * f.row_elems;
        if (f.fp32 && f32_down_mode == 3 && (elems % 4 || (uintptr_t)src % 32 || (uintptr_t)hdst % 16))
          throw DeviceError("float32 download run not aligned for 4-element steps");
        xdown.push_back(f.fp32 ? XferSeg{src, hdst, elems, f32_down_mode}
                               : XferSeg{src, hdst, (int64_t)nb / 16, 0});
        continue;
      }
      if (f.fp32) {  // rounded to float32 (nearest even) in staging, then sent
        char *stage = slot + P.stage_down_off + stage_down;
        launch_f64_to_f32((const double *)src, (float *)stage, (r->hi - r->lo) * f.row_elems, c->s_down);
        timed_call(c, [&] { HIPCHK(hipMemcpyAsync(dst, stage, nb, hipMemcpyDeviceToHost, c->s_down)); }, kCallD2H);
        stage_down += align256(nb);
      } else {
        timed_call(c, [&] { HIPCHK(hipMemcpyAsync(dst, src, nb, hipMemcpyDeviceToHost, c->s_down)); }, kCallD2H);
      }
    }
    if (!xdown.empty()) {
      timed_call(c, [&] { launch_xfer_segments(xdown.data(), (int)xdown.size(), true, narrow_down, c->s_down); },
                 kCallD2H);
      HIPCHK(hipGetLastError());
    }
    if (c->tile_timing && c->capture_g0 < 0) tile_mark(c, 6, c->s_down);
    timed_call(c, [&] { HIPCHK(hipEventRecord(evref(c->ev_down, c, g), c->s_down)); }, kCallRecord);
    if (dbg_sync) HIPCHK(hipStreamSynchronize(c->s_down));
  }
  };  // body

  const bool graph = (c->flags & OOC_FLAG_GRAPH) && !c->timing &&
                     !(c->flags & (OOC_FLAG_DEBUG_POISON | OOC_FLAG_DEBUG_SYNC));
  if (!graph) {
    body();
  } else {
    // The chain runs as one graph launched on the upload stream.  Everything
    // it depends on from earlier chains (compute, reduction commits, the
    // argument-table upload, downloads) is ordered before it.
    for (hipEvent_t *e : {&c->ev_fork, &c->ev_join_c, &c->ev_join_d, &c->ev_pre, &c->ev_post})
      if (!*e) HIPCHK(hipEventCreateWithFlags(e, hipEventDisableTiming));
    HIPCHK(hipEventRecord(c->ev_pre, c->s_comp));
    HIPCHK(hipStreamWaitEvent(c->s_up, c->ev_pre, 0));
    wait_tile(c, c->s_up, c->ev_down, prev_last_tile);
    for (int64_t g = g0; g < g0 + T; g++) {  // create the tile events outside any capture
      (void)evref(c->ev_up, c, g);
      (void)evref(c->ev_comp, c, g);
      (void)evref(c->ev_down, c, g);
    }
    auto it = c->graphs.find(akey);
    if (it != c->graphs.end()) {
      HIPCHK(hipGraphLaunch(it->second.exec, c->s_up));
      c->gtile += T;
      c->st.launches += it->second.launches;
    } else {
      c->capture_g0 = g0;
      HIPCHK(hipStreamBeginCapture(c->s_up, hipStreamCaptureModeThreadLocal));
      HIPCHK(hipEventRecord(c->ev_fork, c->s_up));
      HIPCHK(hipStreamWaitEvent(c->s_comp, c->ev_fork, 0));
      HIPCHK(hipStreamWaitEvent(c->s_down, c->ev_fork, 0));
      hipGraph_t gr = nullptr;
      try {
        body();
        HIPCHK(hipEventRecord(c->ev_join_c, c->s_comp));
        HIPCHK(hipEventRecord(c->ev_join_d, c->s_down));
        HIPCHK(hipStreamWaitEvent(c->s_up, c->ev_join_c, 0));
        HIPCHK(hipStreamWaitEvent(c->s_up, c->ev_join_d, 0));
        HIPCHK(hipStreamEndCapture(c->s_up, &gr));
      } catch (...) {
        c->capture_g0 = -1;
        throw;
      }
      c->capture_g0 = -1;
      hipGraphExec_t ex = nullptr;
      HIPCHK(hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0));
      (void)hipGraphDestroy(gr);
      c->graphs[akey] = {ex, c->st.launches - launches0};
      HIPCHK(hipGraphLaunch(ex, c->s_up));
    }
    // per-tile events for later chains, and the other streams follow the graph
    for (int64_t g = g0; g < g0 + T; g++) {
      HIPCHK(hipEventRecord(evref(c->ev_up, c, g), c->s_up));
      HIPCHK(hipEventRecord(evref(c->ev_comp, c, g), c->s_up));
      HIPCHK(hipEventRecord(evref(c->ev_down, c, g), c->s_up));
    }
    HIPCHK(hipEventRecord(c->ev_post, c->s_up));
    HIPCHK(hipStreamWaitEvent(c->s_comp, c->ev_post, 0));
    HIPCHK(hipStreamWaitEvent(c->s_down, c->ev_post, 0));
  }
  for (const Run &r : P.down)
    for (int64_t q = r.lo; q < r.hi; q++) c->fields[r.f].last_down[q] = g0 + r.t;
  if (P.ring) {
    c->ring_prev_valid = true;
    c->ring_prev_g0 = g0;
    c->ring_prev_T = T;
    c->ring_prev_resA = P.resA;
    c->ring_prev_resB = P.resB;
    c->ring_prev_origin = c->ring_origin;
  }
  // host-copy bookkeeping
  const bool cyclic = (c->flags & OOC_FLAG_CYCLIC) != 0;
  for (size_t f = 0; f < c->fields.size(); f++) {
    Field &fd = c->fields[f];
    if (!P.written[f]) continue;
    if (fd.resident) fd.host_valid = false;
    else fd.stale = cyclic && P.temporary[f];
  }
  c->st.last_issue_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - issue0).count();
  c->st.chains++;
  c->st.tiles += T;
  c->st.bytes_hbm_alg += P.alg_bytes;
  c->st.tile_rows = P.h;
  c->st.ntiles_last = T;
  c->st.slots = S;
  c->st.slot_bytes = P.slot_bytes;
}

void sync_all(ooc_ctx *c) {
  HIPCHK(hipStreamSynchronize(c->s_up));
  HIPCHK(hipStreamSynchronize(c->s_comp));
  HIPCHK(hipStreamSynchronize(c->s_down));
  c->gsynced = c->gtile - 1;
  c->gbase = c->gtile;
}

void collect_timing(ooc_ctx *c) {
  c->st.last_kernel_ms = 0;
  for (const TimedLaunch &t : c->timed) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, t.a, t.b));
    KStat &k = c->kstats[t.kid];
    k.ms += ms;
    k.launches++;
    k.bytes += t.bytes;
    c->st.last_kernel_ms += ms;
  }
  c->timed.clear();
  c->tev_next = 0;
}

// Split the queue into chains and issue them back to back; with wait, block
// until the device has finished everything issued so far.
int flush(ooc_ctx *c, bool wait = true) {
  if (c->flags & OOC_FLAG_PLAN_ONLY) {
    if (c->queue.empty()) return OOC_OK;
    throw ArgError(OOC_E_STATE, "a plan-only context cannot execute");
  }
  if (c->queue.empty()) {
    if (wait && c->ready && c->gtile - 1 > c->gsynced) {
      sync_all(c);
      if (c->timing) collect_timing(c);
      collect_tile_times(c);
    }
    return OOC_OK;
  }
  setup_device(c);
  auto t0 = std::chrono::steady_clock::now();
  c->st.last_bytes_h2d = c->st.last_bytes_d2h = 0;
  c->st.last_issue_ms = 0;
  std::vector<std::pair<int, int>> chains;
  {
    int start = 0;
    std::vector<int> wr;
    int marks0 = c->queue[0].marks_before;
    for (int i = 0; i < (int)c->queue.size(); i++) {
      const LoopRec &L = c->queue[i];
      bool split = c->chain_steps > 0 && L.marks_before - marks0 >= c->chain_steps;
      for (const ArgRec &g : L.args)
        if ((g.kind == OOC_ARG_DEVSCALAR || g.kind == OOC_ARG_RED) &&
            std::find(wr.begin(), wr.end(), g.handle) != wr.end())
          split = true;
      if (split && i > start) {
        chains.push_back({start, i});
        start = i;
        wr.clear();
        marks0 = L.marks_before;
      }
      for (const ArgRec &g : L.args)
        if (g.kind == OOC_ARG_RED) wr.push_back(g.handle);
    }
    chains.push_back({start, (int)c->queue.size()});
  }
  // a non-blocking submit issues only complete chains: with a chain length
  // set, the trailing chain waits until it has all its step marks
  if (!wait && c->chain_steps > 0) {
    auto &last = chains.back();
    if (c->marks - c->queue[last.first].marks_before < c->chain_steps) chains.pop_back();
    if (chains.empty()) return OOC_OK;
  }
  // Cyclic skips downloads of temporaries, which leaves their host copies
  // stale; a later chain that reads such a field before writing it would read
  // garbage.  Follow the stale state through the chains before issuing any.
  {
    std::vector<char> stale(c->fields.size());
    for (size_t f = 0; f < c->fields.size(); f++) stale[f] = c->fields[f].stale;
    const bool cyclic = (c->flags & OOC_FLAG_CYCLIC) != 0;
    for (auto &ch : chains) {
      const Plan &P = get_plan(c, c->queue.data() + ch.first, ch.second - ch.first);
      for (const Run &r : P.up)
        if (stale[r.f]) {
          c->queue.clear();
          throw ArgError(OOC_E_STALE, "field '" + c->fields[r.f].name +
                                          "' is read before written, but its host copy was skipped as a "
                                          "temporary under Cyclic in an earlier chain");
        }
      for (size_t f = 0; f < c->fields.size(); f++)
        if (P.written[f] && !c->fields[f].resident) stale[f] = cyclic && P.temporary[f];
    }
  }
  for (auto &ch : chains) {
    // The host runs at most one chain ahead of the device: a chain is issued
    // once the one two before it has finished.  (With many chains of
    // runtime-copy downloads queued, the runtime blocked the host inside
    // launches for up to 0.4 s and both link directions slowed: hydro2d
    // 15360^2, 559 against 237 ms per step.)
    if (c->prev2_last_tile > c->gsynced && c->prev2_last_tile >= c->gbase)
      timed_call(c, [&] { HIPCHK(hipEventSynchronize(evref(c->ev_down, c, c->prev2_last_tile))); }, kCallWait);
    run_chain(c, c->queue.data() + ch.first, ch.second - ch.first, c->prev_last_tile);
    c->prev2_last_tile = c->prev_last_tile;
    c->prev_last_tile = c->gtile - 1;
  }
  c->queue.erase(c->queue.begin(), c->queue.begin() + chains.back().second);
  if (std::getenv("OOC_PROFILE_HOST")) {
    const char *nm[kCallN] = {"h2d", "d2h", "launch", "wait", "record", "other"};
    std::fprintf(stderr, "[ooc host] issue %.1f ms:", c->st.last_issue_ms);
    for (int k = 0; k < kCallN; k++) {
      std::fprintf(stderr, " %s %d calls %.1f ms (max %.2f)", nm[k], g_call_n[k], g_call_ms[k], g_call_max[k]);
      g_call_ms[k] = g_call_max[k] = 0;
      g_call_n[k] = 0;
    }
    std::fprintf(stderr, "\n");
  }
  if (!wait) return OOC_OK;
  sync_all(c);
  if (c->timing) collect_timing(c);
  collect_tile_times(c);
  c->st.last_flush_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return OOC_OK;
}

void check_loop(ooc_ctx *c, int kid, const int64_t range[6], int nargs, const ooc_arg *args, LoopRec &L) {
  if (kid <= 0 || kid >= OOC_K_MAX_ID || !table()[kid].launch) throw ArgError(OOC_E_ARG, "unknown kernel id " + std::to_string(kid));
  const KernelInfo &ki = table()[kid];
  if (nargs < 0 || (nargs > 0 && !args)) throw ArgError(OOC_E_ARG, "bad argument list");
  L.kid = kid;
  for (int d = 0; d < 3; d++) {
    L.lo[d] = d < c->ndim ? range[2 * d] : 0;
    L.hi[d] = d < c->ndim ? range[2 * d + 1] : 1;
    if (L.hi[d] < L.lo[d]) throw ArgError(OOC_E_ARG, "negative iteration range on axis " + std::to_string(d));
  }
  const bool empty = !loop_nonempty(L, c->ndim);
  int nd = 0, nc = 0, ndv = 0, nr = 0;
  for (int k = 0; k < nargs; k++) {
    const ooc_arg &a = args[k];
    ArgRec r;
    r.kind = a.kind;
    r.handle = a.handle;
    r.access = a.access;
    r.value = a.value;
    switch (a.kind) {
      case OOC_ARG_DAT: {
        if (a.handle < 0 || a.handle >= (int)c->fields.size()) throw ArgError(OOC_E_ARG, "bad field handle");
        if (a.access < OOC_READ || a.access > OOC_INC) throw ArgError(OOC_E_ARG, "bad access mode");
        if (a.npts < 1 || a.npts > 256 || !a.offsets) throw ArgError(OOC_E_ARG, "bad stencil");
        r.offs.assign((size_t)a.npts * 3, 0);
        for (int p = 0; p < a.npts; p++)
          for (int d = 0; d < c->ndim; d++) r.offs[3 * p + d] = a.offsets[p * c->ndim + d];
        if (writes_access(a.access)) {
          for (int v : r.offs)
            if (v != 0 || a.npts != 1)
              throw ArgError(OOC_E_ARG, "field '" + c->fields[a.handle].name +
                                            "' is written through a stencil other than the point itself");
        }
        const Field &f = c->fields[a.handle];
        if (!empty)
          for (int p = 0; p < a.npts; p++)
            for (int d = 0; d < c->ndim; d++) {
              int64_t o = r.offs[3 * p + d];
              if (L.lo[d] + o < f.lo[d] || L.hi[d] + o > f.lo[d] + f.n[d])
                throw ArgError(OOC_E_ARG, std::string("loop ") + table()[kid].name + " reaches outside field '" +
                                              f.name + "' on axis " + std::to_string(d));
            }
        nd++;
      } break;
      case OOC_ARG_CONST: nc++; break;
      case OOC_ARG_DEVSCALAR:
      case OOC_ARG_RED:
        if (a.handle < 0 || a.handle >= (int)c->reds.size()) throw ArgError(OOC_E_ARG, "bad reduction handle");
        if (a.kind == OOC_ARG_RED) nr++;
        else ndv++;
        break;
      default: throw ArgError(OOC_E_ARG, "bad argument kind");
    }
    L.args.push_back(std::move(r));
  }
  int want_c = ki.nconst < 0 ? nd / 2 : ki.nconst;
  if (nd < ki.ndat_min || nd > ki.ndat_max || nc != want_c || ndv != ki.ndev || nr != ki.nred ||
      (ki.nconst < 0 && nd % 2))
    throw ArgError(OOC_E_ARG, std::string("argument list does not match kernel ") + ki.name);
  // points are order-free: a written field may be read elsewhere only where
  // the shifted range cannot meet the written range
  for (size_t w = 0; w < L.args.size(); w++) {
    const ArgRec &aw = L.args[w];
    if (aw.kind != OOC_ARG_DAT || !writes_access(aw.access)) continue;
    for (size_t r = 0; r < L.args.size(); r++) {
      const ArgRec &ar = L.args[r];
      if (ar.kind != OOC_ARG_DAT || ar.handle != aw.handle) continue;
      if (r != w && writes_access(ar.access)) throw ArgError(OOC_E_ARG, "field written twice by one loop");
      if (!reads_access(ar.access)) continue;
      for (int p = 0; p < ar.npts(); p++) {
        bool zero = true, disjoint = false;
        for (int d = 0; d < c->ndim; d++) {
          int64_t o = ar.offs[3 * p + d];
          if (o) zero = false;
          if (L.lo[d] + o >= L.hi[d] || L.hi[d] + o <= L.lo[d]) disjoint = true;
        }
        if (!zero && !disjoint && !empty)
          throw ArgError(OOC_E_ARG, "loop reads field '" + c->fields[aw.handle].name +
                                        "' at a neighbour it also writes (points would not be order-free)");
      }
    }
  }
}

}  // namespace

// ======================================================================= ABI
extern "C" {

int ooc_create(ooc_ctx **out, int ndim, const int64_t dims[3], int halo, size_t budget, uint32_t flags) {
  if (!out || (ndim != 2 && ndim != 3) || !dims || halo < 0 || halo > 8) return OOC_E_ARG;
  if (flags & OOC_FLAG_GRAPH) return OOC_E_ARG;  // switched off: see ooc_set_flags
  for (int d = 0; d < ndim; d++)
    if (dims[d] < 1 || dims[d] > (1 << 24)) return OOC_E_ARG;
  ooc_ctx *c = new (std::nothrow) ooc_ctx();
  if (!c) return OOC_E_NOMEM;
  c->ndim = ndim;
  c->tax = ndim - 1;
  c->halo = halo;
  for (int d = 0; d < 3; d++) c->dims[d] = d < ndim ? dims[d] : 1;
  c->budget = budget;
  c->flags = flags;
  c->pitch = (kXOrigin + dims[0] + halo + 1 + 31) / 32 * 32;
  c->plane = ndim == 3 ? c->pitch * (dims[1] + 2 * halo + 1) : 0;
  *out = c;
  return OOC_OK;
}

int ooc_bind_device(ooc_ctx *c, void *arena, size_t arena_bytes, void *s_up, void *s_comp, void *s_down) {
  GUARD(c);
  if (c->ready || c->bound) return fail(c, OOC_E_STATE, "device already bound");
  const bool no_arena = !arena && arena_bytes == 0 && (c->flags & OOC_FLAG_RING);
  if ((!arena && !no_arena) || (uintptr_t)arena % 256 || !s_up || !s_comp || !s_down)
    return fail(c, OOC_E_ARG, "arena must be 256-byte aligned and all three streams given");
  if (s_up == s_comp || s_up == s_down || s_comp == s_down)
    return fail(c, OOC_E_ARG, "the three streams must be distinct");
  c->arena = (char *)arena;
  c->arena_bytes = arena_bytes;
  c->s_up = (hipStream_t)s_up;
  c->s_comp = (hipStream_t)s_comp;
  c->s_down = (hipStream_t)s_down;
  c->bound = true;
  return OOC_OK;
}

int ooc_decl_field(ooc_ctx *c, const char *name, const int32_t size_delta[3], const double *init, uint32_t fflags,
                   ooc_field *out) {
  GUARD(c);
  if (!out) return OOC_E_ARG;
  if (c->ready) return fail(c, OOC_E_STATE, "fields must be declared before the first flush");
  return guarded(c, [&]() -> int {
    Field f;
    f.name = name ? name : ("field" + std::to_string(c->fields.size()));
    for (int d = 0; d < 3; d++) {
      f.delta[d] = size_delta && d < c->ndim ? size_delta[d] : 0;
      if (f.delta[d] < 0 || f.delta[d] > 1) throw ArgError(OOC_E_ARG, "size_delta must be 0 or 1");
    }
    f.resident = (fflags & OOC_FIELD_RESIDENT) || (c->flags & OOC_FLAG_INCORE);
    f.fp32 = (c->flags & OOC_FLAG_FP32_STREAM) && !f.resident;
    layout_field(c, f);
    bool pin = false;
    const bool plan_only = (c->flags & OOC_FLAG_PLAN_ONLY) != 0;
    if (!plan_only) {
      f.host = alloc_host(c, f.host_bytes(), pin);
      if (!f.host) throw std::bad_alloc();
      par_memcpy(f.host, nullptr, f.host_bytes());
    }
    f.last_down.assign(f.nrows, -1);
    if (pin) map_host(f);
    c->fields.push_back(std::move(f));
    c->pinned.push_back(pin);
    Field &fr = c->fields.back();
    if (init && !plan_only) copy_extent(c, fr, nullptr, init, false);
    *out = (ooc_field)(c->fields.size() - 1);
    return OOC_OK;
  });
}

int ooc_decl_reduction(ooc_ctx *c, int op, ooc_red *out) {
  GUARD(c);
  if (!out || op < OOC_RED_MIN || op > OOC_RED_SUM) return OOC_E_ARG;
  if (c->ready) return fail(c, OOC_E_STATE, "reductions must be declared before the first flush");
  Reduction r;
  r.op = op;
  c->reds.push_back(r);
  *out = (ooc_red)(c->reds.size() - 1);
  return OOC_OK;
}

int ooc_set_reduction(ooc_ctx *c, ooc_red h, double v) {
  GUARD(c);
  if (h < 0 || h >= (int)c->reds.size()) return OOC_E_ARG;
  return guarded(c, [&]() -> int {
    Reduction &r = c->reds[h];
    if (!c->ready) {
      r.host_value = v;
      r.host_set = true;
      return OOC_OK;
    }
    int rc = flush(c);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(r.committed, &v, 8, hipMemcpyHostToDevice, c->s_comp));
    HIPCHK(hipStreamSynchronize(c->s_comp));
    return OOC_OK;
  });
}

int ooc_par_loop(ooc_ctx *c, int kid, const int64_t range[6], int nargs, const ooc_arg *args) {
  GUARD(c);
  if (!range) return OOC_E_ARG;
  return guarded(c, [&]() -> int {
    LoopRec L;
    check_loop(c, kid, range, nargs, args, L);
    L.marks_before = c->marks;
    c->queue.push_back(std::move(L));
    return OOC_OK;
  });
}

int ooc_discard_queue(ooc_ctx *c) {
  GUARD(c);
  c->queue.clear();
  return OOC_OK;
}

int ooc_mark_step(ooc_ctx *c) {
  GUARD(c);
  c->marks++;
  return OOC_OK;
}

int ooc_execute(ooc_ctx *c) {
  GUARD(c);
  return guarded(c, [&]() -> int { return flush(c); });
}

int ooc_submit(ooc_ctx *c) {
  GUARD(c);
  return guarded(c, [&]() -> int { return flush(c, false); });
}

int ooc_reduce(ooc_ctx *c, ooc_red h, double *out) {
  GUARD(c);
  if (h < 0 || h >= (int)c->reds.size() || !out) return OOC_E_ARG;
  return guarded(c, [&]() -> int {
    int rc = flush(c);
    if (rc) return rc;
    if (!c->ready) {
      *out = c->reds[h].host_value;
      return OOC_OK;
    }
    HIPCHK(hipMemcpy(out, c->reds[h].committed, 8, hipMemcpyDeviceToHost));
    return OOC_OK;
  });
}

int ooc_fetch_field(ooc_ctx *c, ooc_field h, double *dst, size_t bytes) {
  GUARD(c);
  if (h < 0 || h >= (int)c->fields.size() || !dst) return OOC_E_ARG;
  return guarded(c, [&]() -> int {
    Field &f = c->fields[h];
    if (bytes != (size_t)(f.n[0] * f.n[1] * f.n[2] * 8)) throw ArgError(OOC_E_ARG, "size mismatch");
    if (!f.host) throw ArgError(OOC_E_STATE, "plan-only context has no field data");
    int rc = flush(c);
    if (rc) return rc;
    if (f.resident && c->ready && !f.host_valid) {
      HIPCHK(hipMemcpy(f.host, f.dev_res, (size_t)f.nrows * f.row_elems * 8, hipMemcpyDeviceToHost));
      f.host_valid = true;
    }
    if (f.stale) throw ArgError(OOC_E_STALE, "field '" + f.name + "' is a temporary not downloaded (Cyclic)");
    copy_extent(c, f, dst, nullptr, true);
    return OOC_OK;
  });
}

int ooc_set_field(ooc_ctx *c, ooc_field h, const double *src, size_t bytes) {
  GUARD(c);
  if (h < 0 || h >= (int)c->fields.size() || !src) return OOC_E_ARG;
  return guarded(c, [&]() -> int {
    Field &f = c->fields[h];
    if (bytes != (size_t)(f.n[0] * f.n[1] * f.n[2] * 8)) throw ArgError(OOC_E_ARG, "size mismatch");
    if (!f.host) throw ArgError(OOC_E_STATE, "plan-only context has no field data");
    int rc = flush(c);
    if (rc) return rc;
    copy_extent(c, f, nullptr, src, false);
    f.stale = false;
    if (f.resident && c->ready) {
      HIPCHK(hipMemcpy(f.dev_res, f.host, (size_t)f.nrows * f.row_elems * 8, hipMemcpyHostToDevice));
      f.host_valid = true;
    }
    return OOC_OK;
  });
}

int ooc_set_flags(ooc_ctx *c, uint32_t set, uint32_t clear) {
  GUARD(c);
  const uint32_t fixed = OOC_FLAG_FP32_STREAM | OOC_FLAG_INCORE | OOC_FLAG_PLAN_ONLY | OOC_FLAG_RING;
  if ((set | clear) & fixed) return fail(c, OOC_E_STATE, "FP32_STREAM, INCORE and RING are fixed at creation");
  // Chain replay from a stream-captured graph is switched off: its first
  // capture ended the process with a host segmentation fault whose cause has
  // not been found in this library's code.
  if (set & OOC_FLAG_GRAPH) return fail(c, OOC_E_ARG, "OOC_FLAG_GRAPH is switched off in this version");
  return guarded(c, [&]() -> int {
    int rc = flush(c);  // flags apply to chains queued from now on
    if (rc) return rc;
    c->flags = (c->flags | set) & ~clear;
    return OOC_OK;
  });
}

int ooc_set_schedule(ooc_ctx *c, int64_t tile_rows, int chain_steps, int slots) {
  GUARD(c);
  if (tile_rows < 0 || chain_steps < 0 || slots < 0 || slots == 1 || slots > 8) return OOC_E_ARG;
  return guarded(c, [&]() -> int {
    int rc = flush(c);
    if (rc) return rc;
    const int s = slots ? slots : 3;
    if (c->ready && s != c->slots && !(c->flags & OOC_FLAG_RING)) {
      const uint64_t base = (uint64_t)(c->slot_base - c->arena);
      const size_t budget = std::min(c->budget, c->arena_bytes);
      c->slot_stride = (budget - base) / s / 256 * 256;
    }
    c->tile_rows = tile_rows;
    c->chain_steps = chain_steps;
    c->slots = s;
    c->plans.clear();
    return OOC_OK;
  });
}

int ooc_get_layout(ooc_ctx *c, int64_t *pitch, int64_t *plane, int64_t *x_origin) {
  if (!c || !pitch || !plane || !x_origin) return OOC_E_ARG;
  *pitch = c->pitch;
  *plane = c->plane;
  *x_origin = kXOrigin;
  return OOC_OK;
}

int ooc_get_stats(ooc_ctx *c, ooc_stats *out) {
  if (!c || !out) return OOC_E_ARG;
  *out = c->st;
  return OOC_OK;
}

int ooc_set_timing(ooc_ctx *c, int on) {
  GUARD(c);
  if (on < 0 || on >= 2 + OOC_K_MAX_ID) return fail(c, OOC_E_ARG, "timing mode out of range");
  c->timing = on != 0;  // read when loops are issued
  c->timing_kid = on >= 2 ? on - 2 : -1;
  c->kstats.clear();
  c->st.max_call_ms = 0;
  c->st.max_call_kind = 0;
  c->st.max_call_chain = 0;
  return OOC_OK;
}

int ooc_set_tile_timing(ooc_ctx *c, int on) {
  GUARD(c);
  c->tile_timing = on != 0;
  return OOC_OK;
}

int ooc_tile_times(ooc_ctx *c, ooc_tile_time *out, int capacity, int *count) {
  if (!c || !count || capacity < 0) return OOC_E_ARG;
  *count = (int)c->tile_times.size();
  if (out)
    for (int i = 0; i < capacity && i < *count; i++) out[i] = c->tile_times[i];
  return OOC_OK;
}

int ooc_kernel_stats(ooc_ctx *c, int kid, double *ms, uint64_t *launches, uint64_t *bytes) {
  if (!c) return OOC_E_ARG;
  auto it = c->kstats.find(kid);
  KStat k = it == c->kstats.end() ? KStat() : it->second;
  if (ms) *ms = k.ms;
  if (launches) *launches = k.launches;
  if (bytes) *bytes = k.bytes;
  return OOC_OK;
}

const char *ooc_last_error(ooc_ctx *c) { return c ? c->err.c_str() : "null context"; }

int ooc_debug_fail_after(ooc_ctx *c, int64_t n) {
  GUARD(c);
  if (n < 0) return fail(c, OOC_E_ARG, "negative call count");
  c->fail_after = n;
  return OOC_OK;
}

int ooc_destroy(ooc_ctx *c) {
  if (!c) return OOC_E_ARG;
  // Work issued before a failure may still read the pinned host arrays and
  // the argument table: wait for all three streams in every case (a failed
  // stream returns an error, which is ignored) before anything is freed.
  if (c->bound) {
    for (hipStream_t s : {c->s_up, c->s_comp, c->s_down})
      if (s) (void)hipStreamSynchronize(s);
    (void)hipGetLastError();
  }
  for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.second.exec);
  for (hipEvent_t e : {c->ev_fork, c->ev_join_c, c->ev_join_d, c->ev_pre, c->ev_post})
    if (e) (void)hipEventDestroy(e);
  for (auto *v : {&c->ev_up, &c->ev_comp, &c->ev_down, &c->tev_pool, &c->tile_pool})
    for (hipEvent_t e : *v) (void)hipEventDestroy(e);
  for (size_t k = 0; k < c->fields.size(); k++) free_host(c->fields[k].host, c->pinned[k]);
  if (c->argtab_host) free_host(c->argtab_host, true);
  if (c->argtab_dev) (void)hipFree(c->argtab_dev);
  free_rings(c);
  if (c->own_streams) {
    (void)hipStreamDestroy(c->s_up);
    (void)hipStreamDestroy(c->s_comp);
    (void)hipStreamDestroy(c->s_down);
  }
  if (c->own_arena) (void)hipFree(c->arena);
  delete c;
  return OOC_OK;
}

int ooc_field_shape(ooc_ctx *c, ooc_field h, int64_t lo[3], int64_t n[3]) {
  if (!c || h < 0 || h >= (int)c->fields.size()) return OOC_E_ARG;
  for (int d = 0; d < 3; d++) {
    if (lo) lo[d] = c->fields[h].lo[d];
    if (n) n[d] = c->fields[h].n[d];
  }
  return OOC_OK;
}

int ooc_debug_plan(ooc_ctx *c, ooc_plan_info *out) {
  GUARD(c);
  if (!out) return OOC_E_ARG;
  return guarded(c, [&]() -> int {
    if (c->queue.empty()) throw ArgError(OOC_E_STATE, "nothing queued");
    // the first chain of the queue, split as a flush would split it
    int end = (int)c->queue.size();
    {
      std::vector<int> wr;
      int marks0 = c->queue[0].marks_before;
      for (int i = 0; i < (int)c->queue.size(); i++) {
        const LoopRec &L = c->queue[i];
        bool split = c->chain_steps > 0 && L.marks_before - marks0 >= c->chain_steps;
        for (const ArgRec &g : L.args)
          if ((g.kind == OOC_ARG_DEVSCALAR || g.kind == OOC_ARG_RED) &&
              std::find(wr.begin(), wr.end(), g.handle) != wr.end())
            split = true;
        if (split && i > 0) {
          end = i;
          break;
        }
        for (const ArgRec &g : L.args)
          if (g.kind == OOC_ARG_RED) wr.push_back(g.handle);
      }
    }
    c->dbg = get_plan(c, c->queue.data(), end);
    const Plan &P = c->dbg;
    const int nf = (int)c->fields.size();
    c->dbg_loop_rows.assign((size_t)P.nloops * P.T * 2, 0);
    for (int i = 0; i < P.nloops; i++)
      for (int t = 0; t < P.T; t++) {
        c->dbg_loop_rows[((size_t)i * P.T + t) * 2] = P.s(i, t);
        c->dbg_loop_rows[((size_t)i * P.T + t) * 2 + 1] = P.en(i, t);
      }
    c->dbg_res.assign((size_t)nf * P.T * 2, 0);
    for (int f : P.slot_fields)
      for (int t = 0; t < P.T; t++) {
        c->dbg_res[((size_t)f * P.T + t) * 2] = P.resA[(size_t)f * P.T + t];
        c->dbg_res[((size_t)f * P.T + t) * 2 + 1] = P.resB[(size_t)f * P.T + t];
      }
    auto pack = [](const std::vector<Run> &v, std::vector<int64_t> &o) {
      o.clear();
      for (const Run &r : v) o.insert(o.end(), {r.f, r.t, r.lo, r.hi});
    };
    pack(P.up, c->dbg_up);
    pack(P.down, c->dbg_down);
    pack(P.edge, c->dbg_edge);
    out->ntiles = P.T;
    out->nloops = P.nloops;
    out->nfields = nf;
    out->slots = c->slots;
    out->tile_rows = P.h;
    out->slot_bytes = P.slot_bytes;
    out->loop_rows = c->dbg_loop_rows.data();
    out->resident = c->dbg_res.data();
    out->nup = (int)P.up.size();
    out->ndown = (int)P.down.size();
    out->nedge = (int)P.edge.size();
    out->up = c->dbg_up.data();
    out->down = c->dbg_down.data();
    out->edge = c->dbg_edge.data();
    out->temporary = P.temporary.data();
    c->dbg_ring.assign(nf, 0);
    if (P.ring)
      for (int f : P.slot_fields) c->dbg_ring[f] = P.ring_rows[f];
    out->ring = P.ring ? 1 : 0;
    out->ring_rows = c->dbg_ring.data();
    return OOC_OK;
  });
}

}  // extern "C"
