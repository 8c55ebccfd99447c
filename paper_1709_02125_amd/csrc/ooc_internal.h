// Internal types of the out-of-core loop-chain runtime.  Host-only parts (queue,
// planner) use no HIP; the device parts include hip_runtime.h themselves.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ooc.h"
#include "../../include/ooc_kernels.h"

namespace ooc {

constexpr int kMaxDat = 32;
constexpr int kMaxConst = 12;
constexpr int kMaxDev = 2;
constexpr int kMaxRed = 5;
constexpr int kMaxStencil = 32;
// storage element of x = 0 within every field row (a multiple of 16 elements)
constexpr int64_t kXOrigin = 16;

// Argument block handed by value to every kernel.  Field pointers are rebased
// so that logical index (i, j[, k]) of a field is p[k*plane + j*pitch + i]
// whether the field lives in a tile slot or is resident (the "adjust base
// pointers for virtual position" step of Algorithm 1).
struct KArgs {
  double *p[kMaxDat];
  int32_t off[kMaxDat][3];         // first stencil point of each DAT argument
  double c[kMaxConst];             // CONST arguments in order
  const double *ds[kMaxDev];       // DEVSCALAR arguments: committed reduction values
  double *red[kMaxRed];            // MIN/MAX: accumulator; SUM: per-row partial array
  int32_t st[kMaxStencil][3];      // full stencil of the second DAT argument
  int32_t nst;
  int32_t ndat;
  int32_t lo[3], hi[3];            // launch range (tiled axis already cut to the tile)
  int64_t pitch, plane;            // elements between y rows / z planes
  int64_t red_rows;                // SUM partials: rows per z plane (3D) ; row index base
  int32_t halo;
};

// Kernel launch shapes.
enum Shape { kPointGrid = 0, kRowReduce = 1 };

struct KernelInfo {
  const char *name = nullptr;
  int ndat_min = 0, ndat_max = 0;  // DAT arguments
  int nconst = 0;                  // -1: equals ndat / 2 (MIRROR)
  int ndev = 0, nred = 0;
  int shape = kPointGrid;
  // host copy (for the grid shape) and device copy (what the kernel reads)
  void (*launch)(const KArgs &, const KArgs *dev, int ndim, void *stream) = nullptr;
};

// Registry filled by the kernel translation units.
KernelInfo *kernel_table();
void register_common_kernels(KernelInfo *t);
void register_hydro2d_kernels(KernelInfo *t);
void register_ns3d_kernels(KernelInfo *t);
void register_hydro3d_kernels(KernelInfo *t);

// Device helpers implemented in kernels_common.hip.
struct CopySeg {
  const double *src;
  double *dst;
  int64_t n;  // doubles
};
void launch_copy_segments(const CopySeg *segs, int nseg, void *stream);
// independent mirror loops of one tile in one launch (host and device argument blocks)
void launch_mirror_batch(const KArgs *const *host_args, const KArgs *const *dev_args, int n, int ndim,
                         void *stream);
void launch_fill(double *dst, int64_t n, double value, void *stream);
// host-link transfer by kernel: mode 0 copies n 16-byte units, mode 1 widens
// n float32 to float64, mode 2 rounds n float64 to float32 with 8-byte stores
// (n even), mode 3 the same with 16-byte stores (n a multiple of 4, source
// 32-byte and destination 16-byte aligned)
struct XferSeg {
  const void *src;
  void *dst;
  int64_t n;
  int mode;
};
// to_host: the copy writes host memory (device-to-host), which takes a smaller grid
// to_host: writing host memory (downloads); narrow: the smallest grid for that
// direction, for chains whose downloads are well under their uploads
void launch_xfer_segments(const XferSeg *segs, int nseg, bool to_host, bool narrow, void *stream);
void launch_red_init(double *acc, double value, void *stream);
void launch_red_commit(const double *acc, double *committed, void *stream);
void launch_sum_finalize(const double *partials, int64_t n, double *committed, void *stream);
void launch_f32_to_f64(const float *src, double *dst, int64_t n, void *stream);
void launch_f64_to_f32(const double *src, float *dst, int64_t n, void *stream);

// ------------------------------------------------------------------ queue
struct ArgRec {
  int kind = 0, handle = -1, access = 0;
  std::vector<int32_t> offs;  // npts * 3
  double value = 0.0;
  int npts() const { return (int)offs.size() / 3; }
};

struct LoopRec {
  int kid = 0;
  int64_t lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
  std::vector<ArgRec> args;
  int marks_before = 0;  // step marks queued before this loop (cumulative)
};

struct Field {
  std::string name;
  int32_t delta[3] = {0, 0, 0};
  int64_t lo[3] = {0, 0, 0}, n[3] = {1, 1, 1};  // logical lower bound and extent
  int64_t nrows = 0;                             // extent along the tiled axis
  int64_t row_elems = 0;                         // elements per stored row
  bool resident = false;
  bool fp32 = false;        // host storage in float32
  void *host = nullptr;     // pinned host array (nrows * row_elems elements)
  void *host_dev = nullptr; // the same array as the device addresses it (pinned only)
  double *dev_res = nullptr;
  bool dev_valid = false;   // resident: device copy initialised
  bool host_valid = true;   // resident: host copy up to date
  bool stale = false;       // temporary whose download was skipped (Cyclic)
  std::vector<int64_t> last_down;  // per stored row: tile id of its last download (-1: none)
  int64_t host_bytes() const { return nrows * row_elems * (fp32 ? 4 : 8); }
  int64_t row_bytes_dev() const { return row_elems * 8; }
  int64_t row_bytes_host() const { return row_elems * (fp32 ? 4 : 8); }
};

struct Reduction {
  int op = OOC_RED_MIN;
  double *acc = nullptr;        // device accumulator (MIN/MAX)
  double *partials = nullptr;   // device per-row partials (SUM)
  int64_t npartials = 0;
  double *committed = nullptr;  // device committed value
  double host_value = 0.0;      // value set from the host before the first bind
  bool host_set = false;
};

// --------------------------------------------------------------- planning
struct Run {
  int f, t;
  int64_t lo, hi;  // stored rows
};

struct Plan {
  int T = 1, S = 3;
  int64_t h = 0;
  int nloops = 0;
  std::vector<int64_t> lo, hi;    // per loop, tiled-axis logical range
  std::vector<int64_t> e;         // [nloops][T] exclusive end row of loop i in tile t
  std::vector<int> slot_fields;   // fields stored in the slots
  std::vector<int64_t> resA, resB;  // [nfields][T] stored-row residency
  std::vector<int64_t> cap;         // [nfields] slab rows
  std::vector<uint64_t> slab_off;   // [nfields] byte offset of the slab inside a slot
  // ring slabs (PlanInput::ring): per field one ring of ring_rows rows in
  // ring_bytes (a multiple of the ring granule), then S staging areas of
  // stage_bytes; slot_bytes is then the whole: rings plus staging
  bool ring = false;
  std::vector<int64_t> ring_rows;   // [nfields]
  std::vector<uint64_t> ring_bytes; // [nfields]
  uint64_t stage_bytes = 0;
  uint64_t slot_bytes = 0;
  uint64_t stage_up_off = 0, stage_down_off = 0;  // float32 staging inside a slot
  std::vector<Run> up, down, edge;
  std::vector<int> temporary;       // [nfields]
  std::vector<int> written;         // [nfields] written anywhere in the chain
  uint64_t alg_bytes = 0;           // Section 5.1 byte count of the chain
  std::vector<uint64_t> loop_alg_bytes;
  int64_t s(int i, int t) const { return t == 0 ? lo[i] : e[i * T + t - 1]; }
  int64_t en(int i, int t) const { return e[i * T + t]; }
};

struct PlanInput {
  int ndim = 2, tax = 1, halo = 2;
  const std::vector<Field> *fields = nullptr;
  const LoopRec *loops = nullptr;
  int nloops = 0;
  bool cyclic = false;
  int S = 3;
  int64_t forced_h = 0;
  uint64_t slot_capacity = 0;  // bytes available to one slot (ring: to all rings and staging)
  bool ring = false;           // ring slabs instead of slots
  uint64_t ring_granule = 1u << 16;  // rings are sized in multiples of this
};

// Ring slabs: every streamed field lives in one ring of device memory mapped
// twice at consecutive virtual addresses, so a tile's rows are contiguous
// wherever they wrap; rings are sized in whole units of at least this many
// bytes (and of the device's mapping granularity).
constexpr uint64_t kRingGranule = 1u << 16;

inline bool writes_access(int a) { return a == OOC_WRITE || a == OOC_RW || a == OOC_INC; }
inline bool reads_access(int a) { return a == OOC_READ || a == OOC_RW || a == OOC_INC; }

// Returns OOC_OK or OOC_E_BUDGET; fills plan.
int make_plan(const PlanInput &in, Plan &plan, std::string &err);

// Ring slabs across consecutive chains.  Rows do not stay in the rings from
// one chain to the next, so each chain may place its rows anywhere: row r of
// field f sits at byte (r * row bytes + origin[f]) mod ring bytes.  For the
// next chain the origins can be chosen -- the same fraction q / kRingOrigins
// of every ring -- so that its first tiles take ring positions that the
// previous chain's last tiles no longer hold; each of its first tiles then
// waits only for the downloads of the previous chain's tiles it overlaps
// (Prefetch, paper Section 4.1), not for the previous chain's last download.
// One origin is used: with eight, some chains ran every download at a
// quarter of the link rate (ns3d 512^3 over 16 chains: 71.8 against 56.6 ms
// per step; the cause was not found), for a gain of 1-3 % in the other
// chains.  The waits are still computed per tile for that origin.
constexpr int kRingOrigins = 1;

// The rows each tile of one chain holds, and where they sit in the rings.
struct RingChain {
  int T = 0;
  const int64_t *resA = nullptr, *resB = nullptr;  // [f * T + t]: held rows [resA, resB)
  const uint64_t *origin = nullptr;                 // per field, bytes
};

// nf fields; ring_bytes[f] (0: the field has no ring) and row_bytes[f].
// Fills origin_out[f] for `next` (its own origin is not read) and, for each
// of next's first S tiles t, wait_out[t]: the last tile of `prev` (index in
// that chain, -1: none) whose ring positions tile t's rows overlap, whose
// download must end before tile t's uploads begin.
void choose_ring_origins(int nf, const uint64_t *ring_bytes, const uint64_t *row_bytes, const RingChain &prev,
                         const RingChain &next, int S, uint64_t *origin_out, int64_t *wait_out);

}  // namespace ooc
