// Loop-chain analysis and tile planning (host only, no HIP).
//
// Given a chain of queued loops (Section 3: lazily queued parallel loops with
// per-argument stencils and access modes) this file computes
//   1. the skewed tiling: for every loop and tile, the rows of the tiled axis
//      that loop executes in that tile, such that every read-after-write,
//      write-after-read and write-after-write dependence between loops is kept
//      and every loop's range is partitioned exactly (no redundant compute);
//   2. per dataset and tile the "full footprint" and the rows held in the
//      tile's slot, from which the left/right edges and the left/right
//      footprints of Section 4 (Figure 2) follow;
//   3. which rows have to be uploaded (read before written) and downloaded
//      (modified) -- the read-only / write-first optimisation of Section 4.1,
//      done per row and element-exact -- and the Cyclic variant that also
//      skips downloads of write-first (temporary) datasets;
//   4. the slot layout and the largest tile height whose S slots fit the
//      device budget (Section 4: tile size set from the fast-memory size).
#include <algorithm>
#include <climits>
#include <map>

#include "ooc_internal.h"

namespace ooc {
namespace {

struct Box {
  int64_t x0, x1, y0, y1;
  bool empty() const { return x0 >= x1 || y0 >= y1; }
};

bool box_contains(const Box &a, const Box &b) {
  return a.x0 <= b.x0 && a.x1 >= b.x1 && a.y0 <= b.y0 && a.y1 >= b.y1;
}

// Is q covered by the union of ws?  Exact, by coordinate compression of the
// box edges that fall inside q.
bool covered(const Box &q, const std::vector<Box> &ws) {
  if (q.empty()) return true;
  for (const Box &w : ws)
    if (box_contains(w, q)) return true;
  std::vector<int64_t> xs{q.x0, q.x1}, ys{q.y0, q.y1};
  for (const Box &w : ws) {
    if (w.x1 <= q.x0 || w.x0 >= q.x1 || w.y1 <= q.y0 || w.y0 >= q.y1) continue;
    xs.push_back(std::clamp(w.x0, q.x0, q.x1));
    xs.push_back(std::clamp(w.x1, q.x0, q.x1));
    ys.push_back(std::clamp(w.y0, q.y0, q.y1));
    ys.push_back(std::clamp(w.y1, q.y0, q.y1));
  }
  std::sort(xs.begin(), xs.end());
  xs.erase(std::unique(xs.begin(), xs.end()), xs.end());
  std::sort(ys.begin(), ys.end());
  ys.erase(std::unique(ys.begin(), ys.end()), ys.end());
  for (size_t a = 0; a + 1 < xs.size(); a++)
    for (size_t b = 0; b + 1 < ys.size(); b++) {
      Box cell{xs[a], xs[a + 1], ys[b], ys[b + 1]};
      bool hit = false;
      for (const Box &w : ws)
        if (box_contains(w, cell)) { hit = true; break; }
      if (!hit) return false;
    }
  return true;
}

// Per loop and dataset: how the loop touches the dataset along the tiled axis.
struct Access {
  int f;
  bool r = false, w = false;
  int64_t rmin = INT64_MAX, rmax = INT64_MIN;  // read offsets along the tiled axis
  int64_t fmin() const { return std::min(r ? rmin : INT64_MAX, w ? (int64_t)0 : INT64_MAX); }
  int64_t fmax() const { return std::max(r ? rmax : INT64_MIN, w ? (int64_t)0 : INT64_MIN); }
};

bool reads(int access) { return access == OOC_READ || access == OOC_RW || access == OOC_INC; }
bool writes(int access) { return access == OOC_WRITE || access == OOC_RW || access == OOC_INC; }

// One access event of a dataset, in program order.
struct Event {
  bool write;
  int64_t r0, r1;  // logical rows of the tiled axis
  Box box;         // in-row region (x, and y in 3D)
};

// Do the byte ranges [a, a + la) and [b, b + lb) of a ring of R bytes meet?
// (a, b < R; la, lb <= R)
bool ring_ranges_meet(uint64_t a, uint64_t la, uint64_t b, uint64_t lb, uint64_t R) {
  if (!la || !lb) return false;
  return (b + R - a) % R < la || (a + R - b) % R < lb;
}

}  // namespace

int make_plan(const PlanInput &in, Plan &P, std::string &err) {
  const std::vector<Field> &F = *in.fields;
  const int nf = (int)F.size();
  const int n = in.nloops;
  const int tax = in.tax;
  P = Plan();
  P.S = in.S;
  P.nloops = n;
  P.lo.resize(n);
  P.hi.resize(n);
  P.temporary.assign(nf, 0);
  P.written.assign(nf, 0);
  P.loop_alg_bytes.assign(n, 0);

  std::vector<std::vector<Access>> acc(n);
  std::vector<char> used(nf, 0);
  int64_t L = INT64_MAX, R = INT64_MIN;
  for (int i = 0; i < n; i++) {
    const LoopRec &lp = in.loops[i];
    P.lo[i] = lp.lo[tax];
    P.hi[i] = lp.hi[tax];
    int64_t pts = 1;
    for (int a = 0; a < in.ndim; a++) pts *= std::max<int64_t>(0, lp.hi[a] - lp.lo[a]);
    for (const ArgRec &g : lp.args) {
      if (g.kind != OOC_ARG_DAT) continue;
      P.loop_alg_bytes[i] += (uint64_t)pts * 8u * (g.access == OOC_RW || g.access == OOC_INC ? 2u : 1u);
      Access *a = nullptr;
      for (Access &x : acc[i])
        if (x.f == g.handle) a = &x;
      if (!a) {
        acc[i].push_back(Access{g.handle});
        a = &acc[i].back();
      }
      if (reads(g.access)) {
        a->r = true;
        for (int k = 0; k < g.npts(); k++) {
          a->rmin = std::min<int64_t>(a->rmin, g.offs[3 * k + tax]);
          a->rmax = std::max<int64_t>(a->rmax, g.offs[3 * k + tax]);
        }
      }
      if (writes(g.access)) a->w = true;
      used[g.handle] = 1;
    }
    P.alg_bytes += P.loop_alg_bytes[i];
    if (pts > 0) {
      L = std::min(L, P.lo[i]);
      R = std::max(R, P.hi[i]);
    }
  }
  if (L >= R) {  // nothing to execute
    P.T = 1;
    P.h = 0;
    P.e.assign(n, 0);
    for (int i = 0; i < n; i++) P.e[i] = P.hi[i];
    P.resA.assign(nf, 0);
    P.resB.assign(nf, 0);
    P.cap.assign(nf, 0);
    P.slab_off.assign(nf, 0);
    P.ring = in.ring;
    P.ring_rows.assign(nf, 0);
    P.ring_bytes.assign(nf, 0);
    return OOC_OK;
  }

  // ---- element-exact first-access analysis, in program order.  Because
  // the tiled schedule keeps every dependence, the order of the accesses to
  // any one element is the same as in the untiled program, so this is
  // independent of the tile height.
  std::vector<std::vector<char>> readfirst(nf), written(nf), full(nf);
  for (int f = 0; f < nf; f++) {
    if (!used[f]) continue;
    const Field &fd = F[f];
    std::vector<Event> ev;
    for (int i = 0; i < n; i++) {
      const LoopRec &lp = in.loops[i];
      bool empty = false;
      for (int a = 0; a < in.ndim; a++)
        if (lp.hi[a] <= lp.lo[a]) empty = true;
      if (empty) continue;
      for (int pass = 0; pass < 2; pass++)
        for (const ArgRec &g : lp.args) {
          if (g.kind != OOC_ARG_DAT || g.handle != f) continue;
          if (pass == 0 && reads(g.access)) {
            for (int k = 0; k < g.npts(); k++) {
              const int32_t *o = &g.offs[3 * k];
              Event e{false, lp.lo[tax] + o[tax], lp.hi[tax] + o[tax],
                      Box{lp.lo[0] + o[0], lp.hi[0] + o[0], 0, 1}};
              if (in.ndim == 3) e.box.y0 = lp.lo[1] + o[1], e.box.y1 = lp.hi[1] + o[1];
              ev.push_back(e);
            }
          }
          if (pass == 1 && writes(g.access)) {
            Event e{true, lp.lo[tax], lp.hi[tax], Box{lp.lo[0], lp.hi[0], 0, 1}};
            if (in.ndim == 3) e.box.y0 = lp.lo[1], e.box.y1 = lp.hi[1];
            ev.push_back(e);
          }
        }
    }
    Box whole{fd.lo[0], fd.lo[0] + fd.n[0], 0, 1};
    if (in.ndim == 3) whole.y0 = fd.lo[1], whole.y1 = fd.lo[1] + fd.n[1];
    std::vector<int64_t> bnd;
    for (const Event &e : ev) {
      bnd.push_back(e.r0);
      bnd.push_back(e.r1);
    }
    std::sort(bnd.begin(), bnd.end());
    bnd.erase(std::unique(bnd.begin(), bnd.end()), bnd.end());
    readfirst[f].assign(fd.nrows, 0);
    written[f].assign(fd.nrows, 0);
    full[f].assign(fd.nrows, 0);
    const int64_t rlo = fd.lo[tax];
    bool any_rf = false;
    for (size_t b = 0; b + 1 < bnd.size(); b++) {
      int64_t r0 = bnd[b], r1 = bnd[b + 1];
      std::vector<Box> ws;
      bool rf = false, wr = false;
      for (const Event &e : ev) {
        if (e.r0 > r0 || e.r1 < r1) continue;  // event does not cover this row band
        if (e.write) {
          ws.push_back(e.box);
          wr = true;
        } else if (!rf && !covered(e.box, ws)) {
          rf = true;
        }
      }
      bool fu = wr && covered(whole, ws);
      for (int64_t r = std::max(r0, rlo); r < std::min(r1, rlo + fd.nrows); r++) {
        readfirst[f][r - rlo] = rf;
        written[f][r - rlo] = wr;
        full[f][r - rlo] = fu;
      }
      any_rf |= rf;
      P.written[f] |= wr;
    }
    P.temporary[f] = !any_rf;
  }

  // fields stored in the slots
  for (int f = 0; f < nf; f++)
    if (used[f] && !F[f].resident) P.slot_fields.push_back(f);

  // ---- transfer predicates.  A row is uploaded when it first becomes held if
  // some element of it is read before written, or if it will be downloaded
  // without every element being written (so the download cannot clobber the
  // host copy with unset values).  A row is downloaded when it stops being
  // held if the chain wrote it -- unless Cyclic skips temporaries.
  std::vector<std::vector<char>> need_up(nf), need_down(nf);
  bool any_fp32 = false;
  for (int f : P.slot_fields) {
    const bool skip_down = in.cyclic && P.temporary[f];
    need_up[f].assign(F[f].nrows, 0);
    need_down[f].assign(F[f].nrows, 0);
    for (int64_t r = 0; r < F[f].nrows; r++) {
      need_down[f][r] = written[f][r] && !skip_down;
      need_up[f][r] = readfirst[f][r] || (need_down[f][r] && !full[f][r]);
    }
    any_fp32 |= F[f].fp32;
  }
  auto count = [](const std::vector<char> &v, int64_t r0, int64_t r1) {
    int64_t n = 0;
    for (int64_t r = std::max<int64_t>(r0, 0); r < std::min<int64_t>(r1, (int64_t)v.size()); r++) n += v[r];
    return n;
  };

  // ---- skewed tiling for a given tile height
  // The ragged remainder of the range goes to the first tile, not the last:
  // the first tile already holds the chain's whole skew, and the last S
  // tiles are what the next chain's first uploads wait for, so a short first
  // tile and full last ones let those uploads overlap the last computes.
  auto tile_plan = [&](int64_t h, Plan &Q) -> uint64_t {
    const int T = (int)((R - L + h - 1) / h);
    const int64_t lead = (int64_t)T * h - (R - L);  // rows the first tile lacks, 0 <= lead < h
    Q.T = T;
    Q.h = h;
    Q.e.assign((size_t)n * T, 0);
    for (int i = 0; i < n; i++) Q.e[(size_t)i * T + T - 1] = P.hi[i];
    for (int t = 0; t + 1 < T; t++) {
      const int64_t cut = L + (int64_t)(t + 1) * h - lead;
      for (int i = n - 1; i >= 0; i--) {
        int64_t v = cut;
        for (int j = i + 1; j < n; j++) {
          const int64_t ej = Q.e[(size_t)j * T + t];
          if (ej <= P.lo[j]) continue;  // loop j has executed nothing yet
          for (const Access &aj : acc[j])
            for (const Access &ai : acc[i]) {
              if (ai.f != aj.f) continue;
              if (ai.w && aj.r) v = std::max(v, ej + aj.rmax);  // read after write
              if (ai.r && aj.w) v = std::max(v, ej - ai.rmin);  // write after read
              if (ai.w && aj.w) v = std::max(v, ej);            // write after write
            }
        }
        const int64_t prev = t == 0 ? P.lo[i] : Q.e[(size_t)i * T + t - 1];
        v = std::max(v, prev);
        Q.e[(size_t)i * T + t] = std::min(std::max(v, P.lo[i]), P.hi[i]);
      }
    }
    // footprints (convex hull of the rows each tile touches), then rows held
    // in the slot: a row stays held from the first to the last tile that
    // touches it, so it can be handed from tile to tile by the edge copy
    Q.resA.assign((size_t)nf * T, 0);
    Q.resB.assign((size_t)nf * T, 0);
    Q.cap.assign(nf, 0);
    std::vector<int64_t> a((size_t)nf * T, INT64_MAX), bb((size_t)nf * T, INT64_MIN);
    for (int t = 0; t < T; t++)
      for (int i = 0; i < n; i++) {
        int64_t s = t == 0 ? P.lo[i] : Q.e[(size_t)i * T + t - 1];
        int64_t en = Q.e[(size_t)i * T + t];
        if (s >= en) continue;
        bool empty = false;
        for (int ax = 0; ax < in.ndim; ax++)
          if (in.loops[i].hi[ax] <= in.loops[i].lo[ax]) empty = true;
        if (empty) continue;
        for (const Access &x : acc[i]) {
          const int64_t rl = F[x.f].lo[tax];
          a[(size_t)x.f * T + t] = std::min(a[(size_t)x.f * T + t], s + x.fmin() - rl);
          bb[(size_t)x.f * T + t] = std::max(bb[(size_t)x.f * T + t], en + x.fmax() - rl);
        }
      }
    uint64_t bytes = 0;
    for (int f : P.slot_fields) {
      int64_t run = INT64_MIN;
      for (int t = 0; t < T; t++) {
        run = std::max(run, bb[(size_t)f * T + t]);
        Q.resB[(size_t)f * T + t] = run;
      }
      run = INT64_MAX;
      for (int t = T - 1; t >= 0; t--) {
        run = std::min(run, a[(size_t)f * T + t]);
        Q.resA[(size_t)f * T + t] = run;
      }
      int64_t cap = 0;
      for (int t = 0; t < T; t++) {
        int64_t &A = Q.resA[(size_t)f * T + t], &B = Q.resB[(size_t)f * T + t];
        A = std::max<int64_t>(A, 0);
        B = std::min<int64_t>(B, F[f].nrows);
        if (B <= A) A = B = 0;  // not held in this tile
        cap = std::max(cap, B - A);
      }
      Q.cap[f] = cap;
      bytes += (uint64_t)((cap * F[f].row_bytes_dev() + 255) / 256 * 256);
    }
    // float32 streaming: staging for one tile's uploads and one tile's downloads
    uint64_t sup = 0, sdown = 0;
    if (any_fp32)
      for (int t = 0; t < T; t++) {
        uint64_t u = 0, d = 0;
        for (int f : P.slot_fields) {
          if (!F[f].fp32) continue;
          const int64_t A = Q.resA[(size_t)f * T + t], B = Q.resB[(size_t)f * T + t];
          if (B <= A) continue;
          const bool prev = t > 0 && Q.resB[(size_t)f * T + t - 1] > Q.resA[(size_t)f * T + t - 1];
          const int64_t new0 = prev ? std::max(A, Q.resB[(size_t)f * T + t - 1]) : A;
          const bool next = t + 1 < T && Q.resB[(size_t)f * T + t + 1] > Q.resA[(size_t)f * T + t + 1];
          const int64_t leave1 = next ? std::min(B, Q.resA[(size_t)f * T + t + 1]) : B;
          u += (uint64_t)((count(need_up[f], new0, B) * F[f].row_bytes_host() + 255) / 256 * 256);
          d += (uint64_t)((count(need_down[f], A, leave1) * F[f].row_bytes_host() + 255) / 256 * 256);
        }
        sup = std::max(sup, u);
        sdown = std::max(sdown, d);
      }
    if (!in.ring) {
      Q.stage_up_off = bytes;
      Q.stage_down_off = bytes + sup;
      Q.slot_bytes = bytes + sup + sdown;
      return Q.slot_bytes;
    }
    // ring slabs: a field's ring holds the rows of S consecutive tiles (the
    // tiles that can be in flight together), from the first held row of the
    // oldest to the last held row of the newest
    Q.ring = true;
    Q.ring_rows.assign(nf, 0);
    Q.ring_bytes.assign(nf, 0);
    uint64_t rbytes = 0;
    for (int f : P.slot_fields) {
      int64_t need = 0;
      for (int t = 0; t < T; t++) {
        if (Q.resB[(size_t)f * T + t] <= Q.resA[(size_t)f * T + t]) continue;
        const int64_t lo = Q.resA[(size_t)f * T + t];
        int64_t hi = Q.resB[(size_t)f * T + t];
        for (int u = t + 1; u < std::min(T, t + in.S); u++)
          if (Q.resB[(size_t)f * T + u] > Q.resA[(size_t)f * T + u]) hi = std::max(hi, Q.resB[(size_t)f * T + u]);
        need = std::max(need, hi - lo);
      }
      Q.ring_rows[f] = need;
      const uint64_t b = (uint64_t)need * F[f].row_bytes_dev();
      Q.ring_bytes[f] = (b + in.ring_granule - 1) / in.ring_granule * in.ring_granule;
      rbytes += Q.ring_bytes[f];
    }
    Q.stage_up_off = 0;
    Q.stage_down_off = sup;
    Q.stage_bytes = (sup + sdown + 255) / 256 * 256;
    Q.slot_bytes = rbytes + (uint64_t)in.S * Q.stage_bytes;
    return Q.slot_bytes;
  };

  const int64_t span = R - L;
  Plan Q;
  int64_t h;
  if (in.forced_h > 0) {
    h = std::min(in.forced_h, span);
    if (tile_plan(h, Q) > in.slot_capacity) {
      err = "tile height " + std::to_string(h) + " needs " + std::to_string(Q.slot_bytes) +
            (in.ring ? " bytes of rings" : " bytes per slot") + ", more than the " +
            std::to_string(in.slot_capacity) + " available";
      return OOC_E_BUDGET;
    }
  } else if (tile_plan(span, Q) <= in.slot_capacity) {
    h = span;
  } else {
    if (tile_plan(1, Q) > in.slot_capacity) {
      err = "even one-row tiles need " + std::to_string(Q.slot_bytes) +
            (in.ring ? " bytes of rings" : " bytes per slot") + ", more than the " +
            std::to_string(in.slot_capacity) + " available";
      return OOC_E_BUDGET;
    }
    int64_t good = 1, bad = span;
    while (bad - good > 1) {
      int64_t mid = good + (bad - good) / 2;
      if (tile_plan(mid, Q) <= in.slot_capacity) good = mid;
      else bad = mid;
    }
    h = good;
  }
  // Ring slabs, tile height chosen by the planner: consecutive chains of the
  // same plan overlap only if the next chain's first tiles take ring
  // positions the previous chain's tiles still in flight do not hold
  // (Prefetch, Section 4.1); otherwise they wait for those tiles'
  // downloads.  Prefer the tallest tile, down to 3/5 of the tallest that
  // fits, whose rings allow that (ns3d 512^3, 4-step chains, 3 slots: 28
  // instead of 39 planes, 43.3 against 45.2 ms per step).
  if (in.ring && in.forced_h <= 0) {
    auto boundary_clean = [&](const Plan &X) {
      const int T = X.T, S = in.S;
      for (int f : P.slot_fields) {
        const uint64_t R = X.ring_bytes[f], rb = F[f].row_bytes_dev();
        if (!R) continue;
        for (int t = 0; t < std::min(T, S); t++) {
          const int64_t A = X.resA[(size_t)f * T + t], B = X.resB[(size_t)f * T + t];
          if (B <= A) continue;
          for (int u = T - 1; u >= 0 && u > T - S + t; u--) {
            const int64_t pA = X.resA[(size_t)f * T + u], pB = X.resB[(size_t)f * T + u];
            if (pB > pA && ring_ranges_meet((uint64_t)A * rb % R, (uint64_t)(B - A) * rb, (uint64_t)pA * rb % R,
                                            (uint64_t)(pB - pA) * rb, R))
              return false;
          }
        }
      }
      return true;
    };
    tile_plan(h, Q);
    if (!boundary_clean(Q))
      for (int64_t h2 = h - 1; h2 >= std::max<int64_t>(1, h * 3 / 5); h2--) {
        Plan Q2;
        if (tile_plan(h2, Q2) <= in.slot_capacity && boundary_clean(Q2)) {
          h = h2;
          break;
        }
      }
  }
  tile_plan(h, Q);
  P.T = Q.T;
  P.h = Q.h;
  P.e.swap(Q.e);
  P.resA.swap(Q.resA);
  P.resB.swap(Q.resB);
  P.cap.swap(Q.cap);
  P.slot_bytes = Q.slot_bytes;
  P.stage_up_off = Q.stage_up_off;
  P.stage_down_off = Q.stage_down_off;
  P.ring = Q.ring;
  P.ring_rows.swap(Q.ring_rows);
  P.ring_bytes.swap(Q.ring_bytes);
  P.stage_bytes = Q.stage_bytes;
  P.slab_off.assign(nf, 0);
  {
    uint64_t off = 0;
    for (int f : P.slot_fields) {
      P.slab_off[f] = off;
      off += (uint64_t)((P.cap[f] * F[f].row_bytes_dev() + 255) / 256 * 256);
    }
  }

  // ---- transfer sets (runs of consecutive rows)
  const int T = P.T;
  for (int f : P.slot_fields) {
    auto up_pred = [&](int64_t r) { return need_up[f][r] != 0; };
    auto down_pred = [&](int64_t r) { return need_down[f][r] != 0; };
    auto emit = [&](std::vector<Run> &out, int t, int64_t r0, int64_t r1, auto pred) {
      int64_t r = r0;
      while (r < r1) {
        while (r < r1 && !pred(r)) r++;
        int64_t s = r;
        while (r < r1 && pred(r)) r++;
        if (r > s) out.push_back(Run{f, t, s, r});
      }
    };
    for (int t = 0; t < T; t++) {
      const int64_t A = P.resA[(size_t)f * T + t], B = P.resB[(size_t)f * T + t];
      if (B <= A) continue;
      int64_t pB = 0;
      bool prev = t > 0 && P.resB[(size_t)f * T + t - 1] > P.resA[(size_t)f * T + t - 1];
      if (prev) pB = P.resB[(size_t)f * T + t - 1];
      const int64_t new0 = prev ? std::max(A, pB) : A;
      emit(P.up, t, new0, B, up_pred);
      if (prev && pB > A) P.edge.push_back(Run{f, t, A, std::min(pB, B)});
      bool next = t + 1 < T && P.resB[(size_t)f * T + t + 1] > P.resA[(size_t)f * T + t + 1];
      const int64_t leave1 = next ? std::min(B, P.resA[(size_t)f * T + t + 1]) : B;
      emit(P.down, t, A, leave1, down_pred);
    }
  }
  return OOC_OK;
}

void choose_ring_origins(int nf, const uint64_t *ring_bytes, const uint64_t *row_bytes, const RingChain &prev,
                         const RingChain &next, int S, uint64_t *origin_out, int64_t *wait_out) {
  // One origin index q for every ring (origin q/kRingOrigins of the ring):
  // then the chains' origins repeat within kRingOrigins chains, and so do the
  // launch-argument tables that depend on them.  For each q and each of the
  // next chain's first S tiles t, the last previous-chain tile still in
  // flight (after the tile S before t) whose rows meet tile t's ring
  // positions in any ring; the lexicographically smallest list of those
  // waits wins, the smaller q on ties.
  std::vector<int64_t> w(S), best(S);
  int best_q = -1;
  for (int q = 0; q < kRingOrigins; q++) {
    std::fill(w.begin(), w.end(), -1);
    for (int f = 0; f < nf; f++) {
      const uint64_t R = ring_bytes[f], rb = row_bytes[f];
      if (!R) continue;
      const uint64_t O = (uint64_t)q * (R / kRingOrigins);
      for (int t = 0; t < S && t < next.T; t++) {
        const int64_t A = next.resA[(size_t)f * next.T + t], B = next.resB[(size_t)f * next.T + t];
        if (B <= A) continue;
        const uint64_t a = ((uint64_t)A * rb + O) % R, la = (uint64_t)(B - A) * rb;
        for (int64_t u = prev.T - 1; u >= 0 && u > (int64_t)prev.T - S + t && u > w[t]; u--) {
          const int64_t pA = prev.resA[(size_t)f * prev.T + u], pB = prev.resB[(size_t)f * prev.T + u];
          if (pB <= pA) continue;
          const uint64_t b = ((uint64_t)pA * rb + prev.origin[f]) % R, lb = (uint64_t)(pB - pA) * rb;
          if (ring_ranges_meet(a, la, b, lb, R)) {
            w[t] = u;
            break;
          }
        }
      }
    }
    if (best_q < 0 || std::lexicographical_compare(w.begin(), w.end(), best.begin(), best.end())) {
      best = w;
      best_q = q;
    }
  }
  for (int f = 0; f < nf; f++) origin_out[f] = ring_bytes[f] ? (uint64_t)best_q * (ring_bytes[f] / kRingOrigins) : 0;
  for (int t = 0; t < S; t++) wait_out[t] = best[t];
}

}  // namespace ooc
