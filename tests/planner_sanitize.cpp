// Host check of the tile planner, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_planner_sanitized.py (plain g++,
// no HIP: the planner is host-only code).  Random chains of loops with random
// stencils on random 2D and 3D grids are planned for many tile heights, slot
// counts and slot capacities; every plan must satisfy the invariants of the
// tiling (Section 3, Section 4 and Figure 2 of the paper):
//   - each loop's range is partitioned exactly by its per-tile row ranges;
//   - every transfer and edge run lies inside the rows its field holds in
//     that tile, and inside the field's storage;
//   - the slot holds every field's rows and fits the slot capacity;
// and any memory error or undefined behaviour aborts the run.
#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "../paper_1709_02125_amd/csrc/ooc_internal.h"

using namespace ooc;

namespace {

int failures = 0;

void check(bool ok, const char *what, int seed) {
  if (!ok) {
    if (failures < 20) std::fprintf(stderr, "seed %d: %s\n", seed, what);
    failures++;
  }
}

struct Case {
  int ndim, tax, halo;
  int64_t dims[3];
  std::vector<Field> fields;
  std::vector<LoopRec> loops;
};

Case random_case(std::mt19937_64 &rng, int seed) {
  Case c;
  c.ndim = (seed % 3 == 0) ? 3 : 2;
  c.tax = c.ndim - 1;
  c.halo = 2;
  auto uni = [&](int64_t a, int64_t b) { return std::uniform_int_distribution<int64_t>(a, b)(rng); };
  c.dims[0] = uni(8, 40);
  c.dims[1] = c.ndim == 3 ? uni(4, 12) : uni(20, 160);
  c.dims[2] = c.ndim == 3 ? uni(20, 80) : 1;
  const int nf = (int)uni(2, 7);
  const int64_t pitch = c.dims[0] + 2 * c.halo + 1 + kXOrigin;
  const int64_t plane = pitch * (c.dims[1] + 2 * c.halo + 1);
  for (int f = 0; f < nf; f++) {
    Field fd;
    fd.name = "f" + std::to_string(f);
    for (int a = 0; a < 3; a++) {
      fd.delta[a] = a < c.ndim ? (int32_t)uni(0, 1) : 0;
      fd.lo[a] = a < c.ndim ? -c.halo : 0;
      fd.n[a] = a < c.ndim ? c.dims[a] + 2 * c.halo + fd.delta[a] : 1;
    }
    fd.nrows = fd.n[c.tax];
    fd.row_elems = c.ndim == 2 ? pitch : plane;
    fd.resident = uni(0, 9) == 0;
    fd.fp32 = uni(0, 3) == 0;
    c.fields.push_back(fd);
  }
  const int nloops = (int)uni(1, 14);
  int marks = 0;
  for (int i = 0; i < nloops; i++) {
    LoopRec L;
    L.kid = OOC_K_AVG;
    const int out = (int)uni(0, nf - 1);
    int in = (int)uni(0, nf - 1);
    // stencil reach along each axis; a loop never reads what it writes at an offset
    int reach[3] = {(int)uni(0, 1), (int)uni(0, 2), c.ndim == 3 ? (int)uni(0, 2) : 0};
    if (in == out) reach[0] = reach[1] = reach[2] = 0;
    for (int a = 0; a < 3; a++) {
      if (a >= c.ndim) {
        L.lo[a] = 0;
        L.hi[a] = 1;
        continue;
      }
      // keep every access inside both fields' extents
      const int64_t lo_min = -c.halo + reach[a];
      const int64_t hi_max = std::min(c.fields[out].n[a], c.fields[in].n[a] - reach[a]) - c.halo;
      int64_t lo = uni(lo_min, std::max(lo_min, hi_max - 1));
      int64_t hi = uni(lo, hi_max);
      if (uni(0, 7) == 0) hi = lo;  // an empty loop now and then
      L.lo[a] = lo;
      L.hi[a] = hi;
    }
    ArgRec w;
    w.kind = OOC_ARG_DAT;
    w.handle = out;
    w.access = uni(0, 3) == 0 ? OOC_RW : OOC_WRITE;
    w.offs = {0, 0, 0};
    ArgRec r;
    r.kind = OOC_ARG_DAT;
    r.handle = in;
    r.access = OOC_READ;
    const int npts = (int)uni(1, 5);
    for (int p = 0; p < npts; p++)
      for (int a = 0; a < 3; a++) r.offs.push_back(a < c.ndim ? (int32_t)uni(-reach[a], reach[a]) : 0);
    L.args = {w, r};
    for (double v : {1.0, 0.0}) {
      ArgRec k;
      k.kind = OOC_ARG_CONST;
      k.value = v;
      L.args.push_back(k);
    }
    if (uni(0, 4) == 0) marks++;
    L.marks_before = marks;
    c.loops.push_back(L);
  }
  return c;
}

void check_plan(const Case &c, const Plan &P, uint64_t capacity, int seed) {
  const int T = P.T, n = (int)c.loops.size(), nf = (int)c.fields.size();
  check(T >= 1, "at least one tile", seed);
  check((int)P.e.size() == n * T, "tile ends sized loops x tiles", seed);
  check(P.slot_bytes <= capacity, "slot fits its capacity", seed);
  if (P.ring) {
    check((int)P.ring_rows.size() == nf && (int)P.ring_bytes.size() == nf, "ring sizes per field", seed);
    for (int f = 0; f < nf; f++) {
      if (P.ring_bytes.size() != (size_t)nf) break;
      check(P.ring_bytes[f] >= (uint64_t)P.ring_rows[f] * c.fields[f].row_bytes_dev(), "ring holds its rows", seed);
      // the rows of S consecutive tiles fit the ring
      for (int t = 0; t < T; t++) {
        int64_t lo = INT64_MAX, hi = INT64_MIN;
        for (int u = t; u < std::min(T, t + P.S); u++) {
          const int64_t A = P.resA[(size_t)f * T + u], B = P.resB[(size_t)f * T + u];
          if (B <= A) continue;
          lo = std::min(lo, A);
          hi = std::max(hi, B);
        }
        if (hi > lo) check(hi - lo <= P.ring_rows[f], "tiles in flight fit the ring", seed);
      }
    }
  }
  for (int i = 0; i < n; i++) {
    if (P.lo[i] >= P.hi[i]) continue;
    check(P.s(i, 0) == P.lo[i], "first tile starts at the loop start", seed);
    check(P.en(i, T - 1) == P.hi[i], "last tile ends at the loop end", seed);
    for (int t = 0; t < T; t++) check(P.s(i, t) <= P.en(i, t), "tile ranges are monotone", seed);
  }
  check((int)P.resA.size() == nf * T && (int)P.resB.size() == nf * T, "residency sized", seed);
  auto inside = [&](const Run &r) {
    if (r.f < 0 || r.f >= nf || r.t < 0 || r.t >= T || r.lo >= r.hi) return false;
    const Field &f = c.fields[r.f];
    if (r.lo < 0 || r.hi > f.nrows) return false;
    const int64_t A = P.resA[(size_t)r.f * T + r.t], B = P.resB[(size_t)r.f * T + r.t];
    return A <= r.lo && r.hi <= B && B - A <= P.cap[r.f];
  };
  for (const Run &r : P.up) check(inside(r), "upload run inside the held rows", seed);
  for (const Run &r : P.down) check(inside(r), "download run inside the held rows", seed);
  for (const Run &r : P.edge) {
    check(inside(r), "edge run inside the held rows", seed);
    if (r.t > 0 && r.f >= 0 && r.f < nf) {
      const int64_t pA = P.resA[(size_t)r.f * T + r.t - 1], pB = P.resB[(size_t)r.f * T + r.t - 1];
      check(pA <= r.lo && r.hi <= pB, "edge run held by the previous tile", seed);
    }
  }
}

// Two consecutive ring chains: with the origins choose_ring_origins picks,
// every tile of the previous chain that may still be in flight when one of
// the next chain's first S tiles uploads (after the tile S before it, and
// after the chosen wait) holds ring bytes disjoint from that tile's, checked
// element by element on a map of each ring.
void check_ring_origins(const Case &c, const Plan &A, const Plan &B, int S, std::mt19937_64 &rng, int seed) {
  const int nf = (int)c.fields.size();
  std::vector<uint64_t> R(nf), rb(nf), prev_origin(nf), origin(nf);
  for (int f = 0; f < nf; f++) {
    R[f] = A.ring_bytes[f];
    rb[f] = c.fields[f].row_bytes_dev();
    const uint64_t units = R[f] / 8;
    prev_origin[f] = units ? (std::uniform_int_distribution<uint64_t>(0, units - 1)(rng)) * 8 : 0;
  }
  RingChain pv, nx;
  pv.T = A.T;
  pv.resA = A.resA.data();
  pv.resB = A.resB.data();
  pv.origin = prev_origin.data();
  nx.T = B.T;
  nx.resA = B.resA.data();
  nx.resB = B.resB.data();
  std::vector<int64_t> wait(S);
  choose_ring_origins(nf, R.data(), rb.data(), pv, nx, S, origin.data(), wait.data());
  for (int t = 0; t < S; t++) check(wait[t] >= -1 && wait[t] < A.T, "wait names a previous tile", seed);
  int q = -1;  // every ring at the same fraction q / kRingOrigins
  for (int f = 0; f < nf; f++) {
    if (!R[f]) continue;
    check(origin[f] < R[f] && origin[f] % (R[f] / kRingOrigins) == 0, "origin is one of the candidates", seed);
    const int qf = (int)(origin[f] / (R[f] / kRingOrigins));
    check(q < 0 || qf == q, "one origin fraction for every ring", seed);
    q = qf;
    const uint64_t units = R[f] / 8, per_row = rb[f] / 8;
    auto cell = [&](int64_t r, uint64_t k, uint64_t o) { return ((uint64_t)r * rb[f] + o) / 8 % units + k; };
    for (int t = 0; t < S && t < B.T; t++) {
      const int64_t nA = B.resA[(size_t)f * B.T + t], nB = B.resB[(size_t)f * B.T + t];
      if (nB <= nA) continue;
      std::vector<char> held(units, 0);
      for (int64_t u = 0; u < A.T; u++) {
        if (u <= (int64_t)A.T - S + t || u <= wait[t]) continue;  // done before tile t uploads
        const int64_t pA = A.resA[(size_t)f * A.T + u], pB = A.resB[(size_t)f * A.T + u];
        for (int64_t r = pA; r < pB; r++)
          for (uint64_t k = 0; k < per_row; k++) held[cell(r, k, prev_origin[f]) % units] = 1;
      }
      bool clash = false;
      for (int64_t r = nA; r < nB && !clash; r++)
        for (uint64_t k = 0; k < per_row && !clash; k++) clash = held[cell(r, k, origin[f]) % units] != 0;
      check(!clash, "next chain's tile takes no ring bytes a tile in flight holds", seed);
    }
  }
}

}  // namespace

int main(int argc, char **argv) {
  const int ncases = argc > 1 ? std::atoi(argv[1]) : 300;
  int planned = 0, budget_refusals = 0, rings_checked = 0;
  for (int seed = 0; seed < ncases; seed++) {
    std::mt19937_64 rng(0x9e3779b97f4a7c15ull ^ (uint64_t)seed);
    Case c = random_case(rng, seed);
    for (int mode = 0; mode < 4; mode++)
      for (int S = 2; S <= 4; S++)
        for (int64_t h : {0, 1, 2, 3, 5, 8, 13, 40}) {
          for (uint64_t capacity : {UINT64_MAX, (uint64_t)1 << 16, (uint64_t)1 << 20, (uint64_t)0}) {
            PlanInput in;
            in.ndim = c.ndim;
            in.tax = c.tax;
            in.halo = c.halo;
            in.fields = &c.fields;
            in.loops = c.loops.data();
            in.nloops = (int)c.loops.size();
            const bool cyclic = (mode & 1) != 0;
            in.cyclic = cyclic;
            in.ring = (mode & 2) != 0;  // ring slabs
            in.S = S;
            in.forced_h = h;
            in.slot_capacity = capacity;
            Plan P;
            std::string err;
            const int rc = make_plan(in, P, err);
            check(rc == OOC_OK || rc == OOC_E_BUDGET, "plan returns OK or BUDGET", seed);
            if (rc == OOC_OK) {
              planned++;
              check_plan(c, P, capacity, seed);
              if (P.ring && capacity == ((uint64_t)1 << 20)) {
                // the next chain: the same plan, or one with other tile heights
                // that fits the rings the first one sized
                check_ring_origins(c, P, P, S, rng, seed);
                PlanInput in2 = in;
                in2.forced_h = h == 0 ? 3 : h + 2;
                Plan P2;
                std::string err2;
                if (make_plan(in2, P2, err2) == OOC_OK) {
                  bool fits = true;
                  for (size_t f = 0; f < P.ring_bytes.size(); f++) fits = fits && P2.ring_bytes[f] <= P.ring_bytes[f];
                  if (fits) {
                    rings_checked++;
                    check_ring_origins(c, P, P2, S, rng, seed);
                  }
                }
              }
            } else {
              budget_refusals++;
              check(!err.empty(), "a refusal says why", seed);
            }
          }
        }
  }
  std::printf("planned %d, refused %d, ring chain pairs %d, failures %d\n", planned, budget_refusals, rings_checked,
              failures);
  return failures ? 1 : 0;
}
