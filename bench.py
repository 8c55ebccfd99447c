"""Benchmark: grid-point updates/s of a stencil chain whose fields are about 3x
the device budget, streamed tile by tile through HBM by the HIP library;
beside it the same grid fully resident (in-core), the dominant kernel's HBM
roofline, the host-link throughput, and the CPU oracle timed on a sample.

Workloads (one step = one time step over the whole grid):
  hydro2d (default)  15360 x 15360 FP64, 25 fields, 55-loop chain, budget 16e9 B
  hydro3d            640^3 FP64, 30 fields, 82-loop chain, budget 1/3 of the fields
  ns3d               512^3 FP64, 15 fields (residual evaluates the gradients; --stored-gradients:
                     27 fields), budget 1/3 of the fields, chains of --chain-steps steps
python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload hydro2d|hydro3d|ns3d]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, published
LINK_PEAK_GBS = 64.0       # PCIe Gen5 x16 per direction, nominal
METRIC = "grid-point updates/s at 3x device-budget oversubscription; % of in-core rate"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


H2D_NAMES = ["h2d_eos", "h2d_eos_p", "h2d_visc", "h2d_pdv_pred", "h2d_pdv_corr", "h2d_accel", "h2d_flux_x",
             "h2d_flux_y", "h2d_adv_vol_x", "h2d_adv_vol_y", "h2d_adv_flux_x", "h2d_adv_flux_y",
             "h2d_adv_cell_x", "h2d_adv_cell_y", "h2d_nflux_x", "h2d_nflux_y", "h2d_nmass_x", "h2d_nmass_y",
             "h2d_mflux_x", "h2d_mflux_y", "h2d_vel_x", "h2d_vel_y", "h2d_dt"]
H3D_NAMES = ["h3d_visc", "h3d_pdv_pred", "h3d_pdv_corr", "h3d_accel"] + \
            ["h3d_%s_%s" % (k, a) for k in ("flux", "adv_vol", "adv_flux", "adv_cell", "nflux", "nmass",
                                            "mflux", "vel") for a in "xyz"] + ["h3d_dt"]
NS_NAMES = ["ns_init", "ns_prims", "ns_grads", "ns_rhs_first", "ns_rhs", "ns_rhs_fused_first", "ns_rhs_fused",
            "ns_rhs_fusedq_first", "ns_rhs_fusedq"]
COMMON = {1: "mirror", 2: "fill", 3: "sum_prod"}


def ablations(pf):
    """The two other combinations of the transfer optimisations the paper
    evaluates (Section 4.1, measured in Section 5.3) beside the headline's
    Prefetch + Cyclic: speculative Prefetch off (a chain's first tile is
    uploaded only once the previous chain's last tile has run), and both
    Prefetch and Cyclic off (write-first data is downloaded too)."""
    return [("no_prefetch_cyclic", 0, {}), ("no_prefetch_no_cyclic", 0, {"cyclic": False})]


def summary_variants(pf, every=10):
    """The headline run with the field summary (volume, mass, internal and
    kinetic energy, pressure) read every `every` steps, the periodic
    diagnostic the paper names as a cause of its CloverLeaf 2D gap (Section
    5.3): folded into that step's chain, and as a chain of its own."""
    return [("field_summary_every_%d_folded" % every, pf, {"summary": ("folded", every)}),
            ("field_summary_every_%d_separate" % every, pf, {"summary": ("separate", every)})]


def summary_runner(app, mode, every):
    """A step loop for timed_run that queues the field summary after every
    `every`-th step and reads it (each read waits for the device)."""
    def run(steps):
        for s in range(1, steps + 1):
            app.queue_step()
            if s % every:
                app.ctx.submit()
                continue
            if mode == "separate":
                app.ctx.submit()
            app.queue_summary()
            app.summary()
        app.ctx.execute()
    return run


class Workload:
    """One benchmark problem: how to build the app at a budget, its sizes,
    kernel names, and its CPU-oracle sample."""

    def __init__(self, args):
        self.args = args


class Hydro2DWork(Workload):
    def __init__(self, args):
        super().__init__(args)
        from paper_1709_02125_amd import hydro2d as h2
        from paper_1709_02125_amd.inputs import hydro_initial_state
        self.mod = h2
        self.n = args.n or 15360
        self.cells = self.n * self.n
        self.footprint = h2.footprint_bytes(self.n, self.n)
        self.budget = int(args.budget) if args.budget else 16_000_000_000
        log("generating input %dx%d" % (self.n, self.n))
        self.rho, self.ene = hydro_initial_state((self.n, self.n))
        self.knames = {**COMMON, **{100 + i: s for i, s in enumerate(H2D_NAMES)}}
        self.dominant = 100 + H2D_NAMES.index("h2d_pdv_corr")

    def make(self, budget, flags, incore=False, **opts):
        h2 = self.mod
        if incore:
            return h2.Hydro2D(self.n, self.n, self.rho, self.ene, budget=h2.device_footprint_bytes(self.n, self.n),
                              flags=flags)
        return h2.Hydro2D(self.n, self.n, self.rho, self.ene, budget=budget, flags=flags,
                          resident_geometry=opts.get("resident_geometry", self.args.resident_geometry),
                          cyclic_after_init=opts.get("cyclic", not self.args.no_cyclic),
                          resident_state=opts.get("resident_state", self.args.resident_state),
                          summary="summary" in opts)

    def variants(self):
        from paper_1709_02125_amd import ooc
        pf = ooc.FLAG_PREFETCH
        return [*ablations(pf),
                ("fp32_stream_resident_geometry", pf | ooc.FLAG_FP32_STREAM, {"resident_geometry": True}),
                ("resident_geometry", pf, {"resident_geometry": True}),
                ("resident_state", pf, {"resident_state": True}),
                ("resident_state_fused", pf | ooc.FLAG_FUSE, {"resident_state": True}),
                *summary_variants(pf)]

    def describe(self):
        return ("hydro2d proxy %dx%d FP64, 25 fields, 55-loop chain per step, device budget %.3g B "
                "(footprint %.3g B, %.2fx oversubscribed), tiles along y" %
                (self.n, self.n, self.budget, self.footprint, self.footprint / self.budget))

    def cpu_baseline(self, target_s=15.0, one_thread=False):
        return cpu_hydro2d(self.n, target_s, one_thread)


class Hydro3DWork(Workload):
    def __init__(self, args):
        super().__init__(args)
        from paper_1709_02125_amd import hydro3d as h3
        from paper_1709_02125_amd.inputs import hydro_initial_state
        self.mod = h3
        self.n = args.n or 640
        self.dims = (self.n, self.n, self.n)
        self.cells = self.n ** 3
        self.footprint = h3.footprint_bytes(self.dims)
        self.budget = int(args.budget) if args.budget else self.footprint // 3
        log("generating input %d^3" % self.n)
        self.rho, self.ene = hydro_initial_state(self.dims)
        self.knames = {**COMMON, 100: "h2d_eos", 101: "h2d_eos_p",
                       **{300 + i: s for i, s in enumerate(H3D_NAMES)}}
        self.dominant = 300 + H3D_NAMES.index("h3d_pdv_corr")

    def make(self, budget, flags, incore=False, **opts):
        h3 = self.mod
        if incore:
            return h3.Hydro3D(self.dims, self.rho, self.ene, budget=h3.device_footprint_bytes(self.dims),
                              flags=flags)
        return h3.Hydro3D(self.dims, self.rho, self.ene, budget=budget, flags=flags,
                          resident_geometry=opts.get("resident_geometry", self.args.resident_geometry),
                          cyclic_after_init=opts.get("cyclic", not self.args.no_cyclic),
                          resident_state=opts.get("resident_state", self.args.resident_state))

    def variants(self):
        from paper_1709_02125_amd import ooc
        pf = ooc.FLAG_PREFETCH
        return [*ablations(pf),
                ("fp32_stream_resident_geometry", pf | ooc.FLAG_FP32_STREAM, {"resident_geometry": True}),
                ("resident_geometry", pf, {"resident_geometry": True})]

    def describe(self):
        return ("hydro3d proxy %d^3 FP64, 30 fields, 82-loop chain per step, device budget %.3g B "
                "(footprint %.3g B, %.2fx oversubscribed), tiles along z" %
                (self.n, self.budget, self.footprint, self.footprint / self.budget))

    def cpu_baseline(self, target_s=15.0, one_thread=False):
        return cpu_hydro3d(self.n, target_s, one_thread)


def ns_form(args):
    """The ns3d chain form: "q" (the default: two copies of the conserved
    variables, primitives and gradients evaluated in the residual kernel),
    True (stored primitives, gradients in the residual) or False (stored
    primitives and gradients)."""
    if getattr(args, "stored_gradients", False):
        return False
    return True if getattr(args, "stored_primitives", False) else "q"


class NS3DWork(Workload):
    def __init__(self, args):
        super().__init__(args)
        from paper_1709_02125_amd import ns3d as N
        from paper_1709_02125_amd.inputs import tgv_initial_state
        self.mod = N
        self.fused = ns_form(args)
        self.n = args.n or 512
        self.cells = self.n ** 3
        self.footprint = N.footprint_bytes(self.n, self.fused)
        self.budget = int(args.budget) if args.budget else self.footprint // 3
        log("generating input %d^3" % self.n)
        self.prims = tgv_initial_state(self.n)
        self.knames = {**COMMON, **{200 + i: s for i, s in enumerate(NS_NAMES)}}
        self.dominant = 200 + NS_NAMES.index({"q": "ns_rhs_fusedq", True: "ns_rhs_fused",
                                              False: "ns_rhs"}[self.fused])

    def make(self, budget, flags, incore=False, **opts):
        N = self.mod
        fused = opts.get("fused", self.fused)
        if incore:
            return N.NS3D(self.n, self.prims, budget=N.device_footprint_bytes(self.n, fused), flags=flags,
                          fused=fused)
        if fused != self.fused and not self.args.budget:  # the other form's own third of its footprint
            budget = N.footprint_bytes(self.n, fused) // 3
        app = N.NS3D(self.n, self.prims, budget=budget, flags=flags, fused=fused,
                     cyclic_after_init=opts.get("cyclic", not self.args.no_cyclic))
        app.ctx.set_schedule(tile_rows=opts.get("tile_rows", self.args.tile_rows),
                             chain_steps=opts.get("chain_steps", self.args.chain_steps),
                             slots=opts.get("slots", self.args.slots))
        return app

    def variants(self):
        from paper_1709_02125_amd import ooc
        dl = ooc.FLAG_MEMCPY_DOWNLOAD if self.args.download == "memcpy" else 0
        pf = ooc.FLAG_PREFETCH | dl
        ring = 0 if self.args.slots_mode else ooc.FLAG_RING
        # the paper's slots with edge copies, with Prefetch and Cyclic, then
        # its two ablations; the ring-slab headline's other chain lengths and
        # its downloads by copy kernel; float32 streaming of the same
        # schedule; the forms with stored primitives and stored gradients.
        # (The default form keeps two copies of the conserved variables, so
        # its chains span an even number of steps.)
        q = self.fused == "q"
        kk = {"chain_steps": 2 if q else 3}
        s2 = {"slots": 2, **kk}  # slots hold the skew of chains this long at this budget
        nm = "_chains_of_%d" % kk["chain_steps"]
        out = [("slots_edge_copies" + nm, pf, s2), ("slots_no_prefetch_cyclic" + nm, dl, s2),
               ("slots_no_prefetch_no_cyclic" + nm, dl, {"cyclic": False, **s2})]
        out += [("chains_of_%d_steps" % k, pf | ring, {"chain_steps": k})
                for k in ((2,) if q else (1, 2, 3)) if k != self.args.chain_steps]
        out += [("copy_kernel_downloads", (pf & ~dl) | ring, {}) if dl else
                ("runtime_copy_downloads", pf | ring | ooc.FLAG_MEMCPY_DOWNLOAD, {}),
                ("fp32_stream", pf | ring | ooc.FLAG_FP32_STREAM, {})]
        if q:
            out += [("stored_primitives_form", pf | ring, {"fused": True}),
                    ("stored_gradients_form_slots_24_planes_chains_of_3", pf,
                     {"fused": False, "slots": 2, "chain_steps": 3, "tile_rows": 24})]
        return out

    def warmup_steps(self, warmup, steps):
        """Untimed steps before the timed ones: at least two whole chains
        (the first after another chain shape sizes the rings; the second
        runs behind a chain of its own shape), and then the trailing partial
        chain the timed steps end with, so that every chain shape the timed
        region runs has been planned and its rings sized before it."""
        k = self.args.chain_steps
        return -(-max(warmup, 2 * k) // k) * k + steps % k

    def describe(self):
        form = {"q": "15 fields (two copies of the conserved variables; primitives and gradients evaluated in "
                     "the residual kernel), 39 loops per step",
                True: "15 fields (gradients evaluated in the residual kernel), 42 loops per step",
                False: "27 fields (12 stored gradients), 45 loops per step"}[self.fused]
        return ("ns3d proxy %d^3 FP64 (Taylor-Green, Mach 0.1), %s, chains of %d "
                "steps, device budget %.3g B (footprint %.3g B, %.2fx oversubscribed), tiles along z" %
                (self.n, form, self.args.chain_steps, self.budget, self.footprint, self.footprint / self.budget))

    def cpu_baseline(self, target_s=15.0, one_thread=False):
        return cpu_ns3d(self.n, target_s, one_thread)


def cpu_hydro2d(n, target_s, one_thread):
    """The oracle on a bounded sample of the hydro2d grid: the benchmark's
    width, half its height (a 256-row strip for the one-thread figure)."""
    import oracle
    import oracle.hydro2d as oh
    from paper_1709_02125_amd.inputs import hydro_initial_state
    oracle.build(force=False)
    nx, ny = n, (min(256, n) if one_thread else max(64, n // 2))
    rho, ene = hydro_initial_state((nx, ny))
    o = oh.Hydro2D(nx, ny)
    o.set_state(rho, ene)
    dt = o.dt()
    steps, t0 = 0, time.perf_counter()
    while steps < 20 and (time.perf_counter() - t0) < target_s:
        dt = o.step(dt)
        steps += 1
    sec = time.perf_counter() - t0
    return nx * ny * steps / sec, "%d x %d cells (same width as the benchmark grid), %d steps, %.1f s" % (
        nx, ny, steps, sec)


def cpu_hydro3d(n, target_s, one_thread):
    """The oracle on a z-slab of the hydro3d grid (8 planes for the
    one-thread figure)."""
    import oracle
    import oracle.hydro3d as oh
    from paper_1709_02125_amd.inputs import hydro_initial_state
    oracle.build(force=False)
    dims = (n, n, 8 if one_thread else max(8, n // 12))
    rho, ene = hydro_initial_state(dims)
    o = oh.Hydro3D(*dims)
    o.set_state(rho, ene)
    dt = o.dt()
    steps, t0 = 0, time.perf_counter()
    while steps < 40 and (time.perf_counter() - t0) < target_s:
        dt = o.step(dt)
        steps += 1
    sec = time.perf_counter() - t0
    cells = dims[0] * dims[1] * dims[2]
    return cells * steps / sec, "%d x %d x %d cells (a z-slab of the benchmark grid), %d steps, %.1f s" % (
        dims + (steps, sec))


def cpu_ns3d(n, target_s, one_thread):
    """The oracle on a smaller cube of the ns3d problem (n/2; 96 points per
    axis for the one-thread figure)."""
    import oracle
    import oracle.ns3d as on
    from paper_1709_02125_amd.inputs import tgv_initial_state
    oracle.build(force=False)
    m = min(96, n) if one_thread else max(16, n // 2)
    o = on.NS3D(m)
    o.set_primitives(*tgv_initial_state(m))
    dt = on.stable_dt(m)
    steps, t0 = 0, time.perf_counter()
    while steps < 40 and (time.perf_counter() - t0) < target_s:
        o.step(dt)
        steps += 1
    sec = time.perf_counter() - t0
    return m ** 3 * steps / sec, "%d^3 points, %d steps, %.1f s" % (m, steps, sec)


CPU_SAMPLES = {"hydro2d": (cpu_hydro2d, 15360), "hydro3d": (cpu_hydro3d, 640), "ns3d": (cpu_ns3d, 512)}


def cpu_one_thread(workload, n, target_s=8.0):
    """The oracle's one-thread rate on a small sample, in a child process
    started with OMP_NUM_THREADS=1 (OpenMP reads it once per process)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    code = ("import json, sys; sys.path.insert(0, %r); import bench; f, n0 = bench.CPU_SAMPLES[%r]; "
            "v, s = f(%d or n0, %r, True); print(json.dumps([v, s]))" % (ROOT, workload, n, target_s))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    if r.returncode != 0:
        log("one-thread oracle sample failed: %s" % r.stderr[-500:])
        return None
    v, sample = json.loads(r.stdout.strip().splitlines()[-1])
    return {"value": v, "sample": sample}


WORKLOADS = {"hydro2d": Hydro2DWork, "hydro3d": Hydro3DWork, "ns3d": NS3DWork}


CALL_KINDS = ("upload copy", "download", "kernel launch", "stream wait", "event record", "other")


def timed_run(app, steps, warmup, knames, dom=None, timing=True, repeats=1, run=None):
    """Warm up, then time `steps` steps with wall clock between device syncs,
    `repeats` times; the run with the median time is reported (its bytes,
    tiles and time) and every run's ms per step is listed.  With timing,
    every launch of the roofline kernel `dom` in the timed steps is bracketed
    by hipEvents on the compute stream (the stream the loops run on), so its
    average comes from the same region as the throughput.  `dom` is the
    workload's dominant kernel: the one with the most time in an in-core
    profile.  (Out of core, strip loops that overlap a download stall and can
    add up to more; the warm-up times every kernel and reports them.)  `run`
    replaces app.run (a step loop with extra work, e.g. a field summary)."""
    import torch
    run = run or app.run
    if timing:
        app.ctx.set_timing(True)
        run(warmup)
        per = {kid: app.ctx.kernel_stats(kid)[0] for kid in knames}
        app.ctx.set_timing(True, kernel_id=dom)
    else:
        run(warmup)
    runs = []
    for _ in range(repeats):
        s0 = app.ctx.stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s1 = app.ctx.stats()
        d = {k: s1[k] - s0[k] for k in ("bytes_h2d", "bytes_d2h", "bytes_edge", "bytes_hbm_alg", "tiles",
                                         "chains", "launches")}
        d["seconds"] = t1 - t0
        runs.append(d)
    order = sorted(range(repeats), key=lambda q: runs[q]["seconds"])
    d = runs[order[repeats // 2]]
    d["runs_ms_per_step"] = [round(r["seconds"] / steps * 1e3, 3) for r in runs]
    d["issue_ms"] = s1["last_issue_ms"]
    d["max_call_ms"] = s1["max_call_ms"]
    d["max_call"] = {"ms": round(s1["max_call_ms"], 2), "kind": CALL_KINDS[min(s1["max_call_kind"], 5)],
                     "chains_before": s1["max_call_chain"]}
    d["ntiles"] = s1["ntiles_last"]
    d["tile_rows"] = s1["tile_rows"]
    d["slot_bytes"] = s1["slot_bytes"]
    d["kernels"] = {}
    if timing:
        ms, n, b = app.ctx.kernel_stats(dom)
        if n:
            d["kernels"][dom] = (ms, n, b)
        d["warmup_kernel_ms"] = {kid: v for kid, v in per.items() if v}
        app.ctx.set_timing(False)
    return d


def tile_stage_summary(app, steps=1, log_path=None):
    """One more, untimed chain of `steps` steps (the workload's chain length)
    with per-tile stage events on the three streams: the average duration per
    tile of the upload, compute, edge-copy and download stages, and the span
    of the chain from the first upload to the last download (ms), also per
    step."""
    app.ctx.set_tile_timing(True)
    app.run(steps)
    recs = app.ctx.tile_times()
    app.ctx.set_tile_timing(False)
    if not recs:
        return None
    if log_path:  # the raw per-tile records, one JSON object per line
        with open(log_path, "w") as fh:
            for r in recs:
                fh.write(json.dumps(r) + "\n")

    def avg(a, b):
        return round(sum(r[b] - r[a] for r in recs) / len(recs) / 1e3, 3)

    span = (max(r["d2h_end_us"] for r in recs) - min(r["h2d_begin_us"] for r in recs)) / 1e3
    return {"steps": steps, "tiles": len(recs), "h2d_ms": avg("h2d_begin_us", "h2d_end_us"),
            "compute_ms": avg("comp_begin_us", "comp_end_us"), "edge_ms": avg("comp_end_us", "edge_end_us"),
            "d2h_ms": avg("d2h_begin_us", "d2h_end_us"), "chain_span_ms": round(span, 2),
            "step_span_ms": round(span / steps, 2),
            # share of the span the compute stream is busy (compute + edge copy)
            "compute_busy_frac": round(sum(r["edge_end_us"] - r["comp_begin_us"] for r in recs) / 1e3 / span, 3)}


def ooc_ceiling(rate, cell_steps, bytes_hbm, bytes_h2d, bytes_d2h, hbm_GBs, h2d_GBs, d2h_GBs):
    """Out-of-core ceiling (an upper bound, grid-point updates/s): the slowest
    of HBM at the copy probe's rate over the algorithmic bytes, and of each
    link direction at its own probe's rate over the bytes it moves, per cell
    and step, as if the three streams overlapped perfectly.  (Both directions
    at once the runtime's copies reach less; the concurrent probe is reported
    beside it, not used here.)  `rate` is the measured updates/s; the result
    carries its fraction of the ceiling."""
    terms = {"hbm": hbm_GBs * 1e9 * cell_steps / bytes_hbm}
    if bytes_h2d:
        terms["h2d"] = h2d_GBs * 1e9 * cell_steps / bytes_h2d
    if bytes_d2h:
        terms["d2h"] = d2h_GBs * 1e9 * cell_steps / bytes_d2h
    bound = min(terms, key=terms.get)
    return {"value": terms[bound], "bound": bound, "terms": {k: round(v) for k, v in terms.items()},
            "frac": round(rate / terms[bound], 3)}


def roofline_of(r, knames, where):
    """Dominant kernel (most time) of a timed run: algorithmic bytes per
    launch / average launch time, against the HBM peak."""
    if not r["kernels"]:
        return None
    kid, (ms, n, b) = max(r["kernels"].items(), key=lambda kv: kv[1][0])
    avg_s = ms / n / 1e3
    achieved = b / n / avg_s / 1e9
    return {"bound": "hbm", "kernel": knames.get(kid, str(kid)), "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "bytes_per_launch": b // n, "avg_launch_us": round(avg_s * 1e6, 2), "launches": n,
            "measured_in": where}


def committed_traffic(kernel, workload, alg_bytes_per_launch):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size),
    used only while the kernel source still hashes to what was profiled and
    the launches process the same points (algorithmic bytes per launch within
    0.1 %: another tile shape reads other halos)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "%s_%s_traffic.txt" % (kernel, workload))
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    for key, hkey in (("source", "source_sha1"), ("point_loop_source", "point_loop_sha1")):
        if key not in kv:
            continue
        src = os.path.join(ROOT, "paper_1709_02125_amd", "csrc", kv[key])
        want = kv.get(hkey)
        if not os.path.exists(src) or hashlib.sha1(open(src, "rb").read()).hexdigest() != want:
            return None
    alg = float(kv.get("algorithmic_bytes_per_launch", 0))
    if not alg or abs(alg - alg_bytes_per_launch) > 1e-3 * alg:
        return None
    return float(kv["hbm_bytes_per_launch"])


def link_probe(nbytes=1 << 30):
    """Host-link peak as this machine delivers it: one pinned 1 GiB buffer copied
    to the device, then back, by the runtime (GB/s each way)."""
    import torch
    h = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    d = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    out = []
    for dst, src in ((d, h), (h, d)):
        dst.copy_(src, non_blocking=True)   # warm
        torch.cuda.synchronize()
        t = time.perf_counter()
        dst.copy_(src, non_blocking=True)
        torch.cuda.synchronize()
        out.append(round(nbytes / (time.perf_counter() - t) / 1e9, 2))
    del h, d
    return out


def hbm_copy_probe(nbytes=4 << 30, reps=3):
    """HBM bandwidth a plain device copy reaches here: 4 GiB copied by the
    runtime's copy kernel, (read + written bytes) / best time, GB/s."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    torch.cuda.empty_cache()
    return round(2 * nbytes / (best * 1e-3) / 1e9, 1)


def link_both_probe(nbytes=1 << 30):
    """Both link directions at once: 1 GiB up and 1 GiB down by the runtime on
    two streams, each direction's rate from events on its own stream (GB/s)."""
    import torch
    hu = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    hd = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    du = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dd = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    su, sd = torch.cuda.Stream(), torch.cuda.Stream()
    rates = None
    for _ in range(2):   # the first pass warms both paths
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        torch.cuda.synchronize()
        with torch.cuda.stream(su):
            ev[0].record()
            du.copy_(hu, non_blocking=True)
            ev[1].record()
        with torch.cuda.stream(sd):
            ev[2].record()
            hd.copy_(dd, non_blocking=True)
            ev[3].record()
        torch.cuda.synchronize()
        rates = (round(nbytes / (ev[0].elapsed_time(ev[1]) * 1e-3) / 1e9, 2),
                 round(nbytes / (ev[2].elapsed_time(ev[3]) * 1e-3) / 1e9, 2))
    del hu, hd, du, dd
    torch.cuda.empty_cache()
    return rates


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def copy_probe(nbytes=1 << 30, reps=3):
    """A plain device copy of known size (counter calibration for rocprofv3)."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def c5_main(args):
    """Configuration 5: the hydro2d (15360^2, 16e9 B) or ns3d (512^3, 1/3
    budget) grid with its streamed fields stored and moved as float32 (the
    hydro2d form keeps the read-only geometry resident), on the schedule the
    device-trained cost model proposes.  The model is trained on the timings
    of an exhaustive sweep of the FP64 form of the same grid (the schedule
    sweep configuration 4 records) and picks among the float32 form's
    schedules from their planned features alone; the exhaustive float32 sweep
    that follows is its yardstick (regret) and fallback.  The training set
    also holds a float32 sweep of a smaller grid at the same oversubscription
    (hydro2d 10240^2, ns3d 384^3): the FP64 hydro2d form is bound by its
    uploads whatever the slot count, and the FP64 ns3d form does not show
    the float32 form's penalty for short tiles, so FP64 timings alone do not
    carry what matters in float32.  The picked schedule
    then runs `--steps` steps from the initial state (the error of every state
    field against the FP64 oracle after those steps is stated) and, warmed,
    `--steps` more timed ones (the throughput)."""
    import torch
    import numpy as np
    from paper_1709_02125_amd import ooc, tune
    torch.cuda.set_device(0)
    f32 = ooc.FLAG_FP32_STREAM
    steps = args.steps or 20
    if args.workload == "ns3d":
        from paper_1709_02125_amd import ns3d as N
        from paper_1709_02125_amd.inputs import tgv_initial_state
        n = args.n or 512
        fused = ns_form(args)
        ring = 0 if args.slots_mode else ooc.FLAG_RING
        budget = int(args.budget) if args.budget else N.footprint_bytes(n, fused) // 3
        # with two copies of the conserved variables a chain spans an even
        # number of steps (the state returns to the copy it started in)
        cands = tune.grid([8, 16, 24, 32, 48, 0], [2, 4] if fused == "q" else [1, 2, 3, 4], [2, 3, 4])
        dl = ooc.FLAG_MEMCPY_DOWNLOAD  # the chain is bound by its kernels
        workload = lambda fl: tune.ns3d_workload(n, budget, fl | ring | dl, fused=fused)
        cells = n ** 3
        names = N.Q

        def fresh(h, k, S):
            app = N.NS3D(n, tgv_initial_state(n), budget=budget, flags=ooc.FLAG_PREFETCH | f32 | ring | dl,
                         fused=fused)
            app.ctx.set_schedule(tile_rows=h, chain_steps=k, slots=S)
            return app

        def incore():
            return N.NS3D(n, tgv_initial_state(n), budget=N.device_footprint_bytes(n, fused), flags=ooc.FLAG_INCORE,
                          fused=fused)

        def oracle_state():
            import oracle.ns3d as on
            o = on.NS3D(n)
            o.set_primitives(*tgv_initial_state(n))
            for q in range(steps):
                o.step(on.stable_dt(n))
                log("oracle ns3d step", q + 1)
            out = {x: o.interior(x).copy() for x in names}
            del o
            return out

        got_state = lambda app: {x: app.interior(x) for x in names}
        n_small = n * 3 // 4 // 32 * 32
        small = (n_small, lambda fl: tune.ns3d_workload(n_small, N.footprint_bytes(n_small, fused) // 3, fl | ring | dl,
                                                         fused=fused),
                 N.footprint_bytes(n_small, fused) // 3)
        form = ("ns3d proxy %d^3 (Taylor-Green, Mach 0.1), %d fields, conserved fields stored and streamed as "
                "float32, compute in FP64, %s, device budget %.3g B (1/3 of the FP64 fields)" %
                (n, 15 if fused else 27, "ring slabs" if ring else "slots with edge copies", budget))
    else:
        from paper_1709_02125_amd import hydro2d as h2
        from paper_1709_02125_amd.inputs import hydro_initial_state
        n = args.n or 15360
        budget = int(args.budget) if args.budget else 16_000_000_000
        cands = tune.grid([384, 768, 1152, 1536, 0], [1], [2, 3, 4])
        workload = lambda fl: tune.hydro2d_workload(n, budget, fl, resident_geometry=bool(fl & f32))
        cells = n * n
        names = ("rho0", "e0", "u0", "v0")
        n_small = n * 2 // 3 // 128 * 128
        small = (n_small, lambda fl: tune.hydro2d_workload(n_small, budget * n_small ** 2 // n ** 2, fl,
                                                            resident_geometry=True),
                 budget * n_small ** 2 // n ** 2)

        def fresh(h, k, S):
            rho, ene = hydro_initial_state((n, n))
            app = h2.Hydro2D(n, n, rho, ene, budget=budget, flags=ooc.FLAG_PREFETCH | f32, resident_geometry=True)
            app.ctx.set_schedule(tile_rows=h, slots=S)
            return app

        def incore():
            rho, ene = hydro_initial_state((n, n))
            return h2.Hydro2D(n, n, rho, ene, budget=h2.device_footprint_bytes(n, n), flags=ooc.FLAG_INCORE)

        def oracle_state():
            import oracle.hydro2d as oh
            rho, ene = hydro_initial_state((n, n))
            o = oh.Hydro2D(n, n)
            o.set_state(rho, ene)
            del rho, ene
            dt = o.dt()
            for q in range(steps):
                dt = o.step(dt)
                log("oracle hydro2d step", q + 1)
            out = {x: o.interior(x, x in ("u0", "v0")).copy() for x in names}
            del o
            return out

        got_state = lambda app: {x: app.interior(x) for x in names}
        form = ("hydro2d proxy %dx%d, state fields stored and streamed as float32, geometry resident, compute "
                "in FP64, device budget %.3g B" % (n, n, budget))

    def run_sweep(fl, what, wl=workload, bud=budget):
        t = time.perf_counter()
        app, plan_ctx, q, cl, rb = wl(fl)
        recs = tune.sweep(app, plan_ctx, q, cl, rb, bud, cands, chains=3, repeats=2,
                          log=lambda m: log("%s sweep: %s" % (what, m)))
        app.close()
        del app
        torch.cuda.empty_cache()
        log("%s sweep: %d schedules, %.0f s" % (what, len(recs), time.perf_counter() - t))
        return recs

    train_fp64 = run_sweep(0, "FP64 (training)")
    train_small = run_sweep(f32, "FP32 %d (training)" % small[0], small[1], small[2]) if small else []
    train = train_fp64 + train_small
    target = run_sweep(f32, "FP32 (yardstick)")
    picks = [tune.transfer_regret(train, target, seed=seed) for seed in (1709, 1, 2)]
    for r in picks:
        log("cost model pick %s: regret %.3f, gain over default %s" % (r["pick"], r["regret"],
                                                                       r["gain_over_default"]))
    # the schedule run below: the pick of the three models together
    ens = tune.ensemble_transfer_regret(train, target, seeds=(1709, 1, 2))
    log("three-model cost model pick %s: regret %.3f, gain over default %s" % (ens["pick"], ens["regret"],
                                                                               ens["gain_over_default"]))
    h, k, S = ens["pick"]

    # the picked schedule from the initial state: error after `steps` steps,
    # then warmed, `steps` timed steps
    app = fresh(h, k, S)
    app.initialise()
    app.run(steps)
    got = got_state(app)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    app.run(steps)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    st = app.ctx.stats()
    app.close()
    del app
    torch.cuda.empty_cache()
    rate = cells * steps / sec
    log("C5 picked schedule h=%d k=%d S=%d: %.3f s/step, %.3g upd/s" % (h, k, S, sec / steps, rate))
    app = incore()
    app.initialise()
    app.run(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    app.run(steps)
    torch.cuda.synchronize()
    inc_sec = time.perf_counter() - t0
    app.close()
    del app
    torch.cuda.empty_cache()
    ref = oracle_state()
    errs = {}
    for x in names:
        m = float(np.abs(ref[x]).max())
        errs[x] = float(np.abs(got[x] - ref[x]).max() / m) if m else float(np.abs(got[x]).max())
        log("FP32 stream error after %d steps, %s: %.3e" % (steps, x, errs[x]))
    inc_rate = cells * steps / inc_sec
    out = {"metric": METRIC, "value": rate, "unit": "grid-point updates/s", "n_gpus": 1, "steps": steps,
           "warmup": steps, "ms_per_step": round(sec / steps * 1e3, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": form, "cells": cells, "schedule": {"tile_rows": h, "chain_steps": k, "slots": S},
                      "tiles": st["ntiles_last"],
                      "picked_by": "cost model trained on the FP64 sweep" +
                                   (" and the FP32 sweep at %d cells per axis" % small[0] if small else "")},
           "incore_value": inc_rate, "pct_of_incore": round(100.0 * rate / inc_rate, 2),
           "incore_ms_per_step": round(inc_sec / steps * 1e3, 3),
           "cost_model": {"picks": picks, "ensemble": ens, "train_schedules": len(train),
                          "target_schedules": len(target)},
           "sweep_fp64": [{k_: r[k_] for k_ in ("h", "k", "S", "sec_per_cell_step")} for r in train_fp64],
           "sweep_fp32_small": [{k_: r[k_] for k_ in ("h", "k", "S", "sec_per_cell_step")} for r in train_small],
           "sweep_fp32": [{k_: r[k_] for k_ in ("h", "k", "S", "sec_per_cell_step")} for r in target],
           "fp32_error_vs_fp64_oracle": {"steps": steps, "max_rel_err": errs}}
    if args.c5_records:
        with open(args.c5_records, "w") as fh:
            json.dump({"train": train, "target": target, "features": tune.FEATURE_NAMES}, fh)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 20 for hydro2d, 10 for hydro3d, two chains for ns3d)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--repeats", type=int, default=3,
                    help="timed runs of --steps steps each for the headline and in-core rates (median reported)")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="hydro2d")
    ap.add_argument("--n", type=int, default=0, help="cells per axis (default: the workload's size)")
    ap.add_argument("--budget", type=float, default=0, help="device bytes (default: the workload's budget)")
    ap.add_argument("--resident-geometry", action="store_true")
    ap.add_argument("--resident-state", action="store_true",
                    help="hydro: keep geometry and state on the device; only temporaries are tiled")
    ap.add_argument("--fp32", action="store_true", help="store and stream fields as float32 on the host")
    ap.add_argument("--no-prefetch", action="store_true")
    ap.add_argument("--kernel-copy", action="store_true", help="host-link transfers by copy kernel")
    ap.add_argument("--download", choices=["kernel", "memcpy"], default=None,
                    help="downloads by the library's copy kernel or by runtime memcpy calls; default: memcpy "
                         "for ns3d (kernel-bound chains), the copy kernel for the hydro proxies")
    ap.add_argument("--fuse", action="store_true", help="fuse independent strip loops per tile")
    ap.add_argument("--no-cyclic", action="store_true")
    ap.add_argument("--no-incore", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--slots", type=int, default=None, help="slot count (default 3; ns3d with stored gradients: 2)")
    ap.add_argument("--tile-rows", type=int, default=None, help="tile height (default: the planner's, the largest that fits, "
                         "on ring slabs the tallest whose chain boundaries stay clear; ns3d with stored gradients: 24)")
    ap.add_argument("--chain-steps", type=int, default=4, help="ns3d: time steps per chain")
    ap.add_argument("--slots-mode", action="store_true",
                    help="ns3d: the paper's per-tile slots with edge copies instead of ring slabs (the default "
                         "for ns3d)")
    ap.add_argument("--ring", action="store_true", help="hydro proxies: ring slabs instead of slots")
    ap.add_argument("--cache-tiling", type=int, nargs="*", default=None,
                    help="also time the in-core run cut into tiles of these heights (cache blocking, no transfers)")
    ap.add_argument("--stored-primitives", action="store_true",
                    help="ns3d: the 15-field chain with a primitives loop and stored primitives (the default "
                         "form evaluates them in the residual kernel from two copies of the conserved variables, "
                         "which needs chains of an even number of steps)")
    ap.add_argument("--stored-gradients", action="store_true",
                    help="ns3d: the 27-field chain with a gradient loop and stored gradients (default: the "
                         "15-field chain whose residual evaluates the gradients itself)")
    ap.add_argument("--no-variants", action="store_true", help="skip the other schedules of the same grid")
    ap.add_argument("--tile-log", default=None,
                    help="write the per-tile stage records of the staged chain to this file (JSON lines, us)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="end with a plain 1 GiB device copy (counter calibration under rocprofv3)")
    ap.add_argument("--c5", action="store_true",
                    help="configuration 5 for --workload hydro2d or ns3d: float32 streaming on the schedule the "
                         "cost model proposes (trained on the FP64 sweep), regret against the float32 sweep, "
                         "error against the FP64 oracle")
    ap.add_argument("--c5-records", default=None, help="write the two sweeps' records (with features) here")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the pipeline runs on a single MI355X "
              "(the multi-GPU sharding is a design note only); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.c5:
        if args.workload == "hydro3d":
            print("configuration 5 covers hydro2d and ns3d", file=sys.stderr)
            sys.exit(2)
        return c5_main(args)
    if args.steps is None:  # ns3d: two whole chains
        args.steps = {"hydro2d": 20, "hydro3d": 10, "ns3d": 2 * args.chain_steps}[args.workload]
    # ns3d runs the form with the primitives and gradients evaluated in the
    # residual kernel, on ring slabs with chains of 4 steps, the planner's
    # tile and 3 slots (42.5 ms per step over two chains).  With stored
    # primitives the same schedule was within 1 % of the fastest of the
    # exhaustive sweep (tile heights 8 .. largest, chains of 1 .. 4 steps,
    # 2 .. 4 slots); with stored gradients on slots, 24-plane tiles, chains
    # of 3 steps and 2 slots were the fastest.  The hydro proxies default to
    # the largest tile and 3 slots.
    ns = args.workload == "ns3d"
    if ns and ns_form(args) == "q" and args.chain_steps % 2 and not args.no_cyclic:
        print("the default ns3d form keeps two copies of the conserved variables: under Cyclic its chains "
              "span an even number of steps (--chain-steps 2 or 4), or use --stored-primitives", file=sys.stderr)
        sys.exit(2)
    if args.slots is None:
        args.slots = 3 if ns and not args.stored_gradients else (2 if ns else 0)
    if args.tile_rows is None:
        args.tile_rows = 24 if ns and args.stored_gradients else 0

    import torch
    from paper_1709_02125_amd import ooc
    torch.cuda.set_device(0)
    w = WORKLOADS[args.workload](args)

    # ---- out of core: budget capped, tiles streamed through HBM
    flags = 0 if args.no_prefetch else ooc.FLAG_PREFETCH
    if args.ring or (ns and not args.slots_mode):
        flags |= ooc.FLAG_RING
    if args.fp32:
        flags |= ooc.FLAG_FP32_STREAM
    if args.kernel_copy:
        flags |= ooc.FLAG_KERNEL_COPY
    if args.download is None:  # runtime copies where the stencils bound the chain
        args.download = "memcpy" if ns else "kernel"
    if args.download == "memcpy":
        flags |= ooc.FLAG_MEMCPY_DOWNLOAD
    if args.fuse:
        flags |= ooc.FLAG_FUSE
    t = time.perf_counter()
    app = w.make(w.budget, flags)
    if args.workload != "ns3d" and (args.slots or args.tile_rows):
        app.ctx.set_schedule(tile_rows=args.tile_rows, slots=args.slots)
    app.initialise()
    log("out-of-core setup %.1f s" % (time.perf_counter() - t))
    args.warmup = w.warmup_steps(args.warmup, args.steps) if hasattr(w, "warmup_steps") else args.warmup
    ooc_r = timed_run(app, args.steps, args.warmup, w.knames, w.dominant, repeats=args.repeats)
    tile_stages = tile_stage_summary(app, args.chain_steps if args.workload == "ns3d" else 1, args.tile_log)
    app.close()
    del app
    torch.cuda.empty_cache()
    ooc_rate = w.cells * args.steps / ooc_r["seconds"]
    log("out-of-core: %.3f s/step (median of %s ms), %.3g upd/s, tiles %d x %d rows, host issue %.1f ms "
        "(max call %.2f ms: %s, after %d chains)" %
        (ooc_r["seconds"] / args.steps, ooc_r["runs_ms_per_step"], ooc_rate, ooc_r["ntiles"], ooc_r["tile_rows"],
         ooc_r["issue_ms"], ooc_r["max_call_ms"], ooc_r["max_call"]["kind"], ooc_r["max_call"]["chains_before"]))

    # ---- in core: same grid and kernels, every field resident
    inc_rate, inc_r = None, None
    if not args.no_incore:
        t = time.perf_counter()
        app = w.make(0, ooc.FLAG_INCORE, incore=True)
        app.initialise()
        log("in-core setup %.1f s" % (time.perf_counter() - t))
        inc_r = timed_run(app, args.steps, args.warmup, w.knames, w.dominant, repeats=args.repeats)
        app.close()
        del app
        torch.cuda.empty_cache()
        inc_rate = w.cells * args.steps / inc_r["seconds"]
        log("in-core: %.3f s/step, %.3g upd/s" % (inc_r["seconds"] / args.steps, inc_rate))

    # ---- other schedules of the same grid and budget (not the headline)
    variants = {}
    if not args.no_variants:
        vlist = list(w.variants())
        if args.cache_tiling:
            # every field resident, the chain still cut into skewed tiles of
            # this many rows (planes), so a tile's rows can be reused from the
            # caches across the chain's loops
            vlist += [("incore_cache_tiled_%d" % h, ooc.FLAG_INCORE, {"incore_tile_rows": h})
                      for h in args.cache_tiling]
        for vname, vflags, vopts in vlist:
            t = time.perf_counter()
            if "incore_tile_rows" in vopts:
                app = w.make(0, vflags, incore=True)
                app.ctx.set_schedule(tile_rows=vopts["incore_tile_rows"], chain_steps=args.chain_steps if ns else 0,
                                     slots=args.slots)
            else:
                app = w.make(w.budget, vflags, **vopts)
            try:
                app.initialise()
                runner = summary_runner(app, *vopts["summary"]) if "summary" in vopts else None
                r = timed_run(app, args.steps, args.warmup, w.knames, timing=False, run=runner)
            except ooc.OocError as e:
                if e.code != ooc.E_BUDGET:
                    raise
                variants[vname] = {"infeasible": str(e)}  # the schedule does not fit this form's budget
                log("variant %s: %s" % (vname, e))
                continue
            finally:
                app.close()
                del app
                torch.cuda.empty_cache()
            rate = w.cells * args.steps / r["seconds"]
            variants[vname] = {"value": rate, "ms_per_step": round(r["seconds"] / args.steps * 1e3, 3),
                               "pct_of_incore": round(100.0 * rate / inc_rate, 2) if inc_rate else None,
                               "h2d_GBs": round(r["bytes_h2d"] / r["seconds"] / 1e9, 2),
                               "d2h_GBs": round(r["bytes_d2h"] / r["seconds"] / 1e9, 2),
                               "tiles": r["ntiles"], "tile_rows": r["tile_rows"]}
            if "summary" in vopts:
                variants[vname]["ms_per_step_over_headline"] = round(
                    (r["seconds"] - ooc_r["seconds"]) / args.steps * 1e3, 3)
            log("variant %s: %.3f s/step, %.3g upd/s (setup+run %.1f s)" %
                (vname, r["seconds"] / args.steps, rate, time.perf_counter() - t))
    if args.copy_probe:
        copy_probe()

    roofline = roofline_of(ooc_r, w.knames, "out-of-core timed steps")
    if roofline:
        roofline["traffic"] = committed_traffic(roofline["kernel"], args.workload, roofline["bytes_per_launch"])
    incore_roofline = roofline_of(inc_r, w.knames, "in-core timed steps") if inc_r else None
    probe_h2d, probe_d2h = link_probe()
    both_h2d, both_d2h = link_both_probe()
    hbm_copy = hbm_copy_probe()
    if roofline:
        roofline["copy_probe_GBs"] = hbm_copy
    link = {"h2d_GBs": round(ooc_r["bytes_h2d"] / ooc_r["seconds"] / 1e9, 2),
            "d2h_GBs": round(ooc_r["bytes_d2h"] / ooc_r["seconds"] / 1e9, 2),
            "peak_per_direction_GBs": LINK_PEAK_GBS,
            "probe_h2d_GBs": probe_h2d, "probe_d2h_GBs": probe_d2h,
            "probe_both_h2d_GBs": both_h2d, "probe_both_d2h_GBs": both_d2h,
            "h2d_frac_of_probe": round(ooc_r["bytes_h2d"] / ooc_r["seconds"] / 1e9 / probe_h2d, 3),
            "h2d_bytes_per_step": ooc_r["bytes_h2d"] // args.steps,
            "d2h_bytes_per_step": ooc_r["bytes_d2h"] // args.steps,
            "edge_bytes_per_step": ooc_r["bytes_edge"] // args.steps}
    avg_bw = ooc_r["bytes_hbm_alg"] / ooc_r["seconds"] / 1e9
    ceiling = ooc_ceiling(ooc_rate, w.cells * args.steps, ooc_r["bytes_hbm_alg"], ooc_r["bytes_h2d"],
                          ooc_r["bytes_d2h"], hbm_copy, probe_h2d, probe_d2h)

    cpu = None
    if not args.no_cpu:
        import oracle
        val, sample = w.cpu_baseline()
        cpu = {"value": val, "unit": "grid-point updates/s", "cores": int(oracle.load().oracle_threads()),
               "kind": "oracle", "sample": sample, "cpu_model": cpu_model(), "nproc": os.cpu_count(),
               "affinity_cpus": len(os.sched_getaffinity(0)),
               "one_thread": cpu_one_thread(args.workload, args.n)}
        log("cpu oracle: %.3g upd/s on %d threads; one thread: %s" % (cpu["value"], cpu["cores"],
                                                                     cpu["one_thread"]))

    ms_step = ooc_r["seconds"] / args.steps * 1e3
    config = {"workload": w.describe(), "cells": w.cells,
              "prefetch": not args.no_prefetch, "cyclic": not args.no_cyclic,
              "resident_geometry": args.resident_geometry, "resident_state": args.resident_state,
              "fp32_stream": args.fp32,
              "kernel_copy": args.kernel_copy, "downloads": args.download, "fuse": args.fuse,
              "tiles": ooc_r["ntiles"],
              "tile_rows": ooc_r["tile_rows"], "slots": args.slots or 3}
    if args.workload == "ns3d":
        config["chain_steps"] = args.chain_steps
    out = {
        "metric": METRIC,
        "value": ooc_rate, "unit": "grid-point updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": config,
        "incore_value": inc_rate,
        "pct_of_incore": round(100.0 * ooc_rate / inc_rate, 2) if inc_rate else None,
        "incore_ms_per_step": round(inc_r["seconds"] / args.steps * 1e3, 3) if inc_r else None,
        "runs_ms_per_step": ooc_r["runs_ms_per_step"],
        "incore_runs_ms_per_step": inc_r["runs_ms_per_step"] if inc_r else None,
        "max_runtime_call": ooc_r["max_call"],
        "average_bandwidth_GBs": round(avg_bw, 1),
        "alg_bytes_per_cell_step": round(ooc_r["bytes_hbm_alg"] / (w.cells * args.steps), 1),
        "roofline": roofline,
        "incore_roofline": incore_roofline,
        "link": link,
        "ooc_ceiling": ceiling,
        "variants": variants,
        "cpu_baseline": cpu,
        "ooc_tile_stages": tile_stages,
        "ooc_warmup_kernel_ms": {w.knames[k]: round(v, 2) for k, v in ooc_r.get("warmup_kernel_ms", {}).items()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
