"""Benchmark: grid-point updates/s of a stencil chain whose fields are about 3x
the device budget, streamed tile by tile through HBM by the HIP library;
beside it the same grid fully resident (in-core), the dominant kernel's HBM
roofline, the host-link throughput, and the CPU oracle timed on a sample.

Workloads (one step = one time step over the whole grid):
  hydro2d (default)  15360 x 15360 FP64, 25 fields, 55-loop chain, budget 16e9 B
  hydro3d            640^3 FP64, 30 fields, 82-loop chain, budget 1/3 of the fields
  ns3d               512^3 FP64, 27 fields, 45 loops per step, budget 1/3 of the fields,
                     chains of --chain-steps steps
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
NS_NAMES = ["ns_init", "ns_prims", "ns_grads", "ns_rhs_first", "ns_rhs"]
COMMON = {1: "mirror", 2: "fill", 3: "sum_prod"}


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

    def make(self, budget, flags, incore=False):
        h2 = self.mod
        if incore:
            return h2.Hydro2D(self.n, self.n, self.rho, self.ene, budget=h2.device_footprint_bytes(self.n, self.n),
                              flags=flags)
        return h2.Hydro2D(self.n, self.n, self.rho, self.ene, budget=budget, flags=flags,
                          resident_geometry=self.args.resident_geometry, cyclic_after_init=not self.args.no_cyclic,
                          resident_state=self.args.resident_state)

    def describe(self):
        return ("hydro2d proxy %dx%d FP64, 25 fields, 55-loop chain per step, device budget %.3g B "
                "(footprint %.3g B, %.2fx oversubscribed), tiles along y" %
                (self.n, self.n, self.budget, self.footprint, self.footprint / self.budget))

    def cpu_baseline(self, target_s=12.0):
        import oracle
        import oracle.hydro2d as oh
        from paper_1709_02125_amd.inputs import hydro_initial_state
        oracle.build(force=False)
        nx, ny = self.n, 1024
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

    def make(self, budget, flags, incore=False):
        h3 = self.mod
        if incore:
            return h3.Hydro3D(self.dims, self.rho, self.ene, budget=h3.device_footprint_bytes(self.dims),
                              flags=flags)
        return h3.Hydro3D(self.dims, self.rho, self.ene, budget=budget, flags=flags,
                          resident_geometry=self.args.resident_geometry, cyclic_after_init=not self.args.no_cyclic,
                          resident_state=self.args.resident_state)

    def describe(self):
        return ("hydro3d proxy %d^3 FP64, 30 fields, 82-loop chain per step, device budget %.3g B "
                "(footprint %.3g B, %.2fx oversubscribed), tiles along z" %
                (self.n, self.budget, self.footprint, self.footprint / self.budget))

    def cpu_baseline(self, target_s=12.0):
        import oracle
        import oracle.hydro3d as oh
        from paper_1709_02125_amd.inputs import hydro_initial_state
        oracle.build(force=False)
        dims = (self.n, self.n, 8)
        rho, ene = hydro_initial_state(dims)
        o = oh.Hydro3D(*dims)
        o.set_state(rho, ene)
        dt = o.dt()
        steps, t0 = 0, time.perf_counter()
        while steps < 10 and (time.perf_counter() - t0) < target_s:
            dt = o.step(dt)
            steps += 1
        sec = time.perf_counter() - t0
        cells = dims[0] * dims[1] * dims[2]
        return cells * steps / sec, "%d x %d x %d cells (a z-slab of the benchmark grid), %d steps, %.1f s" % (
            dims + (steps, sec))


class NS3DWork(Workload):
    def __init__(self, args):
        super().__init__(args)
        from paper_1709_02125_amd import ns3d as N
        from paper_1709_02125_amd.inputs import tgv_initial_state
        self.mod = N
        self.n = args.n or 512
        self.cells = self.n ** 3
        self.footprint = N.footprint_bytes(self.n)
        self.budget = int(args.budget) if args.budget else self.footprint // 3
        log("generating input %d^3" % self.n)
        self.prims = tgv_initial_state(self.n)
        self.knames = {**COMMON, **{200 + i: s for i, s in enumerate(NS_NAMES)}}

    def make(self, budget, flags, incore=False):
        N = self.mod
        if incore:
            return N.NS3D(self.n, self.prims, budget=N.device_footprint_bytes(self.n), flags=flags)
        app = N.NS3D(self.n, self.prims, budget=budget, flags=flags, cyclic_after_init=not self.args.no_cyclic)
        return app

    def schedule(self, app):
        app.ctx.set_schedule(tile_rows=self.args.tile_rows, chain_steps=self.args.chain_steps,
                             slots=self.args.slots)

    def describe(self):
        return ("ns3d proxy %d^3 FP64 (Taylor-Green, Mach 0.1), 27 fields, 45 loops per step, chains of %d "
                "steps, device budget %.3g B (footprint %.3g B, %.2fx oversubscribed), tiles along z" %
                (self.n, self.args.chain_steps, self.budget, self.footprint, self.footprint / self.budget))

    def cpu_baseline(self, target_s=12.0):
        import oracle
        import oracle.ns3d as on
        from paper_1709_02125_amd.inputs import tgv_initial_state
        oracle.build(force=False)
        n = 128
        o = on.NS3D(n)
        o.set_primitives(*tgv_initial_state(n))
        dt = on.stable_dt(n)
        steps, t0 = 0, time.perf_counter()
        while steps < 10 and (time.perf_counter() - t0) < target_s:
            o.step(dt)
            steps += 1
        sec = time.perf_counter() - t0
        return n ** 3 * steps / sec, "%d^3 points, %d steps, %.1f s" % (n, steps, sec)


WORKLOADS = {"hydro2d": Hydro2DWork, "hydro3d": Hydro3DWork, "ns3d": NS3DWork}


def timed_run(app, steps, warmup, timing):
    """Warm up, then time `steps` steps with wall clock between device syncs.
    With timing, a further pass of `timing` steps records every launch with
    hipEvents on the compute stream (kept out of the timed region)."""
    import torch
    app.run(warmup)
    app.ctx.set_timing(False)
    s0 = app.ctx.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    app.run(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s1 = app.ctx.stats()
    d = {k: s1[k] - s0[k] for k in ("bytes_h2d", "bytes_d2h", "bytes_edge", "bytes_hbm_alg", "tiles", "chains",
                                     "launches")}
    d["seconds"] = t1 - t0
    d["issue_ms"] = s1["last_issue_ms"]
    d["max_call_ms"] = s1["max_call_ms"]
    if timing:
        app.ctx.set_timing(True)
        app.run(timing)
    d["ntiles"] = s1["ntiles_last"]
    d["tile_rows"] = s1["tile_rows"]
    d["slot_bytes"] = s1["slot_bytes"]
    return d


def dominant_kernel(app, knames):
    best = None
    for kid in knames:
        ms, n, b = app.ctx.kernel_stats(kid)
        if n and (best is None or ms > best[1]):
            best = (kid, ms, n, b)
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 20; 10 for the 3D workloads)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="hydro2d")
    ap.add_argument("--n", type=int, default=0, help="cells per axis (default: the workload's size)")
    ap.add_argument("--budget", type=float, default=0, help="device bytes (default: the workload's budget)")
    ap.add_argument("--resident-geometry", action="store_true")
    ap.add_argument("--resident-state", action="store_true",
                    help="hydro: keep geometry and state on the device; only temporaries are tiled")
    ap.add_argument("--fp32", action="store_true", help="store and stream fields as float32 on the host")
    ap.add_argument("--no-prefetch", action="store_true")
    ap.add_argument("--kernel-copy", action="store_true", help="host-link transfers by copy kernel")
    ap.add_argument("--fuse", action="store_true", help="fuse independent strip loops per tile")
    ap.add_argument("--no-cyclic", action="store_true")
    ap.add_argument("--no-incore", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--slots", type=int, default=0)
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--chain-steps", type=int, default=2, help="ns3d: time steps per chain")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build's path runs on a single MI355X "
              "(the multi-GPU sharding is a design note only); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.steps is None:
        args.steps = 20 if args.workload == "hydro2d" else 10

    import torch
    from paper_1709_02125_amd import ooc
    torch.cuda.set_device(0)
    w = WORKLOADS[args.workload](args)

    # ---- out of core: budget capped, tiles streamed through HBM
    flags = 0 if args.no_prefetch else ooc.FLAG_PREFETCH
    if args.fp32:
        flags |= ooc.FLAG_FP32_STREAM
    if args.kernel_copy:
        flags |= ooc.FLAG_KERNEL_COPY
    if args.fuse:
        flags |= ooc.FLAG_FUSE
    t = time.perf_counter()
    app = w.make(w.budget, flags)
    if hasattr(w, "schedule"):
        w.schedule(app)
    elif args.slots or args.tile_rows:
        app.ctx.set_schedule(tile_rows=args.tile_rows, slots=args.slots)
    app.initialise()
    log("out-of-core setup %.1f s" % (time.perf_counter() - t))
    ooc_r = timed_run(app, args.steps, args.warmup, timing=2)
    ooc_dom = dominant_kernel(app, w.knames)
    ooc_kernel_ms = {w.knames[k]: app.ctx.kernel_stats(k)[0] for k in w.knames}
    app.close()
    del app
    torch.cuda.empty_cache()
    ooc_rate = w.cells * args.steps / ooc_r["seconds"]
    log("out-of-core: %.3f s/step, %.3g upd/s, tiles %d x %d rows, host issue %.1f ms (max call %.2f ms)" %
        (ooc_r["seconds"] / args.steps, ooc_rate, ooc_r["ntiles"], ooc_r["tile_rows"], ooc_r["issue_ms"],
         ooc_r["max_call_ms"]))

    # ---- in core: same grid and kernels, every field resident
    inc_rate, inc_r, dom = None, None, ooc_dom
    if not args.no_incore:
        t = time.perf_counter()
        app = w.make(0, ooc.FLAG_INCORE, incore=True)
        app.initialise()
        log("in-core setup %.1f s" % (time.perf_counter() - t))
        inc_r = timed_run(app, args.steps, args.warmup, timing=5)
        dom = dominant_kernel(app, w.knames)
        app.close()
        del app
        torch.cuda.empty_cache()
        inc_rate = w.cells * args.steps / inc_r["seconds"]
        log("in-core: %.3f s/step, %.3g upd/s" % (inc_r["seconds"] / args.steps, inc_rate))

    kid, kms, kn, kbytes = dom
    avg_s = kms / kn / 1e3
    achieved = kbytes / kn / avg_s / 1e9
    roofline = {"bound": "hbm", "kernel": w.knames.get(kid, str(kid)), "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None, "bytes_per_launch": kbytes // kn, "avg_launch_us": round(avg_s * 1e6, 2),
                "launches": kn, "measured_in": "in-core" if inc_r else "out-of-core"}
    link = {"h2d_GBs": round(ooc_r["bytes_h2d"] / ooc_r["seconds"] / 1e9, 2),
            "d2h_GBs": round(ooc_r["bytes_d2h"] / ooc_r["seconds"] / 1e9, 2),
            "peak_per_direction_GBs": LINK_PEAK_GBS,
            "h2d_bytes_per_step": ooc_r["bytes_h2d"] // args.steps,
            "d2h_bytes_per_step": ooc_r["bytes_d2h"] // args.steps,
            "edge_bytes_per_step": ooc_r["bytes_edge"] // args.steps}
    avg_bw = ooc_r["bytes_hbm_alg"] / ooc_r["seconds"] / 1e9

    cpu = None
    if not args.no_cpu:
        import oracle
        val, sample = w.cpu_baseline()
        cpu = {"value": val, "unit": "grid-point updates/s", "cores": int(oracle.load().oracle_threads()),
               "kind": "oracle", "sample": sample}
        log("cpu oracle: %.3g upd/s on %d threads" % (cpu["value"], cpu["cores"]))

    ms_step = ooc_r["seconds"] / args.steps * 1e3
    config = {"workload": w.describe(), "global_batch": w.cells, "seq_len": 1, "parallelism": "single-gpu",
              "prefetch": not args.no_prefetch, "cyclic": not args.no_cyclic,
              "resident_geometry": args.resident_geometry, "resident_state": args.resident_state,
              "fp32_stream": args.fp32,
              "kernel_copy": args.kernel_copy, "fuse": args.fuse, "tiles": ooc_r["ntiles"],
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
        "average_bandwidth_GBs": round(avg_bw, 1),
        "alg_bytes_per_cell_step": round(ooc_r["bytes_hbm_alg"] / (w.cells * args.steps), 1),
        "roofline": roofline,
        "link": link,
        "cpu_baseline": cpu,
        "ooc_kernel_ms": {k: round(v, 2) for k, v in ooc_kernel_ms.items() if v},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
