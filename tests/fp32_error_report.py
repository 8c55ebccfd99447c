"""Full-size statement of the FP32-streaming error: the HIP path with streamed
fields stored on the host and moved over the link as float32 (compute, sums
and the time step stay FP64 on the device) against the FP64 CPU oracle on the
same seeded input, after 20 steps; per-field max relative error (max |g - o| /
max |o| over the interior) printed as one JSON line.

Not collected by pytest (a one-off measurement at the benchmark sizes, minutes
of CPU time for the oracle).  On an MI355X:
    python tests/fp32_error_report.py --hydro2d   # 15360^2, budget 16e9 B
    python tests/fp32_error_report.py --ns3d      # 512^3, budget 1/3 of the fields
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel(g, o):
    m = np.abs(o).max()
    return float(np.abs(g - o).max() / m) if m else float(np.abs(g).max())


def hydro2d(n, steps, budget):
    import oracle.hydro2d as oh
    from paper_1709_02125_amd import hydro2d as h2, ooc
    from paper_1709_02125_amd.inputs import hydro_initial_state
    rho, ene = hydro_initial_state((n, n))
    t = time.perf_counter()
    app = h2.Hydro2D(n, n, rho, ene, budget=budget, flags=ooc.FLAG_FP32_STREAM | ooc.FLAG_PREFETCH,
                     resident_geometry=True)
    app.initialise()
    for s in range(steps):
        app.queue_step()
        app.ctx.submit()
    app.ctx.execute()
    got = {f: app.interior(f) for f in ("rho0", "e0", "u0", "v0")}
    app.close()
    say("gpu done %.1f s" % (time.perf_counter() - t))
    o = oh.Hydro2D(n, n)
    o.set_state(rho, ene)
    dt = o.dt()
    for s in range(steps):
        dt = o.step(dt)
        say("oracle step", s + 1)
    out = {}
    for f in got:
        ref = o.interior(f, node=f in ("u0", "v0"))
        out[f] = rel(got[f], ref)
    return out


def ns3d(n, steps, budget):
    import oracle.ns3d as on
    from paper_1709_02125_amd import ns3d as N, ooc
    from paper_1709_02125_amd.inputs import tgv_initial_state
    prims = tgv_initial_state(n)
    t = time.perf_counter()
    app = N.NS3D(n, prims, budget=budget, flags=ooc.FLAG_FP32_STREAM | ooc.FLAG_PREFETCH)
    app.ctx.set_schedule(chain_steps=2)
    app.initialise()
    app.run(steps)
    got = {q: app.interior(q) for q in N.Q}
    app.close()
    say("gpu done %.1f s" % (time.perf_counter() - t))
    o = on.NS3D(n)
    o.set_primitives(*prims)
    for s in range(steps):
        o.step(on.stable_dt(n))
        say("oracle step", s + 1)
    return {q: rel(got[q], o.interior(q)) for q in N.Q}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--hydro2d", action="store_true")
    ap.add_argument("--ns3d", action="store_true")
    ap.add_argument("--steps", type=int, default=20)
    a = ap.parse_args()
    import torch  # noqa: F401  (the library shares torch's HIP runtime)
    res = {"steps": a.steps}
    if a.hydro2d:
        res["hydro2d_15360_fp32_resident_geometry"] = hydro2d(15360, a.steps, 16_000_000_000)
    if a.ns3d:
        from paper_1709_02125_amd import ns3d as N
        n = 512
        res["ns3d_512_fp32"] = ns3d(n, a.steps, N.footprint_bytes(n) // 3)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
