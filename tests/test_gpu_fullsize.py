"""GPU checks at the benchmark's full sizes and step counts, in the launch
configuration the benchmark times: tiled out of core (device budget about a
third of the footprint) against the FP64 oracle run on the whole grid --
every element of every state field (halos included for the hydro proxies, the
interior for the Navier-Stokes proxy, whose halos are rewritten every stage)
to 1e-12 -- and against the same grid fully resident, bit for bit, with the
time-step series and conservation.  Beside them the FP32-streaming runs
(compute, sums and the time step in FP64 on the device) with their per-field
error against the same oracle stated.

Each oracle run is finished, and only its state fields kept, before the GPU
runs start; the oracle prints every step (these runs take tens of seconds)."""
import numpy as np
import pytest

from paper_1709_02125_amd import hydro2d as h2, hydro3d as h3, ns3d as N, ooc
from paper_1709_02125_amd.inputs import hydro_initial_state, tgv_initial_state
from gpu_util import STATE, rel_err, say

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]
TOL = 1e-12


def _oracle_hydro2d(nx, steps):
    import oracle.hydro2d as oh
    rho, ene = hydro_initial_state((nx, nx))
    o = oh.Hydro2D(nx, nx)
    o.set_state(rho, ene)
    del rho, ene
    dt = o.dt()
    dts = [dt]
    for s in range(steps):
        dt = o.step(dt)
        dts.append(dt)
        say("oracle hydro2d step", s + 1)
    out = {n: o.field(n)[:nx + 2 * oh.H + dict(h2.FIELDS)[n][1], :nx + 2 * oh.H + dict(h2.FIELDS)[n][0]].copy()
           for n in STATE}
    del o
    return out, dts


def _gpu_hydro2d(nx, steps, budget, flags, **kw):
    rho, ene = hydro_initial_state((nx, nx))
    app = h2.Hydro2D(nx, nx, rho, ene, budget=budget, flags=flags, **kw)
    del rho, ene
    dts = [app.initialise()]
    app.queue_mass()
    m0 = app.ctx.reduce(app.mass)
    for _ in range(steps):
        app.queue_step()
        dts.append(app.ctx.reduce(app.dt))
    st = app.ctx.stats()   # of the last step's chain
    app.queue_mass()
    m1 = app.ctx.reduce(app.mass)
    out = {n: app.fetch(n) for n in STATE}
    app.close()
    return out, dts, (m0, m1), st


def test_hydro2d_15360_20_steps_equals_oracle_and_in_core():
    nx, steps = 15360, 20
    say("case: hydro2d 15360^2 FP64 oracle on the whole grid, 20 steps")
    ref, odts = _oracle_hydro2d(nx, steps)
    say("case: hydro2d 15360^2 16e9 budget, 20 steps")
    a, adts, am, st = _gpu_hydro2d(nx, steps, int(16e9), ooc.FLAG_PREFETCH)
    assert st["ntiles_last"] >= 3
    for n in STATE:
        e = rel_err(a[n], ref[n])
        say(n, "vs oracle (whole field)", e)
        assert e <= TOL, n
    assert len(adts) == len(odts)
    for g, o in zip(adts, odts):
        assert abs(g - o) <= TOL * o
    assert abs(am[1] - am[0]) <= 1e-12 * am[0]
    say("case: hydro2d 15360^2 in core, 20 steps")
    b, bdts, bm, _ = _gpu_hydro2d(nx, steps, h2.device_footprint_bytes(nx, nx), ooc.FLAG_INCORE)
    for n in STATE:
        assert np.array_equal(a[n], b[n]), n
    assert adts == bdts and am == bm
    del b
    # FP32 streaming with resident geometry (the FP32 form of this grid):
    # stated error per field against the FP64 oracle after 20 steps
    say("case: hydro2d 15360^2 FP32 streaming + resident geometry, 16e9 budget, 20 steps")
    c, cdts, cm, _ = _gpu_hydro2d(nx, steps, int(16e9), ooc.FLAG_PREFETCH | ooc.FLAG_FP32_STREAM,
                                  resident_geometry=True)
    for n in STATE:
        e = rel_err(c[n], ref[n])
        say("FP32 stream error", n, e)
        assert e <= 1e-5, n
    say("FP32 stream dt error", max(abs(g - o) / o for g, o in zip(cdts, odts)))
    say("FP32 stream mass drift", abs(cm[1] - cm[0]) / cm[0])


def test_hydro3d_640_10_steps_equals_oracle_and_in_core():
    import oracle.hydro3d as oh
    n, steps = (640, 640, 640), 10
    names = ("rho0", "e0", "u0", "v0", "w0")
    say("case: hydro3d 640^3 FP64 oracle on the whole grid, 10 steps")
    rho, ene = hydro_initial_state(n)
    o = oh.Hydro3D(*n)
    o.set_state(rho, ene)
    del rho, ene
    dt = o.dt()
    odts = [dt]
    for s in range(steps):
        dt = o.step(dt)
        odts.append(dt)
        say("oracle hydro3d step", s + 1)
    ref = {}
    for q in names:
        c = dict(h3.FIELDS)[q]
        ref[q] = o.field(q)[:n[2] + 2 * oh.H + c[2], :n[1] + 2 * oh.H + c[1], :n[0] + 2 * oh.H + c[0]].copy()
    del o
    res = []
    for incore in (False, True):
        say("case: hydro3d 640^3 %s, 10 steps" % ("in core" if incore else "third-of-footprint budget"))
        flags = ooc.FLAG_INCORE if incore else ooc.FLAG_PREFETCH
        budget = h3.device_footprint_bytes(n) if incore else h3.footprint_bytes(n) // 3
        rho, ene = hydro_initial_state(n)
        app = h3.Hydro3D(n, rho, ene, budget=budget, flags=flags)
        del rho, ene
        dts = [app.initialise()]
        app.queue_mass()
        m0 = app.ctx.reduce(app.mass)
        for _ in range(steps):
            app.queue_step()
            dts.append(app.ctx.reduce(app.dt))
        st = app.ctx.stats()
        app.queue_mass()
        m1 = app.ctx.reduce(app.mass)
        out = {q: app.fetch(q) for q in names}
        if not incore:
            assert st["ntiles_last"] >= 3
        app.close()
        if not incore:
            for q in names:
                e = rel_err(out[q], ref[q])
                say(q, "vs oracle (whole field)", e)
                assert e <= TOL, q
            for g, od in zip(dts, odts):
                assert abs(g - od) <= TOL * od
            assert abs(m1 - m0) <= 1e-12 * m0
            del ref
        res.append((out, dts, m0, m1))
    for q in names:
        assert np.array_equal(res[0][0][q], res[1][0][q]), q
    assert res[0][1:] == res[1][1:]


@pytest.fixture(scope="module")
def ns3d_oracle():
    """The FP64 oracle's conserved fields at 512^3 after 10 and 20 steps."""
    import oracle.ns3d as on
    n = 512
    o = on.NS3D(n)
    o.set_primitives(*tgv_initial_state(n))
    snap = {}
    for s in range(20):
        o.step(on.stable_dt(n))
        say("oracle ns3d step", s + 1)
        if s + 1 in (10, 20):
            snap[s + 1] = {q: o.interior(q).copy() for q in N.Q}
    del o
    return snap


NS_CONFIGS = [
    # the benchmark's headline: 15-field chain (two copies of the conserved
    # variables; primitives and gradients inside the residual) on ring slabs,
    # memcpy downloads, largest tiles, chains of 4 steps, 3 slots
    ("conserved-input residual, ring slabs, memcpy downloads, largest tiles, 4-step chains, 3 slots", "q",
     ooc.FLAG_RING | ooc.FLAG_MEMCPY_DOWNLOAD, (0, 4, 3)),
    # the same schedule with stored primitives
    ("fused residual, ring slabs, memcpy downloads, largest tiles, 4-step chains, 3 slots", True,
     ooc.FLAG_RING | ooc.FLAG_MEMCPY_DOWNLOAD, (0, 4, 3)),
    # its variant with stored gradients on slots with edge copies
    ("stored gradients, slots with edge copies, 24-plane tiles, 3-step chains, 2 slots", False, 0, (24, 3, 2)),
]


@pytest.mark.parametrize("what,fused,extra,sched", NS_CONFIGS, ids=["conserved_input_ring", "fused_ring",
                                                                   "stored_slots"])
def test_ns3d_512_10_steps_equals_oracle_and_in_core(ns3d_oracle, what, fused, extra, sched):
    n, steps = 512, 10
    ref = ns3d_oracle[10]
    prims = tgv_initial_state(n)
    res = []
    for incore in (False, True):
        say("case: ns3d 512^3 FP64 %s, 10 steps" % ("in core" if incore else "third-of-footprint budget, " + what))
        flags = ooc.FLAG_INCORE if incore else ooc.FLAG_PREFETCH | extra
        budget = N.device_footprint_bytes(n, fused) if incore else N.footprint_bytes(n, fused) // 3
        app = N.NS3D(n, prims, budget=budget, flags=flags, fused=fused)
        if not incore:
            app.ctx.set_schedule(tile_rows=sched[0], chain_steps=sched[1], slots=sched[2])
        app.initialise()
        app.run(steps)
        if not incore:
            assert app.ctx.stats()["ntiles_last"] >= 3
        res.append({q: app.interior(q) for q in N.Q})
        app.close()
    for q in N.Q:
        e = rel_err(res[0][q], ref[q])
        say(q, "vs oracle (whole interior)", e)
        assert e <= TOL, q
        assert np.array_equal(res[0][q], res[1][q]), q


def test_ns3d_512_fp32_stream_20_steps_error(ns3d_oracle):
    # FP32 storage and transfer of the streamed fields in the benchmark's
    # form and schedule (conserved-input residual on ring slabs, largest
    # tiles, chains of 4 steps, 3 slots): stated error per field against the
    # FP64 oracle after 20 steps
    n, steps = 512, 20
    ref = ns3d_oracle[20]
    say("case: ns3d 512^3 FP32 streaming, third-of-footprint budget, ring slabs, largest tiles, 4-step chains, "
        "20 steps")
    app = N.NS3D(n, tgv_initial_state(n), budget=N.footprint_bytes(n, "q") // 3,
                 flags=ooc.FLAG_PREFETCH | ooc.FLAG_FP32_STREAM | ooc.FLAG_RING | ooc.FLAG_MEMCPY_DOWNLOAD, fused="q")
    app.ctx.set_schedule(tile_rows=0, chain_steps=4, slots=3)
    app.initialise()
    app.run(steps)
    got = {q: app.interior(q) for q in N.Q}
    app.close()
    for q in N.Q:
        e = rel_err(got[q], ref[q])
        say("FP32 stream error", q, e)
        assert e <= (1e-3 if q == "q_rw" else 1e-5), q
