"""GPU checks at the benchmark's full sizes, in the launch configuration the
benchmark times: tiled out of core (device budget about a third of the
footprint) against the same grid fully resident -- bit-exact -- and against
the FP64 oracle run on the whole grid (its OpenMP loops take seconds per step
at these sizes), compared on sampled rows / planes of the state to 1e-12,
plus conservation.  Each oracle run is finished and freed before the GPU runs
start, so host memory holds one copy of the grid at a time."""
import numpy as np
import pytest

from paper_1709_02125_amd import hydro2d as h2, hydro3d as h3, ns3d as N, ooc
from paper_1709_02125_amd.inputs import hydro_initial_state, tgv_initial_state
from gpu_util import STATE, rel_err, say

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _oracle_hydro2d_rows(nx, steps, rows):
    import oracle.hydro2d as oh
    rho, ene = hydro_initial_state((nx, nx))
    o = oh.Hydro2D(nx, nx)
    o.set_state(rho, ene)
    del rho, ene
    _, nxt = o.run(steps)
    out = {n: o.field(n)[rows, :nx + 2 * oh.H + dict(h2.FIELDS)[n][0]].copy() for n in STATE}
    del o
    return out, nxt


def _oracle_hydro3d_planes(n, steps, planes, names):
    import oracle.hydro3d as oh
    rho, ene = hydro_initial_state(n)
    o = oh.Hydro3D(*n)
    o.set_state(rho, ene)
    del rho, ene
    _, nxt = o.run(steps)
    out = {}
    for q in names:
        c = dict(h3.FIELDS)[q]
        out[q] = o.field(q)[planes, :n[1] + 2 * oh.H + c[1], :n[0] + 2 * oh.H + c[0]].copy()
    del o
    return out, nxt


def _oracle_ns3d_planes(n, steps, planes, names):
    import oracle.ns3d as on
    o = on.NS3D(n)
    o.set_primitives(*tgv_initial_state(n))
    for _ in range(steps):
        o.step(on.stable_dt(n))
    out = {q: o.interior(q)[planes].copy() for q in names}
    del o
    return out


def _hydro(nx, steps, budget, flags):
    rho, ene = hydro_initial_state((nx, nx))
    app = h2.Hydro2D(nx, nx, rho, ene, budget=budget, flags=flags)
    app.initialise()
    app.queue_mass()
    m0 = app.ctx.reduce(app.mass)
    app.run(steps)
    st = app.ctx.stats()   # of the last step's chain
    app.queue_mass()
    m1 = app.ctx.reduce(app.mass)
    dt = app.ctx.reduce(app.dt)
    # sampled rows of the state (the full fields are 1.9 GB each)
    rows = np.linspace(0, nx + 3, 17).astype(int)
    out = {n: app.fetch(n)[rows] for n in STATE}
    app.close()
    return out, (m0, m1, dt), st


def test_hydro2d_15360_out_of_core_equals_in_core_and_oracle():
    nx, steps = 15360, 2
    rows = np.linspace(0, nx + 3, 17).astype(int)
    say("case: hydro2d 15360^2 FP64 oracle on the whole grid, 2 steps")
    ref, odt = _oracle_hydro2d_rows(nx, steps, rows)
    say("case: hydro2d 15360^2 16e9 budget vs in-core, 2 steps")
    a, ra, st = _hydro(nx, steps, int(16e9), ooc.FLAG_PREFETCH)
    assert st["ntiles_last"] >= 3
    for n in STATE:
        e = rel_err(a[n], ref[n])
        say(n, "vs oracle", e)
        assert e <= TOL, n
    assert abs(ra[2] - odt) <= TOL * odt
    b, rb, _ = _hydro(nx, steps, h2.device_footprint_bytes(nx, nx), ooc.FLAG_INCORE)
    for n in STATE:
        assert np.array_equal(a[n], b[n]), n
    assert ra == rb
    m0, m1, _ = ra
    assert abs(m1 - m0) <= 1e-12 * m0


def test_ns3d_512_out_of_core_equals_in_core_and_oracle():
    # the benchmark's schedule: 24-plane tiles, chains of 3 steps, 2 slots
    n, steps = 512, 3
    planes = [0, 1, 100, 255, 256, 400, 510, 511]
    say("case: ns3d 512^3 FP64 oracle on the whole grid, 3 steps")
    ref = _oracle_ns3d_planes(n, steps, planes, N.Q)
    say("case: ns3d 512^3 third-of-footprint budget (24-plane tiles, 3-step chains, 2 slots) vs in-core")
    prims = tgv_initial_state(n)
    res = []
    for incore in (False, True):
        flags = ooc.FLAG_INCORE if incore else ooc.FLAG_PREFETCH
        budget = N.device_footprint_bytes(n) if incore else N.footprint_bytes(n) // 3
        app = N.NS3D(n, prims, budget=budget, flags=flags)
        if not incore:
            app.ctx.set_schedule(tile_rows=24, chain_steps=3, slots=2)
        app.initialise()
        app.run(steps)
        res.append({q: app.interior(q)[planes] for q in N.Q})
        if not incore:
            assert app.ctx.stats()["ntiles_last"] >= 3
        app.close()
    for q in N.Q:
        e = rel_err(res[0][q], ref[q])
        say(q, "vs oracle", e)
        assert e <= TOL, q
        assert np.array_equal(res[0][q], res[1][q]), q


def test_hydro3d_640_out_of_core_equals_in_core_and_oracle():
    n, steps = (640, 640, 640), 1
    planes = [0, 1, 2, 100, 319, 320, 500, 641, 642, 643]   # z extents 644 and 645
    names = ("rho0", "e0", "u0", "v0", "w0")
    say("case: hydro3d 640^3 FP64 oracle on the whole grid, 1 step")
    ref, odt = _oracle_hydro3d_planes(n, steps, planes, names)
    say("case: hydro3d 640^3 third-of-footprint budget vs in-core, 1 step")
    rho, ene = hydro_initial_state(n)
    res = []
    for incore in (False, True):
        flags = ooc.FLAG_INCORE if incore else ooc.FLAG_PREFETCH
        budget = h3.device_footprint_bytes(n) if incore else h3.footprint_bytes(n) // 3
        app = h3.Hydro3D(n, rho, ene, budget=budget, flags=flags)
        app.initialise()
        app.queue_mass()
        m0 = app.ctx.reduce(app.mass)
        app.run(steps)
        st = app.ctx.stats()   # of the last step's chain
        app.queue_mass()
        m1 = app.ctx.reduce(app.mass)
        dt = app.ctx.reduce(app.dt)
        out = {q: app.fetch(q)[planes] for q in names}
        if not incore:
            assert st["ntiles_last"] >= 3
        app.close()
        res.append((out, m0, m1, dt))
    for q in names:
        e = rel_err(res[0][0][q], ref[q])
        say(q, "vs oracle", e)
        assert e <= TOL, q
        assert np.array_equal(res[0][0][q], res[1][0][q]), q
    assert abs(res[0][3] - odt) <= TOL * odt
    assert res[0][1:] == res[1][1:]
    m0, m1 = res[0][1], res[0][2]
    assert abs(m1 - m0) <= 1e-12 * m0
