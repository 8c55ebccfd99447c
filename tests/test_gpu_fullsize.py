"""GPU checks at the benchmark's full sizes, in the launch configuration the
benchmark times: tiled out of core (device budget about a third of the
footprint) against the same grid fully resident -- bit-exact, plus
conservation (properties that hold at any size; the oracle cannot run these
sizes in a test's time)."""
import numpy as np
import pytest

from paper_1709_02125_amd import hydro2d as h2, hydro3d as h3, ns3d as N, ooc
from paper_1709_02125_amd.inputs import hydro_initial_state, tgv_initial_state
from gpu_util import STATE, say

pytestmark = pytest.mark.gpu


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


def test_hydro2d_15360_out_of_core_equals_in_core():
    nx, steps = 15360, 2
    say("case: hydro2d 15360^2 16e9 budget vs in-core, 2 steps")
    a, ra, st = _hydro(nx, steps, int(16e9), ooc.FLAG_PREFETCH)
    assert st["ntiles_last"] >= 3
    b, rb, _ = _hydro(nx, steps, h2.device_footprint_bytes(nx, nx), ooc.FLAG_INCORE)
    for n in STATE:
        assert np.array_equal(a[n], b[n]), n
    assert ra == rb
    m0, m1, _ = ra
    assert abs(m1 - m0) <= 1e-12 * m0


def test_ns3d_512_out_of_core_equals_in_core():
    n, steps = 512, 1
    say("case: ns3d 512^3 third-of-footprint budget vs in-core, 1 step")
    prims = tgv_initial_state(n)
    res = []
    for incore in (False, True):
        flags = ooc.FLAG_INCORE if incore else ooc.FLAG_PREFETCH
        budget = N.device_footprint_bytes(n) if incore else N.footprint_bytes(n) // 3
        app = N.NS3D(n, prims, budget=budget, flags=flags)
        app.ctx.set_schedule(chain_steps=1)
        app.initialise()
        app.run(steps)
        planes = [0, 1, 100, 255, 256, 400, 510, 511]
        res.append({q: app.interior(q)[planes] for q in ("q_r", "q_rw", "q_re")})
        if not incore:
            assert app.ctx.stats()["ntiles_last"] >= 3
        app.close()
    for q in res[0]:
        assert np.array_equal(res[0][q], res[1][q]), q


def test_hydro3d_640_out_of_core_equals_in_core():
    n, steps = (640, 640, 640), 1
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
        planes = [0, 1, 2, 100, 319, 320, 500, 641, 642, 643]
        out = {q: app.fetch(q)[planes] for q in ("rho0", "e0", "w0")}   # z extents 644 and 645
        if not incore:
            assert st["ntiles_last"] >= 3
        app.close()
        res.append((out, m0, m1, dt))
    for q in res[0][0]:
        assert np.array_equal(res[0][0][q], res[1][0][q]), q
    assert res[0][1:] == res[1][1:]
    m0, m1 = res[0][1], res[0][2]
    assert abs(m1 - m0) <= 1e-12 * m0
