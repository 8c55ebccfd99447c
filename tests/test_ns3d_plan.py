"""Host-only: the Navier-Stokes chain's classification and multi-step skew."""
import numpy as np

from paper_1709_02125_amd import ns3d as N, ooc


def _app(n, steps, budget, chain_steps=0, tile_rows=0):
    z = np.zeros((n, n, n))
    app = N.NS3D(n, (z + 1, z, z, z, z + 71.4), budget=budget, bind=False)
    app.ctx.set_flags(ooc.FLAG_CYCLIC, 0)
    app.ctx.set_schedule(tile_rows=tile_rows, chain_steps=chain_steps)
    for _ in range(steps):
        app.queue_step()
    return app


def test_only_conserved_variables_move():
    n = 16
    app = _app(n, 1, 4 * N.device_footprint_bytes(n), tile_rows=4)
    p = app.ctx.debug_plan()
    up = {N.FIELDS[f] for f in p["up"][:, 0]}
    down = {N.FIELDS[f] for f in p["down"][:, 0]}
    assert up == set(N.Q) and down == set(N.Q)
    temp = {N.FIELDS[f] for f in range(len(N.FIELDS)) if p["temporary"][f]}
    assert temp == set(N.FIELDS) - set(N.Q)
    app.close()


def test_skew_of_multi_step_chains():
    # Per Runge-Kutta stage the residual reads the gradients 2 planes away,
    # which read the primitives 2 planes away (read after write: 4 planes);
    # at each stage boundary the next stage's primitives overwrite values the
    # residual still reads 2 planes back (write after read: 2 more).  A chain
    # of k steps = 3k stages: lead = 4 * 3k + 2 * (3k - 1).
    n = 64
    for steps, lead in ((1, 16), (2, 34)):
        app = _app(n, steps, 16 * N.device_footprint_bytes(n), chain_steps=steps, tile_rows=8)
        p = app.ctx.debug_plan()
        e = p["loop_rows"][:, 0, 1]  # end of tile 0
        nloops = 45 * steps
        assert p["nloops"] == nloops
        prims_first = e[12]          # primitives loop of the first stage
        rhs_last = e[nloops - 1]     # residual loop of the last stage
        assert prims_first - rhs_last == lead, (steps, prims_first, rhs_last)
        app.close()


def test_chain_steps_splits_the_queue():
    n = 16
    app = _app(n, 3, 8 * N.device_footprint_bytes(n), chain_steps=2, tile_rows=4)
    p = app.ctx.debug_plan()
    assert p["nloops"] == 90  # the first chain holds two steps
    app.close()


def _fused_app(n, steps, budget, chain_steps=0, tile_rows=0):
    z = np.zeros((n, n, n))
    app = N.NS3D(n, (z + 1, z, z, z, z + 71.4), budget=budget, bind=False, fused=True)
    app.ctx.set_flags(ooc.FLAG_CYCLIC, 0)
    app.ctx.set_schedule(tile_rows=tile_rows, chain_steps=chain_steps)
    for _ in range(steps):
        app.queue_step()
    return app


def test_fused_chain_moves_only_conserved_variables():
    # 15 fields: the increments and the primitives are temporaries
    n = 16
    app = _fused_app(n, 1, 4 * N.device_footprint_bytes(n, True), tile_rows=4)
    p = app.ctx.debug_plan()
    assert p["nfields"] == 15 and p["nloops"] == 42
    up = {N.FIELDS_FUSED[f] for f in p["up"][:, 0]}
    down = {N.FIELDS_FUSED[f] for f in p["down"][:, 0]}
    assert up == set(N.Q) and down == set(N.Q)
    temp = {N.FIELDS_FUSED[f] for f in range(15) if p["temporary"][f]}
    assert temp == set(N.D) | set(N.P)
    app.close()


def test_fused_stencil_is_the_flux_points_of_the_gradient_stencils():
    # 1 centre, 8 points (+-1 .. +-4) on each axis, 16 off-axis points in each
    # of the 3 coordinate planes; reach 4 along every axis
    s = np.array(N.FUSED_STENCIL)
    assert len(s) == 73 and len(set(map(tuple, s))) == 73
    assert (np.abs(s).max(axis=0) == 4).all()
    assert ((s != 0).sum(axis=1) <= 2).all()


def test_skew_of_multi_step_fused_chains():
    # The fused residual reads the primitives 4 planes away (read after
    # write: 4 planes per stage); at each stage boundary the next stage's
    # primitives overwrite values the residual still reads 4 planes back
    # (write after read: 4 more).  A chain of k steps: lead = 4 * 3k + 4 * (3k - 1).
    n = 96
    for steps, lead in ((1, 20), (2, 44), (3, 68)):
        app = _fused_app(n, steps, 16 * N.device_footprint_bytes(n, True), chain_steps=steps, tile_rows=8)
        p = app.ctx.debug_plan()
        e = p["loop_rows"][:, 0, 1]
        nloops = 42 * steps
        assert p["nloops"] == nloops
        assert e[12] - e[nloops - 1] == lead, (steps, e[12], e[nloops - 1])
        app.close()
