"""Helpers shared by the GPU tests: running the hydro proxy through the HIP
library and through the CPU oracle on the same seeded input."""
import sys

import numpy as np
import pytest

from paper_1709_02125_amd import hydro2d as h2, ooc
from paper_1709_02125_amd.inputs import hydro_initial_state

H = 2
STATE = ("rho0", "e0", "u0", "v0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_err(g, o):
    """Max-norm error relative to the oracle field's max magnitude; a field
    that is identically zero in the oracle must be exactly zero."""
    m = np.abs(o).max()
    if m == 0.0:
        return 0.0 if np.all(g == 0.0) else np.inf
    return np.abs(g - o).max() / m


def gpu_hydro(nx, ny, steps, budget=None, flags=0, tile_rows=0, slots=0, incore=False, rho=None, ene=None,
              per_step_dt=False, resident_geometry=False, cyclic=True, resident_state=False):
    if rho is None:
        rho, ene = hydro_initial_state((nx, ny))
    if incore:
        flags |= ooc.FLAG_INCORE
        budget = h2.device_footprint_bytes(nx, ny)
    elif budget is None:
        budget = h2.device_footprint_bytes(nx, ny) // 3
    app = h2.Hydro2D(nx, ny, rho, ene, budget=budget, flags=flags, resident_geometry=resident_geometry,
                     cyclic_after_init=cyclic, resident_state=resident_state)
    if tile_rows or slots:
        app.ctx.set_schedule(tile_rows=tile_rows, slots=slots)
    dts = [app.initialise()]
    if per_step_dt:
        for _ in range(steps):
            app.queue_step()
            dts.append(app.ctx.reduce(app.dt))
    else:
        app.run(steps)
        dts.append(app.ctx.reduce(app.dt))
    out = {n: app.fetch(n) for n in STATE}
    st = app.ctx.stats()
    # a bound context pins all of its host storage (pageable rows would make
    # every transfer of them synchronous)
    assert st["host_pageable_bytes"] == 0 and st["host_pinned_bytes"] > 0, st
    app.close()
    return out, dts, st


def oracle_hydro(nx, ny, steps, rho=None, ene=None):
    import oracle.hydro2d as oh
    if rho is None:
        rho, ene = hydro_initial_state((nx, ny))
    o = oh.Hydro2D(nx, ny)
    o.set_state(rho, ene)
    dts, nxt = o.run(steps)
    out = {}
    for n in STATE:
        a = o.field(n)
        c = dict(h2.FIELDS)[n]
        out[n] = a[:ny + 2 * H + c[1], :nx + 2 * H + c[0]].copy()
    return out, dts + [nxt]


STATE3 = ("rho0", "e0", "u0", "v0", "w0")


def gpu_hydro3d(n, steps, budget=None, flags=0, tile_rows=0, slots=0, incore=False, per_step_dt=False,
                resident_geometry=False, cyclic=True):
    from paper_1709_02125_amd import hydro3d as h3
    rho, ene = hydro_initial_state(n)
    if incore:
        flags |= ooc.FLAG_INCORE
        budget = h3.device_footprint_bytes(n)
    elif budget is None:
        budget = h3.device_footprint_bytes(n) // 3
    app = h3.Hydro3D(n, rho, ene, budget=budget, flags=flags, resident_geometry=resident_geometry,
                     cyclic_after_init=cyclic)
    if tile_rows or slots:
        app.ctx.set_schedule(tile_rows=tile_rows, slots=slots)
    dts = [app.initialise()]
    if per_step_dt:
        for _ in range(steps):
            app.queue_step()
            dts.append(app.ctx.reduce(app.dt))
    else:
        app.run(steps)
        dts.append(app.ctx.reduce(app.dt))
    out = {name: app.fetch(name) for name in STATE3}
    st = app.ctx.stats()   # of the last step's chain
    assert st["host_pageable_bytes"] == 0 and st["host_pinned_bytes"] > 0, st
    app.queue_mass()
    mass = app.ctx.reduce(app.mass)
    app.close()
    return out, dts, st, mass


def oracle_hydro3d(n, steps):
    import oracle.hydro3d as oh
    from paper_1709_02125_amd import hydro3d as h3
    rho, ene = hydro_initial_state(n)
    o = oh.Hydro3D(*n)
    o.set_state(rho, ene)
    dts, nxt = o.run(steps)
    out = {}
    for name in STATE3:
        c = dict(h3.FIELDS)[name]
        out[name] = o.field(name)[:n[2] + 2 * H + c[2], :n[1] + 2 * H + c[1], :n[0] + 2 * H + c[0]].copy()
    return out, dts + [nxt], o.sum_cells("rho0")


# Chain replay from a captured hipGraph is switched off in the library (its
# first capture ended the test process with a host segmentation fault whose
# cause is not yet found); its cases stay listed, skipped.
GRAPH_OFF = pytest.mark.skip(reason="OOC_FLAG_GRAPH switched off: host segfault under stream capture, cause unknown")
