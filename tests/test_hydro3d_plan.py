"""Host-only: the 3D hydro chain's loop count, transfer classification and
per-step skew (no device needed; the context plans without storage)."""
import numpy as np

from paper_1709_02125_amd import hydro3d as h3, ooc


def _app(n, budget, cyclic=True, tile_rows=0):
    shape = n[::-1]
    app = h3.Hydro3D(n, np.full(shape, 0.2), np.full(shape, 1.0), budget=budget, bind=False)
    if cyclic:
        app.ctx.set_flags(ooc.FLAG_CYCLIC, 0)
    if tile_rows:
        app.ctx.set_schedule(tile_rows=tile_rows)
    app.queue_step()
    return app


def test_hydro3d_chain_classification():
    # read-only geometry is uploaded but never downloaded; write-first data is
    # never uploaded; with Cyclic the write-first temporaries stay on the device
    n = (16, 12, 120)
    app = _app(n, h3.device_footprint_bytes(n) // 3)
    p = app.ctx.debug_plan()
    assert p["nloops"] == 82
    names = [x for x, _ in h3.FIELDS]
    up = {names[f] for f in p["up"][:, 0]}
    down = {names[f] for f in p["down"][:, 0]}
    temp = {names[f] for f in range(len(names)) if p["temporary"][f]}
    assert up == {"rho0", "e0", "u0", "v0", "w0", "vol", "xarea", "yarea", "zarea"}
    assert down == {"rho0", "e0", "u0", "v0", "w0"}
    assert temp == set(names) - up
    assert p["ntiles"] > 3
    app.close()


def test_hydro3d_without_cyclic_downloads_temporaries():
    n = (16, 12, 120)
    app = _app(n, h3.device_footprint_bytes(n) // 2, cyclic=False)
    p = app.ctx.debug_plan()
    names = [x for x, _ in h3.FIELDS]
    down = {names[f] for f in p["down"][:, 0]}
    assert {"rho1", "p", "q", "w_mf", "mfz"} <= down
    assert not ({"vol", "xarea", "yarea", "zarea"} & down)
    app.close()


def test_hydro3d_tiles_partition_every_loop():
    # tile t of loop i covers [s_i(t), e_i(t)) with s_i(t) = e_i(t-1): the
    # tiles partition each loop's z range exactly (no redundant compute)
    n = (8, 8, 96)
    app = _app(n, 4 * h3.device_footprint_bytes(n), tile_rows=12)
    p = app.ctx.debug_plan()
    rows = p["loop_rows"]          # [loop, tile, (start, end)]
    assert rows.shape[1] == p["ntiles"] >= 4
    for i in range(p["nloops"]):
        assert np.all(rows[i, 1:, 0] == rows[i, :-1, 1])
        assert np.all(rows[i, :, 1] >= rows[i, :, 0])
    app.close()
