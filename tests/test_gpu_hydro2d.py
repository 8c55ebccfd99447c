"""GPU parity of the 2D hydro proxy: HIP library vs the CPU oracle (1e-12 per
field), and tiled vs untiled runs of the library (bit-exact)."""
import numpy as np
import pytest

from paper_1709_02125_amd import hydro2d as h2, ooc
from gpu_util import GRAPH_OFF, STATE, gpu_hydro, oracle_hydro, rel_err, say

pytestmark = pytest.mark.gpu
TOL = 1e-12


def test_hydro2d_small_tiled_matches_oracle_step_by_step():
    nx, ny, steps = 96, 80, 6
    say("case: hydro2d 96x80 tiled 1/3 budget, dt per step")
    got, gdts, st = gpu_hydro(nx, ny, steps, per_step_dt=True, flags=ooc.FLAG_PREFETCH)
    ref, odts = oracle_hydro(nx, ny, steps)
    assert st["ntiles_last"] > 2
    for n in STATE:
        e = rel_err(got[n], ref[n])
        say(n, e)
        assert e <= TOL, n
    assert np.allclose(gdts, odts, rtol=TOL, atol=0)


def test_hydro2d_c1_config_matches_oracle():
    # 960 x 960, 10 steps, device budget one third of the footprint, tiles on y
    nx = ny = 960
    say("case: hydro2d C1 960^2 10 steps 1/3 budget")
    got, gdts, st = gpu_hydro(nx, ny, 10, flags=ooc.FLAG_PREFETCH)
    ref, odts = oracle_hydro(nx, ny, 10)
    say("tiles", st["ntiles_last"], "rows", st["tile_rows"])
    assert st["ntiles_last"] >= 3
    for n in STATE:
        e = rel_err(got[n], ref[n])
        say(n, e)
        assert e <= TOL, n
    assert abs(gdts[-1] - odts[-1]) <= TOL * odts[-1]


@pytest.mark.parametrize("tile_rows,slots,flags,cyclic", [
    (1, 2, 0, False), (2, 3, 0, True), (3, 3, ooc.FLAG_PREFETCH, True), (7, 4, 0, False),
    (16, 3, ooc.FLAG_DEBUG_POISON, True), (33, 2, ooc.FLAG_PREFETCH, False), (0, 3, ooc.FLAG_DEBUG_SYNC, True),
    (6, 3, ooc.FLAG_FUSE | ooc.FLAG_PREFETCH, True), pytest.param(5, 3, ooc.FLAG_GRAPH, True, marks=GRAPH_OFF),
    pytest.param(9, 2, ooc.FLAG_GRAPH | ooc.FLAG_FUSE | ooc.FLAG_PREFETCH, True, marks=GRAPH_OFF), (4, 3, ooc.FLAG_KERNEL_COPY, True),
    (11, 3, ooc.FLAG_KERNEL_COPY | ooc.FLAG_FUSE | ooc.FLAG_PREFETCH, False),
    # ring slabs (no edge copy)
    (5, 2, ooc.FLAG_RING, True), (7, 3, ooc.FLAG_RING | ooc.FLAG_DEBUG_POISON | ooc.FLAG_PREFETCH, True),
    (9, 2, ooc.FLAG_RING | ooc.FLAG_KERNEL_COPY, False), (3, 4, ooc.FLAG_RING | ooc.FLAG_DEBUG_SYNC, True),
    (7, 3, ooc.FLAG_PREFETCH | ooc.FLAG_MEMCPY_DOWNLOAD, True), (5, 2, ooc.FLAG_RING | ooc.FLAG_MEMCPY_DOWNLOAD, True)])
def test_hydro2d_tiled_equals_untiled_bit_exact(tile_rows, slots, flags, cyclic):
    nx, ny, steps = 40, 51, 5  # several chains: graph mode replays its capture
    say("case: tiled vs in-core", tile_rows, slots, flags, cyclic)
    ref, rdts, _ = gpu_hydro(nx, ny, steps, incore=True)
    # budget large enough for any forced tile height at this slot count (ring
    # slabs: plus one 64 KiB granule per field, which at this tiny grid is
    # more than a field's rows)
    budget = slots * h2.device_footprint_bytes(nx, ny) + (len(h2.FIELDS) << 16 if flags & ooc.FLAG_RING else 0)
    got, gdts, st = gpu_hydro(nx, ny, steps, budget=budget, tile_rows=tile_rows, slots=slots, flags=flags,
                              cyclic=cyclic)
    if tile_rows:
        assert st["ntiles_last"] == -(-(ny + 4) // tile_rows) or st["ntiles_last"] >= 2
    for n in STATE:
        assert np.array_equal(got[n], ref[n]), n
    assert gdts == rdts


def test_hydro2d_incore_matches_oracle():
    nx, ny, steps = 64, 48, 8
    say("case: in-core vs oracle")
    got, gdts, _ = gpu_hydro(nx, ny, steps, incore=True)
    ref, odts = oracle_hydro(nx, ny, steps)
    for n in STATE:
        assert rel_err(got[n], ref[n]) <= TOL, n


def test_hydro2d_resident_state_bit_exact():
    # geometry and state stay on the device; only temporaries are tiled
    nx, ny, steps = 48, 90, 3
    say("case: resident state")
    ref, rdts, _ = gpu_hydro(nx, ny, steps, incore=True)
    got, gdts, st = gpu_hydro(nx, ny, steps, budget=h2.device_footprint_bytes(nx, ny) // 2, resident_state=True)
    assert st["ntiles_last"] >= 2 and st["last_bytes_h2d"] == 0 and st["last_bytes_d2h"] == 0
    for n in STATE:
        assert np.array_equal(got[n], ref[n]), n
    assert gdts == rdts


def test_hydro2d_resident_geometry_bit_exact():
    nx, ny, steps = 48, 60, 3
    say("case: resident geometry")
    ref, _, _ = gpu_hydro(nx, ny, steps, incore=True)
    got, _, st = gpu_hydro(nx, ny, steps, budget=h2.device_footprint_bytes(nx, ny) // 2, resident_geometry=True)
    for n in STATE:
        assert np.array_equal(got[n], ref[n]), n


def test_hydro2d_transfer_bytes_match_plan():
    nx, ny = 64, 90
    say("case: transfer bytes vs plan")
    from paper_1709_02125_amd.inputs import hydro_initial_state
    rho, ene = hydro_initial_state((nx, ny))
    app = h2.Hydro2D(nx, ny, rho, ene, budget=h2.device_footprint_bytes(nx, ny) // 3)
    app.initialise()
    app.queue_step()
    p = app.ctx.debug_plan()
    pitch = app.ctx.layout()[0]
    up = int((p["up"][:, 3] - p["up"][:, 2]).sum()) * pitch * 8
    down = int((p["down"][:, 3] - p["down"][:, 2]).sum()) * pitch * 8
    app.ctx.execute()
    st = app.ctx.stats()
    assert st["last_bytes_h2d"] == up and st["last_bytes_d2h"] == down
    names = [n for n, _ in h2.FIELDS]
    assert {names[f] for f in p["down"][:, 0]} == {"rho0", "e0", "u0", "v0"}
    app.close()


def test_hydro2d_mass_sum_is_tiling_independent_and_conserved():
    nx, ny = 80, 70
    say("case: mass sum")
    from paper_1709_02125_amd.inputs import hydro_initial_state
    import oracle.hydro2d as oh
    rho, ene = hydro_initial_state((nx, ny))
    masses = []
    for incore in (True, False):
        flags = ooc.FLAG_INCORE if incore else 0
        budget = h2.device_footprint_bytes(nx, ny) if incore else h2.device_footprint_bytes(nx, ny) // 3
        app = h2.Hydro2D(nx, ny, rho, ene, budget=budget, flags=flags)
        app.initialise()
        app.queue_mass()
        m0 = app.ctx.reduce(app.mass)
        app.run(5)
        app.queue_mass()
        m1 = app.ctx.reduce(app.mass)
        masses.append((m0, m1))
        app.close()
    assert masses[0] == masses[1]
    m0, m1 = masses[0]
    assert abs(m1 - m0) <= 1e-13 * m0
    o = oh.Hydro2D(nx, ny)
    o.set_state(rho, ene)
    assert abs(o.sum_cells("rho0") - m0) <= 1e-12 * m0


def test_cyclic_before_init_is_refused():
    # Section 4.1: Cyclic is unsafe while the initialisation phase still writes
    # data that later chains read (here: the mesh geometry); the library must
    # refuse the read of a skipped temporary instead of using stale data.
    nx, ny = 32, 40
    say("case: cyclic before init")
    from paper_1709_02125_amd.inputs import hydro_initial_state
    rho, ene = hydro_initial_state((nx, ny))
    app = h2.Hydro2D(nx, ny, rho, ene, budget=h2.device_footprint_bytes(nx, ny), flags=ooc.FLAG_CYCLIC)
    app.queue_init()
    app.ctx.execute()
    app.queue_step()
    with pytest.raises(ooc.OocError) as e:
        app.ctx.execute()
    assert e.value.code == ooc.E_STALE
    app.close()


def test_hydro2d_fp32_streaming_error_is_stated_and_tiling_independent():
    # Extension: streamed fields stored and moved as float32 (rounded to nearest
    # even on the way out, widened exactly on the way in); compute, dt and the
    # sums stay float64.  The error against the float64 oracle is reported, and
    # different tilings give identical results (each chain rounds the state
    # once, whatever the tiles).
    nx, ny, steps = 96, 120, 20
    say("case: fp32 streaming")
    flags = ooc.FLAG_FP32_STREAM | ooc.FLAG_PREFETCH
    a, adts, st = gpu_hydro(nx, ny, steps, flags=flags, resident_geometry=True,
                            budget=h2.device_footprint_bytes(nx, ny) // 3)
    b, bdts, _ = gpu_hydro(nx, ny, steps, flags=flags, resident_geometry=True, tile_rows=5, slots=4,
                           budget=h2.device_footprint_bytes(nx, ny))
    for n in STATE:
        assert np.array_equal(a[n], b[n]), n
    assert st["ntiles_last"] > 2
    c, _, _ = gpu_hydro(nx, ny, steps, flags=flags | ooc.FLAG_KERNEL_COPY, resident_geometry=True,
                        tile_rows=7, budget=h2.device_footprint_bytes(nx, ny))
    for n in STATE:   # conversion in the copy kernel == staging + convert kernels
        assert np.array_equal(a[n], c[n]), n
    g, _, _ = gpu_hydro(nx, ny, steps, flags=flags | ooc.FLAG_MEMCPY_DOWNLOAD, resident_geometry=True,
                        tile_rows=6, budget=h2.device_footprint_bytes(nx, ny))
    for n in STATE:   # downloads rounded in staging and sent by runtime memcpy calls
        assert np.array_equal(a[n], g[n]), n
    ref, odts = oracle_hydro(nx, ny, steps)
    errs = {n: rel_err(a[n], ref[n]) for n in STATE}
    say("fp32 streaming max rel error after %d steps:" % steps, errs)
    for n, e in errs.items():
        assert e < 1e-4, (n, e)
    # geometry streamed too: chains move 4 fields down for 7 up, so the
    # download kernel runs on its narrow grid (converting in flight)
    d, _, std = gpu_hydro(nx, ny, steps, flags=flags, budget=h2.device_footprint_bytes(nx, ny) // 3)
    e, _, _ = gpu_hydro(nx, ny, steps, flags=flags, tile_rows=6, slots=3,
                        budget=h2.device_footprint_bytes(nx, ny))
    assert std["ntiles_last"] > 2
    for n in STATE:
        assert np.array_equal(d[n], e[n]), n
        assert rel_err(d[n], ref[n]) < 1e-4, n


def test_hydro2d_field_summary_folded_into_the_step_chain():
    # the mass summary queued after the last step joins that step's chain:
    # the flush moves exactly the step's bytes, where a summary chain of its
    # own uploads rho0 and vol again; the sum (order-fixed per row) and the
    # state are the same either way
    nx, ny, steps = 64, 90, 3
    say("case: mass summary folded into the step chain", nx, ny)
    from paper_1709_02125_amd.inputs import hydro_initial_state
    rho, ene = hydro_initial_state((nx, ny))

    def make():
        app = h2.Hydro2D(nx, ny, rho, ene, budget=h2.device_footprint_bytes(nx, ny) // 3)
        app.initialise()
        app.run(steps - 1)
        return app

    a = make()
    a.queue_step()
    a.ctx.execute()
    step_bytes = a.ctx.stats()["last_bytes_h2d"]
    a.queue_mass()
    ma = a.ctx.reduce(a.mass)
    summary_bytes = a.ctx.stats()["last_bytes_h2d"]
    b = make()
    b.queue_step()
    b.queue_mass()
    mb = b.ctx.reduce(b.mass)
    folded_bytes = b.ctx.stats()["last_bytes_h2d"]
    assert folded_bytes == step_bytes and summary_bytes > 0
    assert ma == mb
    for n in STATE:
        assert np.array_equal(a.fetch(n), b.fetch(n)), n
    a.close()
    b.close()


def _summary_run(nx, ny, steps, every, budget, flags, folded=True):
    """Run `steps` steps with the field summary every `every` steps; folded:
    queued after the step, before the flush (it joins the step's chain);
    otherwise the step is issued first and the summary is a chain of its own.
    Returns the sums at each summary step, the state and the bytes uploaded
    for each step (its chain and, on summary steps, the summary's)."""
    from paper_1709_02125_amd.inputs import hydro_initial_state
    rho, ene = hydro_initial_state((nx, ny))
    app = h2.Hydro2D(nx, ny, rho, ene, budget=budget, flags=flags, summary=True)
    app.initialise()
    sums, up = [], []
    for s in range(1, steps + 1):
        b0 = app.ctx.stats()["bytes_h2d"]
        app.queue_step()
        if s % every == 0:
            if not folded:
                app.ctx.submit()
            app.queue_summary()
            sums.append(app.summary())
        else:
            app.ctx.submit()
        up.append(app.ctx.stats()["bytes_h2d"] - b0)
    app.ctx.execute()
    st = app.ctx.stats()
    out = {n: app.fetch(n) for n in STATE}
    app.close()
    return sums, out, up, st


def test_hydro2d_field_summary_every_10_steps_matches_oracle():
    # The paper's periodic field summary (volume, mass, internal and kinetic
    # energy, pressure; Section 5.3) every 10 steps, folded into the step's
    # chain: each sum equals the oracle's plain sum of the same state to
    # 1e-12, the sums are bit-identical across tilings (order-fixed per row)
    # and to a summary run as a chain of its own, and folding leaves the state
    # unchanged.  Mass and volume are conserved in the closed box.
    import oracle.hydro2d as oh
    from paper_1709_02125_amd.inputs import hydro_initial_state
    nx, ny, steps, every = 96, 130, 20, 10
    say("case: hydro2d field summary every 10 steps, 96x130, 1/3 budget, folded")
    fs = h2.device_footprint_bytes(nx, ny, summary=True)
    a, sa, upa, sta = _summary_run(nx, ny, steps, every, fs // 3, ooc.FLAG_PREFETCH)
    assert sta["ntiles_last"] >= 3
    rho, ene = hydro_initial_state((nx, ny))
    o = oh.Hydro2D(nx, ny)
    o.set_state(rho, ene)
    dt = o.dt()
    ref = []
    for s in range(1, steps + 1):
        dt = o.step(dt)
        if s % every == 0:
            ref.append(o.field_summary())
    assert len(a) == len(ref) == steps // every
    for g, r in zip(a, ref):
        for q, name in enumerate(h2.SUMMARY):
            e = abs(g[q] - r[q]) / abs(r[q])
            say("summary", name, g[q], r[q], e)
            assert e <= TOL, name
    assert a[0][0] == a[1][0]                          # volume: the mesh does not move
    assert abs(a[1][1] - a[0][1]) <= 1e-13 * a[0][1]   # mass: closed box
    say("case: the same in core and with 7-row tiles, and unfolded")
    b, sb, _, _ = _summary_run(nx, ny, steps, every, fs, ooc.FLAG_INCORE)
    c, sc, _, _ = _summary_run(nx, ny, steps, every, fs // 3, ooc.FLAG_PREFETCH, folded=False)
    for g1, g2, g3 in zip(a, b, c):
        assert np.array_equal(g1, g2) and np.array_equal(g1, g3)
    for n in STATE:
        assert np.array_equal(sa[n], sb[n]) and np.array_equal(sa[n], sc[n]), n


def test_hydro2d_folded_summary_moves_no_extra_bytes():
    # folded into the step's chain the summary reads rows the chain holds
    # anyway: a summary step uploads what any other step does; as a chain of
    # its own the summary uploads vol, rho0, e0, u0 and v0 again
    nx, ny = 64, 150
    say("case: folded field summary bytes", nx, ny)
    fs = h2.device_footprint_bytes(nx, ny, summary=True)
    _, _, up_f, _ = _summary_run(nx, ny, 4, 2, fs // 3, ooc.FLAG_PREFETCH)
    _, _, up_s, _ = _summary_run(nx, ny, 4, 2, fs // 3, ooc.FLAG_PREFETCH, folded=False)
    say("bytes per step, folded", up_f, "separate", up_s)
    assert up_f[0] > 0 and all(u == up_f[0] for u in up_f), up_f
    assert up_s[0] == up_s[2] == up_f[0], up_s
    assert up_s[1] > up_f[0] and up_s[3] > up_f[0], up_s


def test_hydro2d_tile_stage_timing_follows_the_pipeline():
    # per-tile stage events on the three streams: each tile's compute begins
    # after its upload ends, its download after its compute and edge copy;
    # the upload into a slot begins after the download of the tile that held
    # the slot before it (S tiles earlier)
    nx, ny, slots = 64, 300, 3
    say("case: tile stage timing", nx, ny, slots)
    from paper_1709_02125_amd.inputs import hydro_initial_state
    rho, ene = hydro_initial_state((nx, ny))
    app = h2.Hydro2D(nx, ny, rho, ene, budget=h2.device_footprint_bytes(nx, ny))
    app.ctx.set_schedule(tile_rows=20, slots=slots)
    app.initialise()
    app.ctx.set_tile_timing(True)
    app.run(2)
    recs = app.ctx.tile_times()
    st = app.ctx.stats()
    app.close()
    assert st["ntiles_last"] >= 2 * slots
    assert len(recs) == 2 * st["ntiles_last"]
    by = {r["tile"]: r for r in recs}
    eps = 1.0   # us
    order = ["h2d_begin_us", "h2d_end_us", "comp_begin_us", "comp_end_us", "edge_end_us", "d2h_begin_us",
             "d2h_end_us"]
    for r in recs:
        for a, b in zip(order, order[1:]):
            assert r[a] <= r[b] + eps, (r["tile"], a, b, r)
        prev = by.get(r["tile"] - slots)
        if prev is not None:
            assert prev["d2h_end_us"] <= r["h2d_begin_us"] + eps, (r["tile"], prev, r)
    assert recs[0]["h2d_begin_us"] == 0.0 and recs[-1]["d2h_end_us"] > 0.0


def test_hydro2d_incore_cache_tiled_bit_exact():
    # Cache blocking without transfers: every field resident, the chain still
    # cut into skewed tiles (so a tile's rows are reused from cache across
    # the chain's loops) -- bit-identical to the plain in-core run
    nx, ny, steps = 64, 90, 4
    say("case: in-core, tiled for cache")
    ref, rdts, _ = gpu_hydro(nx, ny, steps, incore=True)
    for h in (5, 16):
        got, gdts, st = gpu_hydro(nx, ny, steps, incore=True, tile_rows=h)
        assert st["ntiles_last"] >= ny // h
        assert st["last_bytes_h2d"] == 0 and st["last_bytes_d2h"] == 0
        for n in STATE:
            assert np.array_equal(got[n], ref[n]), (h, n)
        assert gdts == rdts
