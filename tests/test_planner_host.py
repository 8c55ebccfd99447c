"""Host-only tests of the loop-chain analysis and tile planning (no GPU):
the plan is taken from the real library (ooc_debug_plan) and executed by the
numpy tile simulator with NaN-poisoned slots."""
import numpy as np
import pytest

from paper_1709_02125_amd import ooc
from paper_1709_02125_amd.ooc import READ, WRITE, RW, INC, Const, dat
import tile_sim

H = 2
CENTRINGS = [(0, 0), (1, 1), (1, 0), (0, 1)]


def make_ctx(nx, ny, nfields, rng, budget=1 << 30, flags=0, centrings=None):
    c = ooc.Context(2, (nx, ny), H, budget, flags, bind=False)
    host, shapes = {}, {}
    for f in range(nfields):
        cen = centrings[f] if centrings else CENTRINGS[rng.integers(len(CENTRINGS))]
        shape = c.field_shape_for(cen)
        init = rng.standard_normal(shape)
        h = c.decl_field("f%d" % f, cen, init)
        host[h] = init
        shapes[h] = cen
    return c, host, shapes


def extent(nx, ny, cen):
    return (-H, nx + H + cen[0]), (-H, ny + H + cen[1])


def random_chain(nx, ny, shapes, rng, nloops):
    """Random valid toy loops (AVG / INC_ADD / MIRROR / FILL)."""
    fields = list(shapes)
    loops = []
    tries = 0
    while len(loops) < nloops and tries < 2000:
        tries += 1
        kind = rng.choice(["avg", "avg", "avg", "inc", "mirror", "fill"])
        fo = int(rng.choice(fields))
        ex, ey = extent(nx, ny, shapes[fo])
        if kind == "fill":
            x0 = int(rng.integers(ex[0], ex[1]))
            x1 = int(rng.integers(x0 + 1, ex[1] + 1))
            y0 = int(rng.integers(ey[0], ey[1]))
            y1 = int(rng.integers(y0 + 1, ey[1] + 1))
            loops.append(tile_sim.ToyLoop(tile_sim.K_FILL, ((x0, x1), (y0, y1)), [(fo, WRITE, ((0, 0),))],
                                          [float(rng.standard_normal())]))
            continue
        fi = int(rng.choice([f for f in fields if f != fo] or fields))
        if kind == "mirror":
            fi = fo
            ix, iy = extent(nx, ny, shapes[fi])
            side = rng.integers(4)
            dep = int(rng.integers(1, H + 1))
            if side < 2:  # strip along y boundary (bottom/top) rows, mirrored read
                y0 = ey[0] if side == 0 else ey[1] - dep
                y1 = y0 + dep
                oy = (2 * dep) if side == 0 else -(2 * dep)
                rng_ = ((ex[0], ex[1]), (y0, y1))
                off = (0, oy)
            else:
                x0 = ex[0] if side == 2 else ex[1] - dep
                ox = (2 * dep) if side == 2 else -(2 * dep)
                rng_ = ((x0, x0 + dep), (ey[0], ey[1]))
                off = (ox, 0)
            loops.append(tile_sim.ToyLoop(tile_sim.K_MIRROR, rng_, [(fo, WRITE, ((0, 0),)), (fi, READ, (off,))],
                                          [float(rng.choice([-1.0, 1.0]))]))
            continue
        ix, iy = extent(nx, ny, shapes[fi])
        if kind == "inc":
            offs = ((0, 0),)
        else:
            npts = int(rng.integers(1, 5))
            offs = tuple((int(rng.integers(-2, 3)), int(rng.integers(-2, 3))) for _ in range(npts))
        mnx, mxx = min(o[0] for o in offs), max(o[0] for o in offs)
        mny, mxy = min(o[1] for o in offs), max(o[1] for o in offs)
        lx0, lx1 = max(ex[0], ix[0] - mnx), min(ex[1], ix[1] - mxx)
        ly0, ly1 = max(ey[0], iy[0] - mny), min(ey[1], iy[1] - mxy)
        if lx1 <= lx0 or ly1 <= ly0:
            continue
        x0 = int(rng.integers(lx0, lx1))
        x1 = int(rng.integers(x0 + 1, lx1 + 1))
        if rng.random() < 0.5:
            x0, x1 = lx0, lx1
        y0 = int(rng.integers(ly0, ly1))
        y1 = int(rng.integers(y0 + 1, ly1 + 1))
        if rng.random() < 0.6:
            y0, y1 = ly0, ly1
        if kind == "inc":
            loops.append(tile_sim.ToyLoop(tile_sim.K_INC_ADD, ((x0, x1), (y0, y1)),
                                          [(fo, INC, ((0, 0),)), (fi, READ, offs)], [0.5]))
        else:
            loops.append(tile_sim.ToyLoop(tile_sim.K_AVG, ((x0, x1), (y0, y1)),
                                          [(fo, WRITE, ((0, 0),)), (fi, READ, offs)],
                                          [float(rng.uniform(0.5, 1.5)), float(rng.standard_normal())]))
    return loops


def queue(c, loops):
    for lp in loops:
        args = [dat(f, acc, *offs) for (f, acc, offs) in lp.dats] + [Const(v) for v in lp.consts]
        c.par_loop(lp.kid, lp.rng, args)


def test_skew_closed_form_for_jacobi_chain():
    # k radius-1 smoothing loops alternating between two fields: every loop
    # must run exactly one row ahead of the next one (read-after-write plus
    # write-after-read of radius 1), so the first loop leads the last by k-1.
    rng = np.random.default_rng(0)
    nx, ny, k = 6, 60, 7
    c, host, shapes = make_ctx(nx, ny, 2, rng, centrings=[(0, 0), (0, 0)])
    c.set_schedule(tile_rows=10)
    a, b = 0, 1
    for n in range(k):
        src, dst = (a, b) if n % 2 == 0 else (b, a)
        c.par_loop(tile_sim.K_AVG, ((0, nx), (-1, ny + 1)),
                   [dat(dst, WRITE), dat(src, READ, (0, -1), (0, 0), (0, 1)), Const(1.0), Const(0.0)])
    p = c.debug_plan()
    e = p["loop_rows"][:, :, 1]
    T = p["ntiles"]
    assert T == -(-(ny + 2) // 10)
    short = T * 10 - (ny + 2)  # the ragged remainder: the first tile is this much shorter
    for t in range(T - 1):
        lead = e[:, t]
        if lead[0] < ny + 1:  # interior tiles, before the clamp at the range end
            assert list(np.diff(lead)) == [-1] * (k - 1)
            assert lead[-1] == -1 + (t + 1) * 10 - short  # cut: span start + (t+1) h - remainder


@pytest.mark.parametrize("seed", range(12))
def test_random_chains_tiled_equals_untiled(seed):
    rng = np.random.default_rng(seed)
    nx, ny = int(rng.integers(3, 9)), int(rng.integers(5, 14))
    nf = int(rng.integers(2, 5))
    _, _, shapes = make_ctx(nx, ny, nf, np.random.default_rng(seed))
    loops = random_chain(nx, ny, shapes, rng, int(rng.integers(3, 12)))
    rows = ny + 2 * H + 1
    cyclic = bool(seed % 2)
    for slots in (2, 3):
        for h in range(1, rows + 1):
            c, host, shapes2 = make_ctx(nx, ny, nf, np.random.default_rng(seed),
                                        flags=ooc.FLAG_CYCLIC if cyclic else 0)
            assert shapes2 == shapes
            c.set_schedule(tile_rows=h, slots=slots)
            queue(c, loops)
            p = c.debug_plan()
            ref = tile_sim.run_untiled(loops, host, H)
            got = tile_sim.run_tiled(loops, host, p, H, slots)
            for f in host:
                if cyclic and p["temporary"][f] and any(d[0] == f for lp in loops for d in lp.dats):
                    continue  # host copy intentionally stale
                assert np.array_equal(got[f], ref[f]), (seed, h, slots, f)
            # partition: every loop's tile ranges tile its range exactly
            for i, lp in enumerate(loops):
                lr = p["loop_rows"][i]
                assert lr[0, 0] == lp.rng[1][0] and lr[-1, 1] == lp.rng[1][1]
                assert all(lr[t, 1] == lr[t + 1, 0] for t in range(p["ntiles"] - 1))
                assert all(lr[t, 1] >= lr[t, 0] for t in range(p["ntiles"]))
            # each row moves at most once per chain in each direction
            for key in ("up", "down"):
                seen = set()
                for f, t, r0, r1 in p[key]:
                    for r in range(r0, r1):
                        assert (f, r) not in seen
                        seen.add((f, r))
            c.close()


def test_hydro_chain_classification():
    # Section 4.1: read-only data is never downloaded, write-first data never
    # uploaded, and with Cyclic the write-first temporaries are not downloaded.
    from paper_1709_02125_amd import hydro2d as h2
    nx, ny = 24, 300
    app = h2.Hydro2D(nx, ny, np.full((ny, nx), 0.2), np.full((ny, nx), 1.0), budget=h2.footprint_bytes(nx, ny) // 3,
                     bind=False)
    app.ctx.set_flags(ooc.FLAG_CYCLIC, 0)
    app.queue_step()
    p = app.ctx.debug_plan()
    names = [n for n, _ in h2.FIELDS]
    up = {names[f] for f in p["up"][:, 0]}
    down = {names[f] for f in p["down"][:, 0]}
    temp = {names[f] for f in range(len(names)) if p["temporary"][f]}
    assert up == {"rho0", "e0", "u0", "v0", "vol", "xarea", "yarea"}
    assert down == {"rho0", "e0", "u0", "v0"}
    assert temp == set(names) - up
    assert p["ntiles"] > 3
    app.close()


def test_hydro_chain_without_cyclic_downloads_temporaries():
    from paper_1709_02125_amd import hydro2d as h2
    nx, ny = 24, 300
    app = h2.Hydro2D(nx, ny, np.full((ny, nx), 0.2), np.full((ny, nx), 1.0), budget=h2.footprint_bytes(nx, ny) // 2,
                     bind=False)
    app.queue_step()
    p = app.ctx.debug_plan()
    names = [n for n, _ in h2.FIELDS]
    down = {names[f] for f in p["down"][:, 0]}
    assert {"rho1", "p", "q", "w_mf"} <= down
    assert not ({"vol", "xarea", "yarea"} & down)   # read-only: never downloaded
    app.close()


def test_budget_too_small_is_reported():
    rng = np.random.default_rng(1)
    c, host, shapes = make_ctx(8, 8, 2, rng, budget=600, centrings=[(0, 0), (0, 0)])
    c.par_loop(tile_sim.K_AVG, ((0, 8), (0, 8)), [dat(1, WRITE), dat(0, READ, (0, 0)), Const(1.0), Const(0.0)])
    with pytest.raises(ooc.OocError) as e:
        c.debug_plan()
    assert e.value.code == ooc.E_BUDGET


@pytest.mark.parametrize("bad", ["write_offset", "outside", "race", "kernel", "sig"])
def test_par_loop_rejects_invalid_loops(bad):
    rng = np.random.default_rng(2)
    c, host, shapes = make_ctx(8, 8, 2, rng, centrings=[(0, 0), (0, 0)])
    with pytest.raises(ooc.OocError) as e:
        if bad == "write_offset":
            c.par_loop(tile_sim.K_AVG, ((0, 8), (0, 8)), [dat(1, WRITE, (0, 1)), dat(0, READ), Const(1), Const(0)])
        elif bad == "outside":
            c.par_loop(tile_sim.K_AVG, ((0, 8), (0, 8)), [dat(1, WRITE), dat(0, READ, (0, 3)), Const(1), Const(0)])
        elif bad == "race":
            c.par_loop(tile_sim.K_AVG, ((0, 8), (0, 8)), [dat(0, WRITE), dat(0, READ, (0, 1)), Const(1), Const(0)])
        elif bad == "kernel":
            c.par_loop(9999, ((0, 8), (0, 8)), [dat(0, WRITE)])
        else:
            c.par_loop(tile_sim.K_AVG, ((0, 8), (0, 8)), [dat(1, WRITE), dat(0, READ)])
    assert e.value.code == ooc.E_ARG
    c.close()


def test_library_exports_every_declared_symbol():
    import re
    import os
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "ooc.h")).read()
    names = set(re.findall(r"^(?:int|const char \*)\s*(ooc_\w+)\(", hdr, re.M))
    lib = ooc.load_library()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(ooc.EXPORTS) == names


def test_binding_constants_match_the_header():
    # every OOC_FLAG_ / OOC_E_ constant the header defines has the same value
    # in the Python binding
    import re
    import os
    hdr = open(os.path.join(os.path.dirname(__file__), "..", "include", "ooc.h")).read()
    consts = dict((n, int(v)) for n, v in re.findall(r"\bOOC_((?:FLAG|E)_\w+)\s*=\s*(-?\d+)", hdr))
    assert len([n for n in consts if n.startswith("FLAG_")]) >= 12
    for n, v in consts.items():
        assert getattr(ooc, n) == v, n


def test_single_hip_runtime_in_process():
    import re
    ooc.load_library()
    maps = open("/proc/self/maps").read()
    hips = set(re.findall(r"\S*libamdhip64\S*", maps))
    assert len(hips) == 1, hips


def test_graph_replay_flag_is_refused():
    # chain replay from a captured graph is switched off in this version
    with pytest.raises(Exception):
        ooc.Context(2, (8, 8), 1, 1 << 20, ooc.FLAG_GRAPH, bind=False)
    c = ooc.Context(2, (8, 8), 1, 1 << 20, 0, bind=False)
    with pytest.raises(Exception):
        c.set_flags(ooc.FLAG_GRAPH, 0)
    c.close()


@pytest.mark.parametrize("ndim,dims,halo", [(2, (7, 5), 1), (2, (100, 9), 2), (3, (13, 6, 5), 4),
                                            (3, (30, 4, 3), 2)])
def test_storage_layout_and_host_round_trip(ndim, dims, halo):
    c = ooc.Context(ndim, dims, halo, 1 << 30, 0, bind=False)
    pitch, plane, xo = c.layout()
    # x = 0 on a 128-byte boundary, rows a multiple of 256 bytes holding x = -halo .. nx + halo
    assert xo == ooc.X_ORIGIN and xo % 16 == 0 and xo >= halo
    assert pitch == ooc.row_pitch(dims[0], halo) and pitch % 32 == 0 and pitch >= xo + dims[0] + halo + 1
    assert plane == (pitch * (dims[1] + 2 * halo + 1) if ndim == 3 else 0)
    rng = np.random.default_rng(len(dims) + dims[0])
    for cen in [(0,) * ndim, (1,) * ndim]:
        init = rng.standard_normal(c.field_shape_for(cen))
        f = c.decl_field("f%d" % cen[0], cen, init)
        assert np.array_equal(c.fetch_field(f, cen), init)
    c.close()


@pytest.mark.parametrize("dim", [2, 3, "2-summary"])
def test_field_summary_folds_into_the_step_chain(dim):
    # A diagnostic sum queued after a step joins the step's chain (its SUM
    # reduction is not read in the chain, so nothing splits it) and reads only
    # fields the chain holds anyway: the transfer sets are the step's own.
    # "2-summary": the five-sum field summary of the 2D proxy.
    if dim in (2, "2-summary"):
        from paper_1709_02125_amd import hydro2d as hm
        n = (24, 300)
        summ = dim == "2-summary"
        make = lambda: hm.Hydro2D(n[0], n[1], np.full(n[::-1], 0.2), np.full(n[::-1], 1.0),
                                  budget=hm.device_footprint_bytes(*n, summary=summ) // 3, bind=False,
                                  summary=summ)
    else:
        from paper_1709_02125_amd import hydro3d as hm
        n = (16, 12, 120)
        make = lambda: hm.Hydro3D(n, np.full(n[::-1], 0.2), np.full(n[::-1], 1.0),
                                  budget=hm.device_footprint_bytes(n) // 3, bind=False)
    plans = []
    for fold in (False, True):
        app = make()
        app.ctx.set_flags(ooc.FLAG_CYCLIC, 0)
        app.queue_step()
        if fold:
            if dim == "2-summary":
                app.queue_summary()
            else:
                app.queue_mass()
        plans.append(app.ctx.debug_plan())
        app.close()
    step, folded = plans
    assert folded["nloops"] == step["nloops"] + 1
    assert folded["ntiles"] == step["ntiles"]
    for key in ("up", "down"):
        assert np.array_equal(folded[key], step[key]), key


CENTRINGS3 = [(0, 0, 0), (1, 1, 1), (1, 0, 0), (0, 1, 0), (0, 0, 1)]


def random_chain3(n, shapes, rng, nloops):
    """Random valid toy loops in 3D (AVG / INC_ADD / MIRROR / FILL), tiled along z."""
    fields = list(shapes)

    def ext(cen):
        return [(-H, n[a] + H + cen[a]) for a in range(3)]

    loops, tries = [], 0
    while len(loops) < nloops and tries < 4000:
        tries += 1
        kind = rng.choice(["avg", "avg", "avg", "inc", "mirror", "fill"])
        fo = int(rng.choice(fields))
        eo = ext(shapes[fo])
        if kind == "fill":
            r = []
            for a in range(3):
                lo = int(rng.integers(eo[a][0], eo[a][1]))
                r.append((lo, int(rng.integers(lo + 1, eo[a][1] + 1))))
            loops.append(tile_sim.ToyLoop(tile_sim.K_FILL, tuple(r), [(fo, WRITE, ((0, 0, 0),))],
                                          [float(rng.standard_normal())]))
            continue
        if kind == "mirror":   # a boundary layer along one axis, read mirrored across it
            ax, low = int(rng.integers(3)), bool(rng.integers(2))
            dep = int(rng.integers(1, H + 1))
            r = list(eo)
            a0 = eo[ax][0] if low else eo[ax][1] - dep
            r[ax] = (a0, a0 + dep)
            off = [0, 0, 0]
            off[ax] = 2 * dep if low else -2 * dep
            loops.append(tile_sim.ToyLoop(tile_sim.K_MIRROR, tuple(r), [(fo, WRITE, ((0, 0, 0),)),
                                                                        (fo, READ, (tuple(off),))],
                                          [float(rng.choice([-1.0, 1.0]))]))
            continue
        fi = int(rng.choice([f for f in fields if f != fo] or fields))
        ei = ext(shapes[fi])
        if kind == "inc":
            offs = ((0, 0, 0),)
        else:
            offs = tuple(tuple(int(v) for v in rng.integers(-2, 3, size=3)) for _ in range(int(rng.integers(1, 5))))
        r = []
        for a in range(3):
            lo = max(eo[a][0], ei[a][0] - min(o[a] for o in offs))
            hi = min(eo[a][1], ei[a][1] - max(o[a] for o in offs))
            if hi <= lo:
                break
            if rng.random() < 0.6:
                r.append((lo, hi))
            else:
                a0 = int(rng.integers(lo, hi))
                r.append((a0, int(rng.integers(a0 + 1, hi + 1))))
        if len(r) < 3:
            continue
        if kind == "inc":
            loops.append(tile_sim.ToyLoop(tile_sim.K_INC_ADD, tuple(r), [(fo, INC, ((0, 0, 0),)), (fi, READ, offs)],
                                          [0.5]))
        else:
            loops.append(tile_sim.ToyLoop(tile_sim.K_AVG, tuple(r), [(fo, WRITE, ((0, 0, 0),)), (fi, READ, offs)],
                                          [float(rng.uniform(0.5, 1.5)), float(rng.standard_normal())]))
    return loops


@pytest.mark.parametrize("seed", range(6))
def test_random_3d_chains_tiled_along_z_equal_untiled(seed):
    # the planner's 3D form: tiles cut along z, plans replayed plane by plane
    # on NaN-poisoned host slots against the untiled program
    rng = np.random.default_rng(100 + seed)
    n = (int(rng.integers(3, 6)), int(rng.integers(3, 6)), int(rng.integers(5, 12)))
    nf = int(rng.integers(2, 5))
    cens = [CENTRINGS3[int(rng.integers(len(CENTRINGS3)))] for _ in range(nf)]
    loops = None
    cyclic = bool(seed % 2)
    planes = n[2] + 2 * H + 1
    for slots in (2, 3):
        for h in range(1, planes + 1, 2):
            c = ooc.Context(3, n, H, 1 << 30, ooc.FLAG_CYCLIC if cyclic else 0, bind=False)
            frng = np.random.default_rng(seed)
            host, shapes = {}, {}
            for f in range(nf):
                init = frng.standard_normal(c.field_shape_for(cens[f]))
                hnd = c.decl_field("f%d" % f, cens[f], init)
                host[hnd], shapes[hnd] = init, cens[f]
            if loops is None:
                loops = random_chain3(n, shapes, rng, int(rng.integers(3, 10)))
            c.set_schedule(tile_rows=h, slots=slots)
            queue(c, loops)
            p = c.debug_plan()
            ref = tile_sim.run_untiled3(loops, host, H)
            got = tile_sim.run_tiled3(loops, host, p, H, slots)
            for f in host:
                if cyclic and p["temporary"][f] and any(d[0] == f for lp in loops for d in lp.dats):
                    continue  # host copy intentionally stale
                assert np.array_equal(got[f], ref[f]), (seed, h, slots, f)
            for i, lp in enumerate(loops):
                lr = p["loop_rows"][i]
                assert lr[0, 0] == lp.rng[2][0] and lr[-1, 1] == lp.rng[2][1]
                assert all(lr[t, 1] == lr[t + 1, 0] for t in range(p["ntiles"] - 1))
            c.close()


@pytest.mark.parametrize("seed", range(8))
def test_random_chains_on_ring_slabs_equal_untiled(seed):
    # Ring slabs (OOC_FLAG_RING): the same random toy chains replayed with
    # one ring per field (row r at r mod R, no edge copy, new rows poisoned)
    # against the untiled program, 2D and 3D; every ring holds the rows of
    # the tiles the pipeline can have in flight.
    rng = np.random.default_rng(200 + seed)
    cyclic = bool(seed % 2)
    flags = ooc.FLAG_RING | (ooc.FLAG_CYCLIC if cyclic else 0)
    if seed < 5:
        nx, ny = int(rng.integers(3, 9)), int(rng.integers(5, 14))
        nf = int(rng.integers(2, 5))
        _, _, shapes = make_ctx(nx, ny, nf, np.random.default_rng(seed))
        loops = random_chain(nx, ny, shapes, rng, int(rng.integers(3, 12)))
        rows, ndim = ny + 2 * H + 1, 2
    else:
        n = (int(rng.integers(3, 6)), int(rng.integers(3, 6)), int(rng.integers(5, 12)))
        nf = int(rng.integers(2, 5))
        cens = [CENTRINGS3[int(rng.integers(len(CENTRINGS3)))] for _ in range(nf)]
        loops, rows, ndim = None, n[2] + 2 * H + 1, 3
    for slots in (2, 3):
        for h in range(1, rows + 1):
            if ndim == 2:
                c, host, shapes2 = make_ctx(nx, ny, nf, np.random.default_rng(seed), flags=flags)
            else:
                c = ooc.Context(3, n, H, 1 << 30, flags, bind=False)
                frng = np.random.default_rng(seed)
                host, shapes = {}, {}
                for f in range(nf):
                    init = frng.standard_normal(c.field_shape_for(cens[f]))
                    hnd = c.decl_field("f%d" % f, cens[f], init)
                    host[hnd], shapes[hnd] = init, cens[f]
                if loops is None:
                    loops = random_chain3(n, shapes, rng, int(rng.integers(3, 10)))
            c.set_schedule(tile_rows=h, slots=slots)
            queue(c, loops)
            p = c.debug_plan()
            assert p["ring"]
            ref = (tile_sim.run_untiled if ndim == 2 else tile_sim.run_untiled3)(loops, host, H)
            got = tile_sim.run_tiled_ring(loops, host, p, H, slots, ndim)
            for f in host:
                if cyclic and p["temporary"][f] and any(d[0] == f for lp in loops for d in lp.dats):
                    continue  # host copy intentionally stale
                assert np.array_equal(got[f], ref[f]), (seed, h, slots, f)
            c.close()


def test_ring_slabs_hold_taller_tiles_without_edge_copies():
    # The 15-field Navier-Stokes chain at 512^3 on a third of its footprint,
    # chains of 3 steps, 2 slots: rings hold each field's rows once, so the
    # same budget fits taller tiles than slots that each hold a copy of the
    # skew; ring sizes are whole multiples of the granule
    from paper_1709_02125_amd import ns3d as N
    n = 512
    budget = N.footprint_bytes(n, True) // 3
    rows = {}
    for ring in (False, True):
        app = N.NS3D(n, None, budget=budget, flags=ooc.FLAG_RING if ring else 0, plan_only=True, fused=True)
        app.ctx.set_flags(ooc.FLAG_CYCLIC, 0)
        app.ctx.set_schedule(tile_rows=0, chain_steps=3, slots=2)
        for _ in range(3):
            app.queue_step()
        p = app.ctx.debug_plan()
        assert p["ring"] == ring
        assert p["slot_bytes"] * (1 if ring else p["slots"]) <= budget
        if ring:
            plane = ooc.row_pitch(n, N.NH) * (n + 2 * N.NH + 1) * 8
            assert (p["ring_rows"] > 0).sum() == 15
        rows[ring] = p["tile_rows"]
        app.close()
    assert rows[True] >= 2 * rows[False], rows
