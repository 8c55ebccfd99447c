"""GPU: random toy loop chains through the HIP library; every schedule must be
bit-identical to the plain untiled numpy run of the same toy loops."""
import numpy as np
import pytest

from paper_1709_02125_amd import ooc
import tile_sim
from gpu_util import say
from test_planner_host import CENTRINGS, H, queue, random_chain

pytestmark = pytest.mark.gpu


def make_ctx_bound(nx, ny, nf, seed, flags):
    """Same seeded declarations and data as test_planner_host.make_ctx, with
    the device bound."""
    rng = np.random.default_rng(seed)
    c = ooc.Context(2, (nx, ny), H, 1 << 26, flags)
    host, shapes = {}, {}
    for f in range(nf):
        cen = CENTRINGS[rng.integers(len(CENTRINGS))]
        init = rng.standard_normal(c.field_shape_for(cen))
        h = c.decl_field("f%d" % f, cen, init)
        host[h] = init
        shapes[h] = cen
    return c, host, shapes


@pytest.mark.parametrize("seed", range(8))
def test_random_chain_gpu_matches_untiled(seed):
    rng = np.random.default_rng(seed)
    nx, ny = int(rng.integers(3, 40)), int(rng.integers(5, 40))
    nf = int(rng.integers(2, 5))
    c0, _, shapes = make_ctx_bound(nx, ny, nf, seed, 0)
    c0.close()
    loops = random_chain(nx, ny, shapes, rng, int(rng.integers(3, 12)))
    rows = ny + 2 * H + 1
    for tile_rows, slots, flags in [(0, 3, ooc.FLAG_INCORE), (1, 2, 0), (3, 3, ooc.FLAG_DEBUG_POISON),
                                    (rows // 2 + 1, 4, 0), (5, 3, ooc.FLAG_CYCLIC),
                                    (2, 2, ooc.FLAG_RING | ooc.FLAG_DEBUG_POISON), (4, 3, ooc.FLAG_RING)]:
        say("case: toy seed", seed, "tile_rows", tile_rows, "slots", slots, "flags", flags)
        c, host, shapes2 = make_ctx_bound(nx, ny, nf, seed, flags)
        assert shapes2 == shapes
        c.set_schedule(tile_rows=tile_rows, slots=slots)
        queue(c, loops)
        p = c.debug_plan()
        c.execute()
        ref = tile_sim.run_untiled(loops, host, H)
        for f in host:
            if (flags & ooc.FLAG_CYCLIC) and p["temporary"][f] and \
                    any(d[0] == f for lp in loops for d in lp.dats):
                with pytest.raises(ooc.OocError):
                    c.fetch_field(f, shapes2[f])
                continue
            got = c.fetch_field(f, shapes2[f])
            assert np.array_equal(got, ref[f]), (seed, tile_rows, slots, flags, f)
        c.close()


@pytest.mark.parametrize("seed", range(6))
def test_prefetch_across_different_consecutive_chains(seed):
    # Speculative prefetch (Section 4.1, opt 3): a chain's first upload may
    # start while the previous chain still runs, ordered only after the
    # downloads of the host rows it reads.  Here three different random
    # chains (other fields, shifted ranges) follow each other in one flush,
    # split by step marks with one step per chain, so every chain's first
    # tile reads rows the previous chain's last tiles write and download.
    # Each schedule must equal the untiled run of all loops in order.
    rng = np.random.default_rng(100 + seed)
    nx, ny = int(rng.integers(3, 40)), int(rng.integers(12, 60))
    nf = int(rng.integers(3, 6))
    c0, _, shapes = make_ctx_bound(nx, ny, nf, 100 + seed, 0)
    c0.close()
    chains = [random_chain(nx, ny, shapes, rng, int(rng.integers(3, 10))) for _ in range(3)]
    rows = ny + 2 * H + 1
    for tile_rows, slots, flags in [(2, 2, ooc.FLAG_PREFETCH), (5, 3, ooc.FLAG_PREFETCH),
                                    (rows // 3 + 1, 4, ooc.FLAG_PREFETCH | ooc.FLAG_DEBUG_POISON),
                                    (3, 3, 0), (4, 2, ooc.FLAG_PREFETCH | ooc.FLAG_RING | ooc.FLAG_DEBUG_POISON),
                                    (2, 3, ooc.FLAG_PREFETCH | ooc.FLAG_RING)]:
        say("case: toy prefetch seed", seed, "tile_rows", tile_rows, "slots", slots, "flags", flags)
        c, host, shapes2 = make_ctx_bound(nx, ny, nf, 100 + seed, flags)
        assert shapes2 == shapes
        c.set_schedule(tile_rows=tile_rows, chain_steps=1, slots=slots)
        for ch in chains:
            queue(c, ch)
            c.mark_step()
        c.execute()
        assert c.stats()["chains"] == 3
        ref = tile_sim.run_untiled([lp for ch in chains for lp in ch], host, H)
        for f in host:
            assert np.array_equal(c.fetch_field(f, shapes2[f]), ref[f]), (seed, tile_rows, slots, flags, f)
        c.close()
