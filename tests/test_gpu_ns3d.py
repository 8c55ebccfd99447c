"""GPU parity of the 3D Navier-Stokes proxy: HIP library vs the CPU oracle
(1e-12 per field), and tiled / multi-step chains vs in-core (bit-exact)."""
import numpy as np
import pytest

import oracle.ns3d as on
from paper_1709_02125_amd import ns3d as N, ooc
from paper_1709_02125_amd.inputs import tgv_initial_state
from gpu_util import GRAPH_OFF, rel_err, say

pytestmark = pytest.mark.gpu
TOL = 1e-12


def gpu_ns(n, steps, tile_rows=0, chain_steps=0, slots=0, incore=False, flags=0, budget=None, prims=None,
           fused=False):
    prims = prims if prims is not None else tgv_initial_state(n)
    if incore:
        flags |= ooc.FLAG_INCORE
        budget = N.device_footprint_bytes(n, fused)
    elif budget is None:
        budget = 8 * N.device_footprint_bytes(n, fused)
    app = N.NS3D(n, prims, budget=budget, flags=flags, fused=fused)
    app.ctx.set_schedule(tile_rows=tile_rows, chain_steps=chain_steps, slots=slots)
    app.initialise()
    app.run(steps)
    out = {q: app.interior(q) for q in N.Q}
    st = app.ctx.stats()
    assert st["host_pageable_bytes"] == 0 and st["host_pinned_bytes"] > 0, st
    app.close()
    return out, st


def test_ns3d_tiled_matches_oracle():
    n, steps = 24, 2
    say("case: ns3d 24^3 tiled vs oracle")
    got, st = gpu_ns(n, steps, tile_rows=6, chain_steps=1)
    assert st["ntiles_last"] >= 3
    o = on.NS3D(n)
    o.set_primitives(*tgv_initial_state(n))
    for _ in range(steps):
        o.step(on.stable_dt(n))
    for q in N.Q:
        e = rel_err(got[q], o.interior(q))
        say(q, e)
        assert e <= TOL, q


@pytest.mark.parametrize("tile_rows,chain_steps,slots,flags", [
    (2, 1, 3, ooc.FLAG_PREFETCH), (3, 2, 2, ooc.FLAG_PREFETCH), (5, 2, 4, 0), (7, 3, 3, ooc.FLAG_PREFETCH),
    (0, 1, 3, 0), (4, 1, 3, ooc.FLAG_FUSE), (6, 2, 3, ooc.FLAG_KERNEL_COPY | ooc.FLAG_PREFETCH),
    (6, 2, 2, ooc.FLAG_RING | ooc.FLAG_PREFETCH), (3, 3, 3, ooc.FLAG_RING | ooc.FLAG_DEBUG_POISON),
    # one step per chain on rings with Prefetch: each chain's first tiles
    # start before the previous chain's last downloads (rotated ring origins)
    (4, 1, 2, ooc.FLAG_RING | ooc.FLAG_PREFETCH | ooc.FLAG_DEBUG_POISON), (2, 1, 3, ooc.FLAG_RING | ooc.FLAG_PREFETCH),
    # downloads by runtime memcpy calls instead of the copy kernel
    (6, 2, 2, ooc.FLAG_RING | ooc.FLAG_PREFETCH | ooc.FLAG_MEMCPY_DOWNLOAD),
    (5, 3, 3, ooc.FLAG_PREFETCH | ooc.FLAG_MEMCPY_DOWNLOAD),
    pytest.param(4, 1, 3, ooc.FLAG_FUSE | ooc.FLAG_GRAPH, marks=GRAPH_OFF)])
def test_ns3d_tiled_equals_incore(tile_rows, chain_steps, slots, flags):
    n, steps = 20, 3
    say("case: ns3d tiled vs in-core", tile_rows, chain_steps, slots, flags)
    ref, _ = gpu_ns(n, steps, incore=True)
    got, st = gpu_ns(n, steps, tile_rows=tile_rows, chain_steps=chain_steps, slots=slots,
                     flags=flags, budget=16 * N.device_footprint_bytes(n))
    for q in N.Q:
        assert np.array_equal(got[q], ref[q]), q


def test_ns3d_conserves_mass_and_energy_on_gpu():
    n, steps = 24, 4
    say("case: ns3d conservation")
    prims = tgv_initial_state(n)
    z, _ = gpu_ns(n, 0, incore=True, prims=prims)
    got, _ = gpu_ns(n, steps, tile_rows=4, chain_steps=2, prims=prims)
    for q in ("q_r", "q_re"):
        m0, m1 = z[q].sum(), got[q].sum()
        assert abs(m1 - m0) <= 1e-13 * abs(m0), q


def test_ns3d_two_block_columns_match_oracle_and_incore():
    # x spans two 64-wide block columns with a ragged tail (72 = 64 + 8; the
    # gradients' range starts at -2), so the marching kernels' x-halo loads
    # cross blocks; tiled with 2-step chains against in-core (bit-exact) and
    # in-core against the oracle
    n, steps = 72, 2
    say("case: ns3d 72^3 two block columns, tiled vs in-core vs oracle")
    got, st = gpu_ns(n, steps, tile_rows=9, chain_steps=2)
    ref, _ = gpu_ns(n, steps, incore=True)
    assert st["ntiles_last"] >= 4
    o = on.NS3D(n)
    o.set_primitives(*tgv_initial_state(n))
    for _ in range(steps):
        o.step(on.stable_dt(n))
    for q in N.Q:
        assert np.array_equal(got[q], ref[q]), q
        e = rel_err(ref[q], o.interior(q))
        say(q, e)
        assert e <= TOL, q



@pytest.mark.parametrize("tile_rows,chain_steps,slots,flags", [
    (0, 1, 3, 0), (3, 2, 2, ooc.FLAG_PREFETCH), (5, 3, 2, ooc.FLAG_PREFETCH), (7, 1, 4, ooc.FLAG_FUSE),
    (4, 3, 2, ooc.FLAG_RING | ooc.FLAG_PREFETCH), (6, 2, 3, ooc.FLAG_RING | ooc.FLAG_DEBUG_POISON)])
def test_ns3d_fused_residual_equals_stored_gradients(tile_rows, chain_steps, slots, flags):
    # The residual that evaluates the gradients itself (15 fields) against
    # the chain with the 12 stored gradient fields: bit for bit, in core and
    # tiled over several schedules
    n, steps = 20, 3
    say("case: ns3d fused residual vs stored gradients", tile_rows, chain_steps, slots, flags)
    ref, _ = gpu_ns(n, steps, incore=True)
    inc, _ = gpu_ns(n, steps, incore=True, fused=True)
    got, st = gpu_ns(n, steps, tile_rows=tile_rows, chain_steps=chain_steps, slots=slots, flags=flags,
                     budget=16 * N.device_footprint_bytes(n, True), fused=True)
    for q in N.Q:
        assert np.array_equal(inc[q], ref[q]), q
        assert np.array_equal(got[q], ref[q]), q


@pytest.mark.parametrize("tile_rows,chain_steps,slots,flags", [
    (4, 2, 3, 0), (3, 2, 2, ooc.FLAG_PREFETCH), (7, 2, 4, ooc.FLAG_FUSE),
    (5, 4, 3, ooc.FLAG_RING | ooc.FLAG_PREFETCH | ooc.FLAG_MEMCPY_DOWNLOAD),
    (4, 2, 2, ooc.FLAG_RING | ooc.FLAG_DEBUG_POISON), (6, 4, 3, ooc.FLAG_RING | ooc.FLAG_PREFETCH)])
def test_ns3d_conserved_input_residual_equals_fused(tile_rows, chain_steps, slots, flags):
    # The residual that evaluates the primitives as well (one copy of the
    # conserved variables in, the other out; no primitive fields or loop in
    # the chain) against the fused form with stored primitives: bit for bit,
    # in core (also after an odd number of steps, the state then in the other
    # copy) and tiled over several schedules with chains of even length
    n = 20
    say("case: ns3d conserved-input residual vs fused", tile_rows, chain_steps, slots, flags)
    for steps in (3, 4):
        ref, _ = gpu_ns(n, steps, incore=True, fused=True)
        inc, _ = gpu_ns(n, steps, incore=True, fused="q")
        for q in N.Q:
            assert np.array_equal(inc[q], ref[q]), (steps, q)
    got, st = gpu_ns(n, 4, tile_rows=tile_rows, chain_steps=chain_steps, slots=slots, flags=flags,
                     budget=16 * N.device_footprint_bytes(n, "q"), fused="q")
    assert st["ntiles_last"] >= 3
    for q in N.Q:
        assert np.array_equal(got[q], ref[q]), q


def test_ns3d_conserved_input_odd_chains_under_cyclic_are_refused():
    # With Cyclic, a chain of an odd number of steps leaves the state in the
    # copy its first stage writes, which Cyclic takes for a temporary and does
    # not download: the library refuses to read that field afterwards
    say("case: ns3d conserved-input residual, odd chain under Cyclic")
    n = 20
    app = N.NS3D(n, tgv_initial_state(n), budget=8 * N.device_footprint_bytes(n, "q"), fused="q")
    try:
        app.ctx.set_schedule(tile_rows=5, chain_steps=1)
        app.initialise()
        with pytest.raises(ooc.OocError) as e:
            app.run(3)
        assert e.value.code == ooc.E_STALE
    finally:
        app.close()


def test_ns3d_conserved_input_two_block_columns_match_oracle():
    n, steps = 72, 2
    say("case: ns3d 72^3 conserved-input residual, tiled vs oracle")
    got, st = gpu_ns(n, steps, tile_rows=9, chain_steps=2, fused="q", flags=ooc.FLAG_RING | ooc.FLAG_PREFETCH)
    assert st["ntiles_last"] >= 4
    o = on.NS3D(n)
    o.set_primitives(*tgv_initial_state(n))
    for _ in range(steps):
        o.step(on.stable_dt(n))
    for q in N.Q:
        e = rel_err(got[q], o.interior(q))
        say(q, e)
        assert e <= TOL, q


def test_ns3d_fused_two_block_columns_match_oracle():
    # x over two 64-wide block columns with a ragged tail, tiled with 2-step
    # chains: the fused residual against the oracle and, bit for bit, against
    # the stored-gradient chain in core
    n, steps = 72, 2
    say("case: ns3d 72^3 fused residual, tiled vs oracle vs stored gradients")
    got, st = gpu_ns(n, steps, tile_rows=9, chain_steps=2, fused=True)
    ref, _ = gpu_ns(n, steps, incore=True)
    assert st["ntiles_last"] >= 4
    o = on.NS3D(n)
    o.set_primitives(*tgv_initial_state(n))
    for _ in range(steps):
        o.step(on.stable_dt(n))
    for q in N.Q:
        e = rel_err(got[q], o.interior(q))
        say(q, e)
        assert e <= TOL, q
        assert np.array_equal(got[q], ref[q]), q


@pytest.mark.parametrize("k,ring,dl", [(6, False, 0), (2, False, 0), (2, True, 0), (2, True, ooc.FLAG_MEMCPY_DOWNLOAD),
                                       (6, False, ooc.FLAG_MEMCPY_DOWNLOAD)])
def test_ns3d_fp32_streaming_matches_oracle_with_the_same_roundings(k, ring, dl):
    # Extension: the streamed fields are stored on the host and moved as
    # float32; compute stays float64 on the device.  The initial primitives
    # are rounded once on the way in, and every chain of k steps rounds the
    # conserved variables once on the way out, whatever the tiles -- so the
    # float64 oracle doing the same roundings gives the same values.  With
    # k = 6 the chain's kernels move more than 60x its link bytes and the
    # download kernel keeps 8-byte host stores; with k = 2 it uses 16-byte
    # stores; with runtime-copy downloads the rows are rounded into a staging
    # area first.
    n, steps = 24, 6
    say("case: ns3d fp32 streaming, chains of", k, "ring", ring, "runtime-copy downloads", bool(dl))
    prims = tgv_initial_state(n)
    flags = ooc.FLAG_FP32_STREAM | ooc.FLAG_PREFETCH | (ooc.FLAG_RING if ring else 0) | dl
    got, st = gpu_ns(n, steps, tile_rows=6, chain_steps=k, slots=2, flags=flags, prims=prims)
    assert st["ntiles_last"] >= 3
    if k == 6:
        other, _ = gpu_ns(n, steps, tile_rows=4, chain_steps=k, slots=3, flags=flags, prims=prims)
        for q in N.Q:
            assert np.array_equal(got[q], other[q]), q

    def r32(x):
        return np.asarray(x, dtype=np.float32).astype(np.float64)

    o = on.NS3D(n)
    o.set_primitives(*[r32(p) for p in prims])

    def round_conserved():
        for q in N.Q:
            fld = o.field(q)
            fld[...] = r32(fld)

    round_conserved()
    for s in range(steps):
        o.step(on.stable_dt(n))
        if (s + 1) % k == 0:
            round_conserved()
    for q in N.Q:
        e = rel_err(got[q], o.interior(q))
        say(q, e)
        assert e <= TOL, q


def test_ns3d_incore_cache_tiled_bit_exact():
    # every field resident, chains of 2 steps cut into skewed 5-plane tiles
    n, steps = 24, 2
    say("case: ns3d in-core, tiled for cache")
    ref, _ = gpu_ns(n, steps, incore=True, fused=True)
    got, st = gpu_ns(n, steps, incore=True, fused=True, tile_rows=5, chain_steps=2)
    assert st["ntiles_last"] >= 5
    for q in N.Q:
        assert np.array_equal(got[q], ref[q]), q


def test_ns3d_fp32_ring_schedule_changes_equal_slots():
    # Ring slabs keep their float32 staging areas across schedule changes only
    # while the allocation holds one area per slot at its stride: a
    # sweep-like sequence -- a long first tile, then a shorter one, then more
    # slots -- must end in the same state as the same sequence on slots (the
    # float32 roundings fall at the same chain ends)
    n = 24
    say("case: ns3d fp32 ring slabs across schedule changes")
    prims = tgv_initial_state(n)
    seq = [(2, 4, 2, 4), (6, 1, 2, 2), (6, 1, 3, 2), (4, 2, 4, 2)]
    outs = []
    for ring in (False, True):
        flags = ooc.FLAG_FP32_STREAM | ooc.FLAG_PREFETCH | (ooc.FLAG_RING if ring else 0)
        app = N.NS3D(n, prims, budget=16 * N.device_footprint_bytes(n, True), flags=flags, fused=True)
        app.initialise()
        for h, k, S, steps in seq:
            app.ctx.set_schedule(tile_rows=h, chain_steps=k, slots=S)
            app.run(steps)
        outs.append({q: app.interior(q) for q in N.Q})
        app.close()
    for q in N.Q:
        assert np.array_equal(outs[0][q], outs[1][q]), q
