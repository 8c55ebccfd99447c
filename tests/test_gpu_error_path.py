"""GPU: the error path of a pipeline with work in flight.  A runtime call is
reported as failed from the host (ooc_debug_fail_after) after it was issued,
at several points of a tiled hydro2d run (set-up, inside the first chain,
deep inside later chains): the call returns OOC_E_DEVICE, every later call
OOC_E_FAILED, and ooc_destroy waits for the issued work and frees.  The device
itself never faults: every issued copy and kernel is valid and completes.
Afterwards a fresh context on the same device still matches the oracle."""
import numpy as np
import pytest

from paper_1709_02125_amd import hydro2d as h2, ooc
from paper_1709_02125_amd.inputs import hydro_initial_state
from gpu_util import gpu_hydro, oracle_hydro, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1, 9, 80, 700, 3000])
def test_injected_failure_fails_the_context_and_destroy_frees(n):
    nx, ny = 64, 72
    say("case: injected failure after %d checked runtime calls, hydro2d %dx%d" % (n, nx, ny))
    rho, ene = hydro_initial_state((nx, ny))
    app = h2.Hydro2D(nx, ny, rho, ene, budget=h2.device_footprint_bytes(nx, ny) // 3, flags=ooc.FLAG_PREFETCH)
    app.ctx.debug_fail_after(n)
    with pytest.raises(ooc.OocError) as e:
        app.initialise()
        app.run(4)
        app.fetch("rho0")
    assert e.value.code == ooc.E_DEVICE, e.value
    assert "injected" in str(e.value)
    with pytest.raises(ooc.OocError) as e2:
        app.ctx.execute()
    assert e2.value.code == ooc.E_FAILED
    app.close()
    say("destroyed after the failure")


def test_device_still_good_after_injected_failures():
    say("case: hydro2d 64x72 after the injected failures, vs oracle")
    got, dts, _ = gpu_hydro(64, 72, 3, flags=ooc.FLAG_PREFETCH)
    ref, odts = oracle_hydro(64, 72, 3)
    for k in got:
        assert rel_err(got[k], ref[k]) <= 1e-12, k
