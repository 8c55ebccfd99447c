"""Host-side checks of the benchmark driver: the multi-GPU refusal, and every
workload's set-up, description, kernel names and CPU-oracle sample at a tiny
size (no device needed)."""
import subprocess
import sys
import types

import pytest

import bench


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], capture_output=True, text=True,
                       cwd=bench.ROOT)
    assert r.returncode == 2 and "one GPU" in r.stderr


@pytest.mark.parametrize("name,n", [("hydro2d", 64), ("hydro3d", 16), ("ns3d", 16)])
def test_workloads_build_on_host(name, n):
    args = types.SimpleNamespace(n=n, budget=0, resident_geometry=False, resident_state=False, no_cyclic=False, chain_steps=3,
                                 tile_rows=0, slots=0)
    w = bench.WORKLOADS[name](args)
    assert w.cells > 0 and w.footprint > 0 and w.budget > 0
    assert name in w.describe()
    assert all(isinstance(k, int) and isinstance(v, str) for k, v in w.knames.items())
    val, sample = w.cpu_baseline(target_s=0.5)
    assert val > 0 and sample
