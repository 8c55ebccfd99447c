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
                                 tile_rows=0, slots=0, stored_gradients=False,
                                 stored_primitives=False)
    w = bench.WORKLOADS[name](args)
    assert w.cells > 0 and w.footprint > 0 and w.budget > 0
    assert name in w.describe()
    assert all(isinstance(k, int) and isinstance(v, str) for k, v in w.knames.items())
    val, sample = w.cpu_baseline(target_s=0.5)
    assert val > 0 and sample


def test_ooc_ceiling_is_the_slowest_stream():
    # hydro2d 15360^2 per cell and step: 1168 algorithmic HBM bytes, 56 B up
    # and 32 B down (FP64, every field streamed); probes 5000 / 57.5 / 57.1 GB/s
    cells = 15360 * 15360 * 20
    c = bench.ooc_ceiling(1.0e9, cells, 1168 * cells, 56 * cells, 32 * cells, 5000.0, 57.5, 57.1)
    assert c["bound"] == "h2d"
    assert c["value"] == pytest.approx(57.5e9 / 56)
    assert c["terms"]["hbm"] == round(5000e9 / 1168) and c["terms"]["d2h"] == round(57.1e9 / 32)
    assert c["frac"] == round(1.0e9 / (57.5e9 / 56), 3)
    # in core nothing crosses the link: HBM alone bounds it
    c = bench.ooc_ceiling(4.0e9, cells, 1168 * cells, 0, 0, 5000.0, 57.5, 57.1)
    assert c["bound"] == "hbm" and set(c["terms"]) == {"hbm"}


def test_ablation_variants_are_the_papers_combinations():
    names = [v[0] for v in bench.ablations(2)]
    assert names == ["no_prefetch_cyclic", "no_prefetch_no_cyclic"]
    assert all(flags == 0 for _, flags, _ in bench.ablations(2))   # Prefetch off in both
    assert bench.ablations(2)[1][2] == {"cyclic": False}


def test_benchmark_configurations_plan_as_measured():
    # The planner alone (no storage) at the benchmark sizes and budgets gives
    # the tile shapes the measured runs used, within the budget.
    from paper_1709_02125_amd import hydro2d as h2, hydro3d as h3, ns3d as N, ooc
    pf = ooc.FLAG_PREFETCH

    cases = []
    a = h2.Hydro2D(15360, 15360, None, None, budget=16_000_000_000, flags=pf, plan_only=True)
    cases.append((a, 1, 16_000_000_000, 9, 1730))
    a = h2.Hydro2D(15360, 15360, None, None, budget=16_000_000_000, flags=pf | ooc.FLAG_FP32_STREAM,
                   plan_only=True, resident_geometry=True)
    cases.append((a, 1, 16_000_000_000, 15, 1072))
    n3 = (640, 640, 640)
    a = h3.Hydro3D(n3, None, None, budget=h3.footprint_bytes(n3) // 3, flags=pf, plan_only=True)
    cases.append((a, 1, h3.footprint_bytes(n3) // 3, 10, 65))
    a = N.NS3D(512, None, budget=N.footprint_bytes(512) // 3, flags=pf, plan_only=True)
    a.ctx.set_schedule(tile_rows=24, chain_steps=3, slots=2)
    cases.append((a, 3, N.footprint_bytes(512) // 3, 22, 24))
    a = N.NS3D(512, None, budget=N.footprint_bytes(512, True) // 3, flags=pf, plan_only=True, fused=True)
    a.ctx.set_schedule(tile_rows=0, chain_steps=3, slots=2)
    cases.append((a, 3, N.footprint_bytes(512, True) // 3, 38, 14))
    for app, steps, budget, tiles, rows in cases:
        app.ctx.set_flags(ooc.FLAG_CYCLIC, 0)
        for _ in range(steps):
            app.queue_step()
        p = app.ctx.debug_plan()
        assert (p["ntiles"], p["tile_rows"]) == (tiles, rows)
        assert p["slots"] * p["slot_bytes"] <= budget
        app.close()


def test_committed_traffic_only_for_the_profiled_launch_shape():
    # the committed counter summaries match the current kernel sources and the
    # benchmark plans' bytes per launch; another tile shape gets no traffic
    for kernel, workload in (("h2d_pdv_corr", "hydro2d"), ("h3d_pdv_corr", "hydro3d"), ("ns_rhs_fusedq", "ns3d")):
        kv = {}
        for line in open(bench.os.path.join(bench.ROOT, "profiles", "%s_%s_traffic.txt" % (kernel, workload))):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        alg = int(kv["algorithmic_bytes_per_launch"])
        assert bench.committed_traffic(kernel, workload, alg) == float(kv["hbm_bytes_per_launch"])
        assert bench.committed_traffic(kernel, workload, alg * 1.01) is None
    assert bench.committed_traffic("no_such_kernel", "ns3d", 1) is None


def test_ensemble_pick_minimises_the_mean_log_prediction():
    from paper_1709_02125_amd import tune
    import numpy as np
    # model 0 alone would pick candidate 2, model 1 candidate 0; together
    # candidate 1 has the lowest mean log time
    logs = np.log([[4.0, 1.5, 1.0], [1.0, 1.5, 4.0]])
    i, mean = tune.ensemble_pick(logs)
    assert i == 1 and np.allclose(mean, (logs[0] + logs[1]) / 2)
    assert tune.ensemble_pick(np.log([[1.0, 1.0]]))[0] == 0  # ties: the first
