"""Schedule search for a loop-chain workload (an extension beyond the paper).

A schedule is (tile height h, chain length k in time steps, slot count S).
`plan_features` describes a schedule from the library's own plan of one chain
(transfer bytes, edge bytes, skew, tiles, slot use) without running it, using
a plan-only context.  `sweep` is the exhaustive autotuner: it measures every
feasible schedule on the device.  `CostModel` wraps the library's
device-trained MLP (ooc_mlp_*): it learns log(seconds per cell-step) from the
sweep's records and proposes the schedule with the lowest prediction; the
exhaustive sweep is its fallback and the yardstick of its regret."""
from __future__ import annotations

import math
import time

import numpy as np

from . import ooc

FEATURE_NAMES = ["log2_h", "h_over_span", "tiles", "chain_steps", "slots", "slot_frac", "up_B_per_cell_step",
                 "down_B_per_cell_step", "edge_B_per_cell_step", "lead_over_h", "launches_per_step",
                 "inv_tiles"]


def plan_features(plan_ctx, queue_steps, cells, row_bytes, budget, h, k, S):
    """Features of schedule (h, k, S) for a workload whose loops
    `queue_steps(k)` queues on the plan-only context; None if infeasible."""
    try:
        plan_ctx.set_schedule(tile_rows=h, chain_steps=k, slots=S)
        queue_steps(k)
        p = plan_ctx.debug_plan()
    except ooc.OocError as e:
        plan_ctx.discard_queue()
        if e.code == ooc.E_BUDGET:
            return None
        raise
    plan_ctx.discard_queue()
    T = p["ntiles"]
    lr = p["loop_rows"]
    span = max(1, int(lr[:, -1, 1].max() - lr[:, 0, 0].min()))
    hh = p["tile_rows"] if p["tile_rows"] > 0 else span
    nrows = lambda runs: int((runs[:, 3] - runs[:, 2]).sum()) if len(runs) else 0
    denom = float(cells) * k
    up = nrows(p["up"]) * row_bytes / denom
    down = nrows(p["down"]) * row_bytes / denom
    edge = nrows(p["edge"]) * row_bytes / denom
    ends0 = lr[:, 0, 1]
    nonempty = ends0 > lr[:, 0, 0]
    lead = float(ends0[nonempty].max() - ends0[nonempty].min()) if nonempty.any() else 0.0
    launches = int((lr[:, :, 1] > lr[:, :, 0]).sum())
    return np.array([math.log2(hh), hh / span, T / 16.0, float(k), float(S), p["slot_bytes"] * S / budget,
                     up / 100.0, down / 100.0, edge / 100.0, lead / hh, launches / (100.0 * k), 1.0 / T])


def grid(hs, ks, ss):
    return [(h, k, s) for h in hs for k in ks for s in ss]


def measure(app, cells, h, k, S, chains=2):
    """Seconds per cell-step of schedule (h, k, S) on a live app (one warm-up
    chain, then `chains` timed chains issued back to back)."""
    import torch
    app.ctx.set_schedule(tile_rows=h, chain_steps=k, slots=S)
    app.run(k)  # warm-up: plan, argument table, first transfers
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    app.run(chains * k)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / (cells * chains * k)


def sweep(app, plan_ctx, queue_steps, cells, row_bytes, budget, candidates, chains=2, log=None, repeats=1):
    """Exhaustive autotuner: features and measured time of every feasible
    candidate (the fastest of `repeats` measurements, which filters the
    occasional chain whose downloads ran slow).  Returns a list of records."""
    recs = []
    for (h, k, S) in candidates:
        f = plan_features(plan_ctx, queue_steps, cells, row_bytes, budget, h, k, S)
        if f is None:
            continue
        try:
            t = min(measure(app, cells, h, k, S, chains) for _ in range(repeats))
        except ooc.OocError as e:
            if e.code == ooc.E_BUDGET:
                continue
            raise
        recs.append({"h": h, "k": k, "S": S, "features": f.tolist(), "sec_per_cell_step": t})
        if log:
            log("h=%d k=%d S=%d: %.3e s/cell-step" % (h, k, S, t))
    return recs


class CostModel:
    """The library's MLP on standardised plan features -> log time."""

    def __init__(self, n_hidden: int = 32, seed: int = 1709):
        self.n_hidden, self.seed = n_hidden, seed
        self.net = None

    def fit(self, records, epochs: int = 3000, lr: float = 3e-3) -> float:
        X = np.array([r["features"] for r in records], dtype=np.float64)
        y = np.log(np.array([r["sec_per_cell_step"] for r in records]))
        self.mu, self.sd = X.mean(0), X.std(0) + 1e-12
        self.ymu, self.ysd = y.mean(), y.std() + 1e-12
        if self.net is None:
            self.net = ooc.Mlp(X.shape[1], self.n_hidden, self.seed)
        return self.net.train((X - self.mu) / self.sd, (y - self.ymu) / self.ysd, epochs, lr)

    def predict(self, features) -> np.ndarray:
        X = np.atleast_2d(np.asarray(features, dtype=np.float64))
        return np.exp(self.net.predict((X - self.mu) / self.sd) * self.ysd + self.ymu)

    def propose(self, candidates_with_features):
        """candidates_with_features: list of ((h, k, S), features); returns
        the candidate with the lowest predicted time."""
        feats = np.array([f for _, f in candidates_with_features])
        pred = self.predict(feats)
        i = int(np.argmin(pred))
        return candidates_with_features[i][0], float(pred[i])

    def close(self):
        if self.net is not None:
            self.net.close()


def candidate_features(plan_ctx, queue_steps, cells, row_bytes, budget, candidates):
    """((h, k, S), features) of every candidate the budget admits, from
    planning alone (nothing runs)."""
    out = []
    for c in candidates:
        f = plan_features(plan_ctx, queue_steps, cells, row_bytes, budget, *c)
        if f is not None:
            out.append((c, f.tolist()))
    return out


def transfer_regret(train_records, target_records, n_hidden=32, seed=1709, epochs=4000, lr=3e-3):
    """Train the cost model on one sweep's records and let it pick among the
    schedules of another configuration (their features from planning alone);
    judge the pick against that configuration's exhaustive sweep.  Returns
    the pick, its regret against the best measured schedule of the target,
    and its gain over the target's default schedule."""
    model = CostModel(n_hidden=n_hidden, seed=seed)
    try:
        loss = model.fit(train_records, epochs=epochs, lr=lr)
        (h, k, S), pred = model.propose([((r["h"], r["k"], r["S"]), r["features"]) for r in target_records])
    finally:
        model.close()
    t = {(r["h"], r["k"], r["S"]): r["sec_per_cell_step"] for r in target_records}
    best = min(t, key=t.get)
    d = default_schedule(target_records)
    return {"loss": loss, "pick": [h, k, S], "predicted_sec_per_cell_step": pred,
            "measured_sec_per_cell_step": t[(h, k, S)], "best": list(best), "best_sec_per_cell_step": t[best],
            "regret": t[(h, k, S)] / t[best] - 1.0,
            "gain_over_default": (d["sec_per_cell_step"] / t[(h, k, S)]) if d else None}


def ensemble_transfer_regret(train_records, target_records, seeds=(1709, 1, 2), n_hidden=32, epochs=4000,
                             lr=3e-3):
    """As transfer_regret, with one cost model per seed: the pick minimises
    the mean of their predicted log times, which steadies it against the
    one initialisation that lands in a poor minimum of so few samples."""
    keys = [(r["h"], r["k"], r["S"]) for r in target_records]
    feats = [r["features"] for r in target_records]
    logs = []
    for seed in seeds:
        model = CostModel(n_hidden=n_hidden, seed=seed)
        try:
            model.fit(train_records, epochs=epochs, lr=lr)
            logs.append(np.log(model.predict(feats)))
        finally:
            model.close()
    i, mean = ensemble_pick(logs)
    h, k, S = keys[i]
    t = {kk: r["sec_per_cell_step"] for kk, r in zip(keys, target_records)}
    best = min(t, key=t.get)
    d = default_schedule(target_records)
    return {"seeds": list(seeds), "pick": [h, k, S], "predicted_sec_per_cell_step": float(np.exp(mean[i])),
            "measured_sec_per_cell_step": t[(h, k, S)], "best": list(best), "best_sec_per_cell_step": t[best],
            "regret": t[(h, k, S)] / t[best] - 1.0,
            "gain_over_default": (d["sec_per_cell_step"] / t[(h, k, S)]) if d else None}


def ensemble_pick(log_predictions):
    """Index of the candidate with the lowest mean predicted log time over
    the models (rows: models, columns: candidates; first index on ties), and
    the means."""
    mean = np.mean(np.asarray(log_predictions, dtype=np.float64), axis=0)
    return int(np.argmin(mean)), mean


def default_schedule(records):
    """The schedule the library uses without guidance: largest tile height
    that fits (h = 0), one step per chain, 3 slots -- or, where chains must
    span an even number of steps (the Navier-Stokes form with two copies of
    the conserved variables), two steps per chain."""
    for key in ((0, 1, 3), (0, 2, 3)):
        for r in records:
            if (r["h"], r["k"], r["S"]) == key:
                return r
    return None


def holdout_regret(records, train_frac=0.5, seed=1709, n_hidden=32, epochs=4000, lr=3e-3):
    """Train the cost model on a seeded subset of the measured schedules and
    let it pick among all of them (their features come from planning alone).
    Returns a dict with the pick, its regret against the best measured
    schedule, and its gain over the default schedule."""
    rng = np.random.default_rng(seed)
    idx = rng.permutation(len(records))
    ntr = max(4, int(round(train_frac * len(records))))
    train = [records[i] for i in idx[:ntr]]
    model = CostModel(n_hidden=n_hidden, seed=seed)
    try:
        loss = model.fit(train, epochs=epochs, lr=lr)
        (h, k, S), _ = model.propose([((r["h"], r["k"], r["S"]), r["features"]) for r in records])
    finally:
        model.close()
    t = {(r["h"], r["k"], r["S"]): r["sec_per_cell_step"] for r in records}
    best = min(t.values())
    d = default_schedule(records)
    return {"train": ntr, "of": len(records), "loss": loss, "pick": [h, k, S], "pick_in_train":
            any((r["h"], r["k"], r["S"]) == (h, k, S) for r in train),
            "regret": t[(h, k, S)] / best - 1.0,
            "gain_over_default": (d["sec_per_cell_step"] / t[(h, k, S)]) if d else None}


# ------------------------------------------------------------ workloads
def hydro2d_workload(n: int, budget: int, flags: int = 0, resident_geometry: bool = False):
    """The same for the 2D hydro proxy at n^2 (one step per chain: the time
    step is a reduction read by the next step); resident_geometry keeps the
    read-only geometry on the device."""
    from . import hydro2d as h2
    from .inputs import hydro_initial_state
    rho, ene = hydro_initial_state((n, n))
    app = h2.Hydro2D(n, n, rho, ene, budget=budget, flags=flags | ooc.FLAG_PREFETCH,
                     resident_geometry=resident_geometry)
    del rho, ene
    app.initialise()
    planner = h2.Hydro2D(n, n, None, None, budget=budget, flags=flags, plan_only=True,
                         resident_geometry=resident_geometry)
    planner.ctx.set_flags(ooc.FLAG_CYCLIC, 0)

    def queue_steps(k):
        for _ in range(k):
            planner.queue_step()

    pitch = ooc.row_pitch(n, h2.H)
    row_bytes = pitch * (4 if flags & ooc.FLAG_FP32_STREAM else 8)
    return app, planner.ctx, queue_steps, n * n, row_bytes


def ns3d_workload(n: int, budget: int, flags: int = 0, fused=False):
    """(live app, plan-only context, queue_steps, cells, row_bytes) for the
    Navier-Stokes proxy at n^3 (Taylor-Green input); fused: the 15-field
    chain whose residual evaluates the gradients itself."""
    from . import ns3d as N
    from .inputs import tgv_initial_state
    app = N.NS3D(n, tgv_initial_state(n), budget=budget, flags=flags | ooc.FLAG_PREFETCH, fused=fused)
    app.initialise()
    planner = N.NS3D(n, None, budget=budget, flags=flags, plan_only=True, fused=fused)
    planner.ctx.set_flags(ooc.FLAG_CYCLIC, 0)

    def queue_steps(k):
        for _ in range(k):
            planner.queue_step()

    pitch = ooc.row_pitch(n, N.NH)
    row_bytes = pitch * (n + 2 * N.NH + 1) * (4 if flags & ooc.FLAG_FP32_STREAM else 8)
    return app, planner.ctx, queue_steps, n ** 3, row_bytes


def main():
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="exhaustive schedule sweep + cost model")
    ap.add_argument("--workload", choices=["ns3d", "hydro2d"], default="ns3d")
    ap.add_argument("--n", type=int, default=0, help="cells per axis (default 512 for ns3d, 15360 for hydro2d)")
    ap.add_argument("--budget-frac", type=float, default=1.0 / 3.0)
    ap.add_argument("--hs", default="8,16,24,32,48,0")
    ap.add_argument("--ks", default="1,2,3")
    ap.add_argument("--ss", default="2,3,4")
    ap.add_argument("--chains", type=int, default=2)
    ap.add_argument("--fp32", action="store_true")
    ap.add_argument("--out", default="tune_records.json")
    a = ap.parse_args()
    flags = ooc.FLAG_FP32_STREAM if a.fp32 else 0
    log = lambda *x: print(*x, file=sys.stderr, flush=True)
    if a.workload == "ns3d":
        from . import ns3d as N
        a.n = a.n or 512
        budget = int(N.footprint_bytes(a.n) * a.budget_frac)
        app, plan_ctx, q, cells, rb = ns3d_workload(a.n, budget, flags)
    else:
        from . import hydro2d as h2
        a.n = a.n or 15360
        budget = int(h2.footprint_bytes(a.n, a.n) * a.budget_frac)
        app, plan_ctx, q, cells, rb = hydro2d_workload(a.n, budget, flags)
    cands = grid([int(x) for x in a.hs.split(",")], [int(x) for x in a.ks.split(",")],
                 [int(x) for x in a.ss.split(",")])
    recs = sweep(app, plan_ctx, q, cells, rb, budget, cands, a.chains, log)
    app.close()
    best = min(recs, key=lambda r: r["sec_per_cell_step"])
    log("best h=%d k=%d S=%d %.3e s/cell-step (%.3g updates/s)" %
        (best["h"], best["k"], best["S"], best["sec_per_cell_step"], 1.0 / best["sec_per_cell_step"]))
    learned = [holdout_regret(recs, 0.5, seed) for seed in (1, 2, 3)]
    for r in learned:
        log("cost model (trained on %d of %d): pick h=%d k=%d S=%d, regret %.3f, gain over default %s" %
            (r["train"], r["of"], *r["pick"], r["regret"],
             "%.3f" % r["gain_over_default"] if r["gain_over_default"] else "n/a"))
    with open(a.out, "w") as f:
        json.dump({"workload": a.workload, "n": a.n, "budget": budget, "fp32": a.fp32, "features": FEATURE_NAMES,
                   "records": recs, "best": [best["h"], best["k"], best["S"]], "learned": learned}, f)


if __name__ == "__main__":
    main()
