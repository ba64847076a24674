"""Autotuner for the launch geometry and the V-cycle damping of a plan.

The quantity minimised is the predicted time to tolerance: (device time per outer step)
x (outer steps to reach tol at the contraction rate measured over a few probe steps).
The grid targets change only how the sweeping kernels are cut into workgroups; the
Jacobi damping omega of the cycle also changes the inner approximation and hence the
contraction rate, which is why the rate is measured rather than assumed.

The search is coordinate-wise (the inner method, omega, the slot-vector grid, the time-axis
grid, then per-sweep overrides of the slot grid for the restriction, up and operator sweeps,
whose best workgroup counts differ), each over a short candidate list, starting from the
library defaults. The
inner method axis compares the one-step Galerkin step on a V(0,1) and on a V(1,1) cycle with
COCG of a few steps and with COCG stopped per frequency at a relative tolerance: more inner
work per step against fewer outer steps, which is what the predicted time to tolerance
weighs. Results are kept in a plain JSON table keyed by grid, period, batch size and
precision.
"""
from __future__ import annotations

import json
import math
import os
from typing import Callable, Dict, List, Optional, Sequence

# The damping changes the contraction rate, and a rate measured over a dozen probe steps
# predicts the rate of the whole solve poorly, so it is searched only on request.
OMEGAS = (0.8,)
GRID_SLOT = (1024, 2048, 4096, 8192, 16384)
# per-sweep overrides of the slot grid (0 = the slot grid): restriction, up sweep, operator sweep
GRID_SWEEP = (0, 2048, 4096, 16384)
GRID_TEAM = (16384, 65536, 262144, 1048576)
# inner methods: (inner, inner_iters, inner_rtol, cycle); COCG needs the symmetric V(1,1)
INNER = (("galerkin1", 1, 0.0, "v01"), ("galerkin1", 1, 0.0, "v11"), ("cocg", 2, 0.0, "v11"),
         ("cocg", 4, 0.1, "v11"))


def _probe(make_plan: Callable, kw: Dict, steps: int, tol: float) -> Dict:
    import torch
    short = max(2, steps // 2)
    plan = make_plan(max_outer=short, **kw)
    try:
        plan.solve(raise_on_error=False)                     # warm-up (and graph capture)
        _, a = plan.solve(raise_on_error=False)
        plan.close()
        plan = make_plan(max_outer=steps, **kw)
        plan.solve(raise_on_error=False)
        _, b = plan.solve(raise_on_error=False)
    finally:
        plan.close()
        torch.cuda.empty_cache()
    a = a[0] if isinstance(a, list) else a
    bl = b if isinstance(b, list) else [b]
    step_ms = max(1e-6, (bl[0].time_ms - a.time_ms) / (steps - short))
    # slowest instance decides the batch: its rate over the probe steps (skipping the first two)
    rate = 0.0
    for s in bl:
        h = s.history
        if len(h) > 3 and h[2] > 0 and h[-1] > 0:
            rate = max(rate, (h[-1] / h[2]) ** (1.0 / (len(h) - 3)))
    rate = min(max(rate, 1e-3), 0.9999)
    need = math.log(tol) / math.log(rate)
    return {"step_ms": step_ms, "rate": rate, "steps_to_tol": need, "cost_ms": step_ms * need}


def tune(make_plan: Callable, *, tol: float = 1e-8, steps: int = 12, omegas: Sequence[float] = OMEGAS,
         grid_slot: Sequence[int] = GRID_SLOT, grid_team: Sequence[int] = GRID_TEAM,
         grid_sweep: Sequence[int] = GRID_SWEEP, inner: Sequence = INNER, log=None) -> Dict:
    """make_plan(max_outer=..., vc_omega=..., grid_slot=..., grid_team=..., grid_restrict=..., grid_up=...,
    grid_matvec=..., inner=..., inner_iters=..., inner_rtol=..., cycle=...) -> Plan or BatchPlan.
    Returns {"best": kwargs, "trials": [...]}."""
    best = {"inner": "galerkin1", "inner_iters": 1, "inner_rtol": 0.0, "cycle": "v01", "vc_omega": 0.8,
            "grid_slot": 0, "grid_team": 0, "grid_restrict": 0, "grid_up": 0, "grid_matvec": 0}
    trials: List[Dict] = []
    cache = {}

    def run(kw):
        key = tuple(sorted(kw.items()))
        if key not in cache:
            r = _probe(make_plan, kw, steps, tol)
            r.update(kw)
            cache[key] = r
            trials.append(r)
            if log:
                log(f"tune {kw}: {r['step_ms']:.3f} ms/step, rate {r['rate']:.4f}, "
                    f"predicted {r['cost_ms']:.1f} ms")
        return cache[key]["cost_ms"]

    scores = {}
    for c in inner:
        kw = dict(best, inner=c[0], inner_iters=c[1], inner_rtol=c[2], cycle=c[3])
        scores[c] = run(kw)
    c = min(scores, key=scores.get)
    best.update(inner=c[0], inner_iters=c[1], inner_rtol=c[2], cycle=c[3])
    for name, cands in (("vc_omega", omegas), ("grid_slot", grid_slot), ("grid_team", grid_team),
                        ("grid_restrict", grid_sweep), ("grid_up", grid_sweep), ("grid_matvec", grid_sweep)):
        scores = {}
        for c in cands:
            kw = dict(best)
            kw[name] = c
            scores[c] = run(kw)
        best[name] = min(scores, key=scores.get)
    return {"best": best, "trials": trials}


def load_table(path: str) -> Dict:
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def save_table(path: str, table: Dict) -> None:
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)


def tune_many(problems, precision: str, tol: float = 1e-8, table: Optional[Dict] = None, log=None,
              **search) -> Dict:
    """Tune every distinct batch plan (grid, period, batch size) that the work-list solver
    forms for `problems`; returns the table (updated in place if given)."""
    from . import BatchPlan
    from .batch import plan_groups, tune_key
    table = {} if table is None else table
    for ix in plan_groups(problems):
        key = tune_key(problems[ix[0]], len(ix), precision)
        if key in table:
            continue
        members = [problems[i] for i in ix]

        def make(max_outer, members=members, **kw):
            return BatchPlan(members, precision=precision, tol=tol, max_outer=max_outer, graph=True, **kw)

        r = tune(make, tol=tol, log=log, **search)
        table[key] = r["best"]
        if log:
            log(f"{key}: {r['best']}")
    return table


def main():
    import argparse
    import sys
    ap = argparse.ArgumentParser(description="tune the plans of a seeded workload: the 64-instance batching "
                                             "set (c4) or the 1024^2 x 512 single problem (c3)")
    ap.add_argument("--workload", default="c4", choices=["c3", "c4"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", default="fp32,fp64")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    import torch
    import workloads as W
    assert torch.cuda.is_available(), "tuning needs a GPU"
    problems = W.config4(args.seed) if args.workload == "c4" else [W.config3(args.seed)]
    table = load_table(args.out)
    say = lambda m: print(m, file=sys.stderr, flush=True)
    for prec in [p.strip() for p in args.precision.split(",") if p.strip()]:
        tune_many(problems, prec, args.tol, table, log=say)
        save_table(args.out, table)
    say(f"wrote {args.out}")


if __name__ == "__main__":
    main()
