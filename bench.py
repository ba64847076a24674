#!/usr/bin/env python3
"""Benchmark: space-time DoFs/s of the periodic solve to a relative residual of 1e-8.

One "step" is one complete solve of the time-periodic problem: the fixed-point iteration
(eqs. (iter1)-(iter2)) from U^0 = 0 until ||F - A(U)|| <= 1e-8 ||F||, i.e. every kernel of
the hot path (residual sweep + time DFT, batched V-cycle-preconditioned solve of all
frequency systems, inverse DFT + update, outer control) runs inside the timed region. The
inputs (problem tables, workspace) are resident in HBM before timing starts.

Workload: 1024 x 1024 cells (1,050,625 nodes), N = 512 time steps, seeded materials
(J0 and iron jitter from seed 0), 535,822,848 space-time DoFs (free nodes x N). Both the
FP32+refinement mode (reported as `value`) and the plain FP64 path are timed; both stop
on the same FP64 residual. The line states the error of each result: the relative L2
difference of the FP32+refinement and FP64 solutions, and of both against the FP64 CPU
oracle's solution on the 2x-coarsened copy (512 x 512 cells, N = 256, stored by
tests/golden/make_oracle_solutions.py) when that file is present.

Per-kernel durations come from HIP events that the library records on the solve stream: one
untimed solve brackets every launch (per-kernel pass), and the timed solves bracket the
launches of the two kernel classes with the most device time in that pass, from which the
roofline entry takes the dominant kernel. Each mode reports the mean wall time per solve over
the K timed solves (`ms_per_step`, `value`) and the median of their device times.
The CPU baseline is the FP64 oracle on a bounded sample of the same workload family, one
copy per host core, run before the GPU is touched.

Batching sub-record (`batching`, skipped with --no-batching; alone with --workload c4): the
64 seeded instances of uneven grid and period (n in {64,128,256,512}, N in {64,128,256},
J0 and iron corners seeded), grouped into batch plans and solved by the concurrent
work-list runner with graph replay; one step solves all 64 to 1e-8, in FP32+refinement and
FP64. It is compared with the plain FP64 path (each instance alone, eager launches, one
after the other; plans, workspaces and fields built and warmed up before timing), with its
own roofline (a serial pass with per-kernel events) and CPU baseline.

Loss-gradient workload (--workload c5): the differentiation-mode instance (256 x 256 cells, N = 256, a
log-normal per-cell nu scale); one step is one evaluation of the eddy-current loss and its per-cell
gradients (forward solve, adjoint solve, gradient kernels), with the roofline of the adjoint residual
sweep and the oracle's adjoint as the CPU baseline.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3|c2|c1|c4|c5|tr] [--paper-stop]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name, seed):
    import workloads as W
    if name == "c3":
        return W.config3(seed), "1024x1024 cells, N=512, seeded materials"
    if name == "c2":
        return W.config2(seed), "256x256 cells, N=256, seeded materials"
    if name == "c1":
        return W.config1(), "32x32 cells, N=32"
    if name == "tr":
        return (W.transformer(256, 512, khat_factor=TR_KHAT),
                f"transformer cross-section (Sec. 4 layout and exp-capped law on the unit square), 256x256 cells, "
                f"N=512, per-region Khat {TR_KHAT} nu(0)")
    raise SystemExit(f"unknown workload {name}")


TR_KHAT = 1.2   # the transformer workload's Khat coefficient per region, in units of the law at zero field


def run_many(P, problems, mode, steps, warmup, tol, nstreams, graph, tuning, trace_gap=0.0, **opts):
    """Time `steps` solves of all problems by the work-list runner; returns (timings, solver,
    last result). The solver is left open (its fields hold the last solutions). trace_gap: idle
    seconds between the warmup and the timed solves (marks the timed window in a kernel trace)."""
    import torch
    from paper_2502_21013_amd.batch import ManySolver
    ms = ManySolver(problems, precision=mode, tol=tol, max_outer=2000, graph=graph, nstreams=nstreams,
                    tuning=tuning, **opts)
    for w in range(warmup):
        r = ms.solve()
        log(f"{mode} many warmup {w}: {len(ms.plans)} plans, max outer "
            f"{max(s.outer_iters for s in r.stats)}")
    torch.cuda.synchronize()
    if trace_gap > 0:
        time.sleep(trace_gap)
    t0 = time.perf_counter()
    for k in range(steps):
        r = ms.solve()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = {"ms_per_step": 1e3 * wall / steps, "plans": len(ms.plans),
           "batch_sizes": [len(b) for b in ms.batches],
           "outer_iters_max": max(s.outer_iters for s in r.stats),
           "rel_residual_max": max(s.rel_residual for s in r.stats)}
    return out, ms, r


def run_plain_each(P, problems, steps, warmup, tol):
    """The plain FP64 path: each instance alone, eager launches, one after the other. Plans,
    workspaces and output fields are built, and every plan solved once, before the timer."""
    import torch
    plans = [P.Plan(p, tol=tol, precision="fp64", max_outer=2000) for p in problems]
    fields = [pl.new_time_field() for pl in plans]
    for pl in plans:
        pl.workspace()
    for w in range(warmup):
        for pl, U in zip(plans, fields):
            pl.solve(U)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outer = []
    for k in range(steps):
        outer = []
        for pl, U in zip(plans, fields):
            _, st = pl.solve(U)
            outer.append(st.outer_iters)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for pl in plans:
        pl.close()
    del plans, fields
    torch.cuda.empty_cache()
    return {"ms_per_step": 1e3 * wall / steps, "outer_iters_max": max(outer)}


def batch_roofline(P, problems, tol, tuning):
    """Per-kernel-class device time of one serial pass (one stream, eager launches with events)
    of the batching workload, against the algorithmic bytes of every launch: the dominant
    class's achieved bandwidth = its bytes over all plans / its time over all plans."""
    import torch
    _, ms, r = run_many(P, problems, "fp32", 1, 1, tol, 1, False, tuning, timing=True)
    by_cls_ms, by_cls_bytes, by_cls_n = {}, {}, {}
    for k, ix in enumerate(r.batches):
        st = r.stats[ix[0]]                      # every instance of a plan carries the plan's totals
        pr = problems[ix[0]]
        ab = algorithmic_bytes(pr, 8, len(ix))
        for name, b in ab.items():
            if name in st.kernel_ms:
                n = st.kernel_launches[name]
                by_cls_ms[name] = by_cls_ms.get(name, 0.0) + st.kernel_ms[name]
                by_cls_bytes[name] = by_cls_bytes.get(name, 0.0) + b * n
                by_cls_n[name] = by_cls_n.get(name, 0) + n
    ms.close()
    del ms
    torch.cuda.empty_cache()
    dom = max(by_cls_ms, key=by_cls_ms.get)
    gbs = by_cls_bytes[dom] / (by_cls_ms[dom] * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
            "launches": by_cls_n[dom], "alg_bytes_all_launches": by_cls_bytes[dom],
            "avg_launch_ms": round(by_cls_ms[dom] / by_cls_n[dom], 4),
            "note": "FP32+refinement, one stream, per-kernel HIP events; bytes and time summed over the "
                    "launches of all batch plans"}


def rel_l2_pairs(A, B):
    """(max over instance pairs of ||a - b|| / ||b||, index of that pair) (device tensors)."""
    worst, at = 0.0, -1
    for i, (a, b) in enumerate(zip(A, B)):
        nb = float(b.norm())
        e = float((a - b).norm()) / nb if nb > 0 else float((a - b).norm())
        if e > worst or at < 0:
            worst, at = e, i
    return worst, at


def batching_record(args, P, cpu=None):
    import torch
    import workloads as W
    from paper_2502_21013_amd import autotune as AT
    problems = W.config4(args.seed)
    total = sum(p.st_dofs for p in problems)
    log(f"batching workload: {len(problems)} instances, {total} space-time DoFs in total")
    tuning = AT.load_table(args.tuning) if args.tuning else None
    steps, warmup = args.c4_steps, args.c4_warmup
    res, sols = {}, {}
    for m in [x.strip() for x in args.c4_modes.split(",") if x.strip()]:
        res[m], ms, r = run_many(P, problems, m, steps, warmup, args.tol, args.streams, not args.no_graph, tuning,
                                 trace_gap=args.trace_gap)
        sols[m] = (ms, r)
        log(f"{m}: {res[m]['ms_per_step']:.1f} ms for all instances")
    err = worst = None
    if len(sols) == 2:
        err, at = rel_l2_pairs(sols["fp32"][1].U, sols["fp64"][1].U)
        # the instance where the modes differ most: its outer steps and final residuals in both modes
        worst = {"instance": at, **{m: {"outer_iters": sols[m][1].stats[at].outer_iters,
                                         "rel_residual": sols[m][1].stats[at].rel_residual} for m in sols}}
    for m in sols:
        sols[m][0].close()
    del sols
    torch.cuda.empty_cache()
    plain = roof = None
    if not args.no_plain:
        log("plain FP64 path, instance by instance")
        plain = run_plain_each(P, problems, steps, warmup, args.tol)
        log(f"plain fp64: {plain['ms_per_step']:.1f} ms")
        plain["value"] = total / (plain["ms_per_step"] * 1e-3)
    if not args.no_batch_roofline:
        log("batching roofline pass (one stream, per-kernel events)")
        roof = batch_roofline(P, problems, args.tol, tuning)
    first = next(iter(res))
    return {
        "workload": "64 seeded instances, n in {64,128,256,512}, N in {64,128,256}, J0 log-uniform in "
                    "[1,100], iron corners in [0.2,0.8]^2",
        "seed": args.seed, "st_dofs": total, "tol": args.tol, "steps": steps, "warmup": warmup,
        "streams": args.streams, "graph": not args.no_graph, "tuned": bool(tuning),
        "value": total / (res[first]["ms_per_step"] * 1e-3), "unit": "space-time DoFs/s",
        "ms_per_step": res[first]["ms_per_step"],
        "modes": {m: dict(res[m], value=total / (res[m]["ms_per_step"] * 1e-3)) for m in res},
        "plain_fp64_each": plain,
        "err_fp32_vs_fp64_max_rel_l2": err,
        "err_fp32_vs_fp64_worst_instance": worst,
        "roofline": roof,
        "cpu_baseline": cpu,
    }


def main_many(args, P, cpu=None):
    rec = batching_record(args, P, cpu)
    out = {
        "metric": "space-time DoFs/s to rel. residual 1e-8 (FP32+refine vs FP64); % HBM peak",
        "value": rec["value"], "unit": "space-time DoFs/s",
        "n_gpus": 1, "steps": rec["steps"], "warmup": rec["warmup"], "ms_per_step": rec["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "batching: " + rec["workload"], "seed": args.seed, "st_dofs": rec["st_dofs"],
                   "tol": args.tol, "streams": args.streams, "graph": rec["graph"], "tuned": rec["tuned"]},
        "roofline": rec["roofline"], "cpu_baseline": cpu,
        "modes": rec["modes"], "plain_fp64_each": rec["plain_fp64_each"],
        "err_fp32_vs_fp64_max_rel_l2": rec["err_fp32_vs_fp64_max_rel_l2"],
        "err_fp32_vs_fp64_worst_instance": rec["err_fp32_vs_fp64_worst_instance"],
    }
    print(json.dumps(out), flush=True)


def main_adjoint(args, P, cpu=None):
    """Config 5 (differentiation mode, 256^2 x 256, log-normal per-cell nu scale): one evaluation of the
    eddy-current loss and its gradients with respect to the per-cell nu scale and the conductivity is a
    forward solve, an adjoint solve (both to --tol) and the gradient kernels. Per mode: a per-kernel pass
    (every launch of both solves bracketed by HIP events), then --steps timed evaluations after --warmup.
    The roofline is taken on the adjoint residual sweep: U, lambda and dl/dU read (8 B each per DoF), the
    residual written in the solver precision."""
    import torch
    import workloads as W
    prob = W.config5(args.seed)
    theta = torch.from_numpy(prob.theta).to("cuda:0")
    nodes, N = (prob.n + 1) ** 2, prob.N
    modes = [m.strip() for m in args.modes.split(",") if m.strip()]
    rec, grads = {}, {}
    for m in modes:
        plan = P.Plan(prob, theta=theta, tol=args.tol, precision=m, adjoint=True, timing=True,
                      max_outer=args.max_outer)
        U, sf = plan.solve()
        Lam, sa = plan.adjoint_solve(U)
        adj_ms, adj_n = dict(sa.kernel_ms), dict(sa.kernel_launches)
        plan.close()
        del plan
        torch.cuda.empty_cache()
        plan = P.Plan(prob, theta=theta, tol=args.tol, precision=m, adjoint=True, max_outer=args.max_outer)
        U = plan.new_time_field()
        Lam = plan.new_time_field()
        def evaluate():
            _, f = plan.solve(U)
            _, a = plan.adjoint_solve(U, Lam)
            loss, gt, gs = plan.loss_gradients(U, Lam, per_cell=True)
            return f, a, loss, gt, gs
        for _ in range(args.warmup):
            evaluate()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            f, a, loss, gt, gs = evaluate()
            torch.cuda.synchronize()
            log(f"{m} evaluation {k}: forward {f.outer_iters} steps {f.time_ms:.1f} ms, adjoint {a.outer_iters} "
                f"steps {a.time_ms:.1f} ms, loss {loss:.6e}")
        wall = (time.perf_counter() - t0) / args.steps
        e = 8 if m == "fp32" else 16
        alg = nodes * N * (24 + e // 2)
        avg = adj_ms["residual_sweep"] / adj_n["residual_sweep"]
        rec[m] = {"value": prob.st_dofs / wall, "ms_per_step": 1e3 * wall, "forward_ms": f.time_ms,
                  "adjoint_ms": a.time_ms, "forward_outer_iters": f.outer_iters, "adjoint_outer_iters": a.outer_iters,
                  "rel_residual": f.rel_residual, "adjoint_rel_residual": a.rel_residual, "loss": loss,
                  "adjoint_kernel_ms_pass": adj_ms,
                  "roofline": {"bound": "hbm", "achieved": round(alg / (avg * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": round(alg / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                               "traffic": None, "kernel": "adjoint residual sweep (k_adj_residual)",
                               "alg_bytes_per_launch": alg, "avg_launch_ms": round(avg, 4)}}
        grads[m] = (gt.clone(), gs.clone(), loss)
        plan.close()
        del plan, U, Lam
        torch.cuda.empty_cache()
    errors = {}
    if "fp32" in grads and "fp64" in grads:
        (t32, s32, l32), (t64, s64, l64) = grads["fp32"], grads["fp64"]
        errors = {"loss_rel": abs(l32 - l64) / abs(l64),
                  "dl_dtheta_rel_l2": float((t32 - t64).norm() / t64.norm()),
                  "dl_dsigma_rel_l2": float((s32 - s64).norm() / s64.norm())}
    primary = modes[0]
    r0 = rec[primary]
    out = {
        "metric": "space-time DoFs/s of one loss-gradient evaluation (forward + adjoint solve to rel. residual "
                  "tol, then dl/dtheta and dl/dsigma per cell)",
        "value": r0["value"], "unit": "space-time DoFs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r0["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if primary == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": f"adjoint gradients: {prob.n}x{prob.n} cells, N={N}, log-normal per-cell nu scale "
                               f"(sd 0.1), seed {args.seed}", "st_dofs": prob.st_dofs, "tol": args.tol},
        "roofline": r0["roofline"], "cpu_baseline": cpu, "modes": rec, "errors": errors,
    }
    print(json.dumps(out), flush=True)


def algorithmic_bytes(p, elem, count=1):
    """Bytes each dominant kernel must move per launch (all (n+1)^2 grid nodes, `count`
    instances of the grid and period of p stacked in one batch plan).

    residual_sweep:           read U (8 B per node-time), write the residual spectrum R^ (its
                              packed DFT, fused into the sweep: elem per node-slot)
    rfft (packed DFT):        read R, write R^ (elem per node-slot each); outside the
                              fixed-point step (preconditioner applications of other solvers)
    vcycle_down_fine:         read r (fine), write r_c (coarse)
    vcycle_up_fine:           read r (fine), read x_c (coarse), write x (fine)
    matvec_dot:               read p (fine)
    inverse (DFT + update):   read p, read U, write U
    """
    n, N = p.n, p.N
    S = N // 2 * count
    nodes = (n + 1) ** 2
    nc = (n // 2 + 1) ** 2
    slot = nodes * S * elem
    cslot = nc * S * elem
    tfield = nodes * N * count * 8
    return {
        "residual_sweep": tfield + slot,
        "rfft": 2 * slot,
        "vcycle_down_fine": slot + cslot,
        "vcycle_up_fine": 2 * slot + cslot,
        "matvec_dot": slot,
        "inverse_rfft_update": slot + 2 * tfield,
    }


def _code_only(text):
    """C++ source without comments and whitespace runs (a comment edit is not a kernel change)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash(csrc=None):
    """Hash of the kernel sources' code (comments and layout ignored)."""
    h = hashlib.sha256()
    csrc = csrc or os.path.join(ROOT, "paper_2502_21013_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if not f.endswith((".hip", ".h")):
            continue
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            h.update(f.encode())
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def load_traffic(kernel, mode, wl):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary, or None
    when there is none for this workload or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "pmc_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        data = json.load(fh)
    if data.get("source_hash") != kernel_source_hash() or data.get("workload") != wl:
        return None
    ent = data.get("kernels", {}).get(mode, {}).get(kernel)
    if not ent:
        return None
    return ent.get("hbm_bytes_per_launch")


def run_mode(P, prob, mode, steps, warmup, tol, max_outer=2000, tuned=None, inner=None, extra=None):
    """Time `steps` solves after `warmup` untimed ones. Before them, one untimed solve with every
    kernel class bracketed by HIP events gives the per-class device times; the timed solves then
    bracket only the two classes with the most device time (two event records per launch of
    those, instead of around every launch), which is where the roofline kernel comes from."""
    import torch
    kw = dict(inner or {})
    kw.update(tuned or {})   # a tuning table entry overrides the inner method given on the command line
    kw.update(extra or {})   # problem tables (region ids) and the stopping protocol
    plan = P.Plan(prob, tol=tol, precision=mode, timing=True, max_outer=max_outer, **kw)
    U = plan.new_time_field()
    plan.workspace()
    _, st = plan.solve(U, raise_on_error=max_outer >= 2000)
    all_ms, all_n = dict(st.kernel_ms), dict(st.kernel_launches)
    # the two slowest of the kernels the roofline is taken on (in a run of a few steps, set-up
    # classes can outweigh them)
    rl = algorithmic_bytes(prob, 8)
    top = sorted((c for c in all_ms if c in rl), key=all_ms.get, reverse=True)[:2]
    log(f"{mode} per-kernel pass: outer={st.outer_iters} {st.time_ms:.1f} ms; timed classes {top}")
    plan.close()
    del plan, U
    torch.cuda.empty_cache()
    plan = P.Plan(prob, tol=tol, precision=mode, timing=tuple(top), max_outer=max_outer, **kw)
    U = plan.new_time_field()
    plan.workspace()
    for w in range(warmup):
        _, st = plan.solve(U, raise_on_error=max_outer >= 2000)
        log(f"{mode} warmup {w}: outer={st.outer_iters} rel={st.rel_residual:.3e} {st.time_ms:.1f} ms")
    kms, kcnt, outer, dev_ms, init = {}, {}, [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        _, st = plan.solve(U, raise_on_error=max_outer >= 2000)
        outer.append(st.outer_iters)
        dev_ms.append(st.time_ms)
        init.append(st.init_iters)
        for name, v in st.kernel_ms.items():
            kms[name] = kms.get(name, 0.0) + v
            kcnt[name] = kcnt.get(name, 0) + st.kernel_launches[name]
        log(f"{mode} step {k}: outer={st.outer_iters} rel={st.rel_residual:.3e} {st.time_ms:.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.close()
    del plan
    torch.cuda.empty_cache()
    return {"ms_per_step": 1e3 * wall / steps, "kernel_ms": kms, "kernel_launches": kcnt,
            "kernel_ms_pass": all_ms, "kernel_launches_pass": all_n, "solve_ms_device": dev_ms, "init_iters": init,
            "outer_iters": outer, "rel_residual": st.rel_residual, "U": U}


GOLDEN_HALF = os.path.join(ROOT, "tests", "golden", "oracle_c3half_seed0_n512_N256.npz")


def error_vs_oracle(P, seed, path=GOLDEN_HALF, tol=1e-11):
    """Relative L2 error of both modes against the FP64 CPU oracle's solution of the
    2x-coarsened copy of the workload (512^2 cells, N = 256; stored sampled slices and
    full-field sums), each mode solved on the GPU to `tol`. None when the file is absent."""
    import numpy as np
    import torch
    import workloads as W
    if not os.path.exists(path):
        return None
    z = np.load(path)
    meta = json.loads(str(z["meta"]))
    pr = meta["problem"]
    if pr["seed"] != seed:
        return None
    prob = W.with_size(W.config3(seed), pr["n"], pr["N"])
    idx, s = [int(j) for j in z["slice_idx"]], int(z["stride"])
    ref = z["slices"]
    out = {"workload": f"{pr['n']}x{pr['n']} cells, N={pr['N']} (2x-coarsened copy), seed {seed}",
           "oracle": meta["solver"], "oracle_rel_residual": meta["rel_final"], "gpu_tol": tol}
    for m in ("fp32", "fp64"):
        plan = P.Plan(prob, tol=tol, precision=m, max_outer=4000)
        U, st = plan.solve()
        g = U.cpu().numpy()
        plan.close()
        sl = np.stack([g[j, ::s, ::s] for j in idx])
        e_sl = float(np.linalg.norm(sl - ref) / np.linalg.norm(ref))
        nrm = float(np.sqrt(float((U * U).sum())))
        e_nrm = abs(nrm - float(np.sqrt(z["u_sq_sum"]))) / float(np.sqrt(z["u_sq_sum"]))
        out[m] = {"rel_l2_sampled_slices": e_sl, "rel_diff_full_norm": e_nrm, "outer_iters": st.outer_iters,
                  "rel_residual": st.rel_residual}
        del U
        torch.cuda.empty_cache()
    return out


PAPER_CONTEXT = {
    "note": "the paper's own timings of its method (M1): the same outer fixed-point iteration with "
            "multigrid in time for the periodic linear solves, on an unstructured transformer mesh "
            "with the exp-capped law, tol 1e-4 relative to a static start; a different problem, "
            "tolerance, inner solver and machine, quoted as context only",
    "hardware": "one node of LLNL Dane, 112-core Intel Sapphire Rapids; (M1) on 8 MPI ranks (tab:runtime), "
                "16-512 ranks over several nodes (tab:scaling)",
    "tab_runtime_M1": [
        {"N": 128, "N_V": 8208, "iters": 13, "seconds": 8.25036},
        {"N": 128, "N_V": 32451, "iters": 10, "seconds": 24.6771},
        {"N": 256, "N_V": 8208, "iters": 13, "seconds": 16.0703},
        {"N": 256, "N_V": 32451, "iters": 10, "seconds": 49.6497},
        {"N": 512, "N_V": 8208, "iters": 13, "seconds": 30.3863},
        {"N": 512, "N_V": 32451, "iters": 10, "seconds": 98.5296},
    ],
    "tab_scaling_M1_best": {"N": 2048, "N_V": 8208, "ranks": 512, "seconds": 5.04528},
    "derived_st_dofs_per_s": {"tab_runtime_max": 1.69e5, "tab_scaling_best": 3.3e6},
}


def _oracle_sample_worker(job):
    """One oracle solve of a bounded sample (one host thread); returns (DoFs, seconds, outer steps)."""
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import fem, periodic as pp
    kind, seed, n, N, tol = job
    if kind == "c4":
        base = W.config4(seed)[0]
    elif kind == "tr":
        base = W.transformer(n, N, khat_factor=TR_KHAT)
    elif kind == "c5":
        base = W.config5(seed, n, N)
    else:
        base = W.config3(seed)
    p = W.with_size(base, n, N) if kind != "c5" else base
    with threadpool_limits(1):
        t0 = time.perf_counter()
        d = fem.discretise(p)
        r = pp.fixed_point(d, tol=tol, max_iter=2000)
        if kind == "c5":
            from oracle import adjoint as AD
            AD.gradients(d, r.U)     # the adjoint state by sparse LU, then both gradients
        dt = time.perf_counter() - t0
    return p.st_dofs, dt, r.iters


def host_cores():
    try:
        c = len(os.sched_getaffinity(0))
    except AttributeError:
        c = os.cpu_count() or 1
    return max(1, min(16, c))


def cpu_baseline(kind, seed, n=32, N=64, tol=1e-8):
    """The FP64 oracle (space-time sparse LU inside the same fixed-point loop) on a bounded
    sample: one copy of the sample problem per host core (at most 16), run concurrently, each
    on one thread. Throughput = total DoFs / the longest solve time."""
    import concurrent.futures as cf
    import multiprocessing as mp
    cores = host_cores()
    jobs = [(kind, seed, n, N, tol)] * cores
    with cf.ProcessPoolExecutor(max_workers=cores, mp_context=mp.get_context("spawn")) as ex:
        res = list(ex.map(_oracle_sample_worker, jobs))
    dofs = sum(r[0] for r in res)
    tmax = max(r[1] for r in res)
    what = {"c4": "config-4 instance 0's materials and source",
            "tr": "the same transformer cross-section and per-region Khat",
            "c5": "a log-normal per-cell nu scale (the same recipe), forward solve + adjoint state + gradients"
            }.get(kind, "the same seeded materials/source")
    return {"value": dofs / tmax, "unit": "space-time DoFs/s", "cores": cores, "kind": "oracle",
            "sample": f"{cores} concurrent copies (one per host core, one thread each) of {n}x{n} cells, N={N}, "
                      f"{what}, tol {tol:g}, {res[0][2]} outer steps, longest {tmax:.1f} s "
                      f"(sparse LU of the space-time matrix + fixed point)"}


# ---------------------------------------------------------------- HBM traffic from rocprofv3 counters

KERNEL_CLASSES = [("k_residual", "residual_sweep"), ("k_rfft", "rfft"), ("k_vc_down", "vcycle_down_fine"),
                  ("k_vc_restrict", "vcycle_down_fine"), ("k_vc_up", "vcycle_up_fine"), ("k_matvec", "matvec_dot"),
                  ("k_inverse", "inverse_rfft_update")]


def _pmc_rows(db_path):
    """(kernel name, counter, value, duration) of every dispatch in a rocprofv3 --pmc database."""
    import re
    import sqlite3
    db = sqlite3.connect(db_path)
    cols = [d[1] for d in db.execute("pragma table_info(counters_collection)")]
    ni, vi, ci, di = (cols.index(c) for c in ("kernel_name", "value", "counter_name", "duration"))
    out = []
    for r in db.execute("select * from counters_collection"):
        out.append((re.sub(r"\(.*", "", r[ni]).replace("void ", ""), r[ci], float(r[vi]), float(r[di])))
    return out


def _per_class(rows, counter):
    """Average counter value (KiB) per dispatch of the finest-level launches of each kernel class:
    the dispatches lasting at least half as long as the longest one of that kernel."""
    res = {}
    for cls in dict.fromkeys(c for _, c in KERNEL_CLASSES):
        keys = [k for k, c in KERNEL_CLASSES if c == cls]
        ds = [(v, d) for (k, c, v, d) in rows if c == counter and any(key in k for key in keys)]
        if not ds:
            continue
        dmax = max(d for _, d in ds)
        vals = [v for v, d in ds if d >= 0.5 * dmax]
        res[cls] = sum(vals) / len(vals)
    return res


def trace_idle(csv_path, gap_ns=0.5e9):
    """Device busy time of the kernels of a rocprofv3 kernel trace (csv) in the window after the
    last idle gap of at least gap_ns: the union of the kernels' [start, end] intervals over the
    window's span (first start to last end). Kernels on different streams may overlap; the union
    counts the device as busy while any kernel runs."""
    import csv
    with open(csv_path, newline="") as fh:
        rows = list(csv.DictReader(fh))
    iv = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]) for r in rows)
    cut = 0
    reach = iv[0][1]
    for k in range(1, len(iv)):
        if iv[k][0] - reach >= gap_ns:
            cut = k
        reach = max(reach, iv[k][1])
    win = iv[cut:]
    busy, cs, ce = 0, win[0][0], win[0][1]
    for a, b, _ in win[1:]:
        if a > ce:
            busy += ce - cs
            cs, ce = a, b
        else:
            ce = max(ce, b)
    busy += ce - cs
    span = max(b for _, b, _ in win) - win[0][0]
    out = {"trace": os.path.basename(csv_path), "kernels_in_window": len(win), "window_ms": span / 1e6,
           "busy_ms": busy / 1e6, "idle_frac": 1.0 - busy / span}
    print(json.dumps(out), flush=True)
    return out


def copy_bandwidth(gib=2.0, reps=5):
    """Median bandwidth of a plain device-to-device copy (torch's copy kernel) of `gib` GiB, read
    + write bytes over the event time: the practical streaming rate of this device, beside the
    8 TB/s peak the roofline fractions use."""
    import torch
    n = int(gib * 2 ** 30)
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rates = []
    for _ in range(reps):
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        rates.append(2 * n / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del src, dst
    torch.cuda.empty_cache()
    return round(statistics.median(rates), 1)


def copy_calibration(gib=1.0, reps=3):
    """A plain device copy of a known size, for scaling FETCH_SIZE / WRITE_SIZE to bytes."""
    import torch
    n = int(gib * 2 ** 30)
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "reps": reps}), flush=True)


def pmc_summary(fetch_db, write_db, cal_fetch_db, cal_write_db, workload, mode, out, commands):
    """HBM bytes per launch of each kernel class: FETCH_SIZE and WRITE_SIZE (separate runs),
    each scaled by what the same counter reads for the 1 GiB calibration copy."""
    def copy_val(db, counter):
        vals = [v for (k, c, v, d) in _pmc_rows(db) if c == counter and ("copy" in k.lower() or "elementwise" in k)]
        return max(vals)
    n = 2 ** 30
    ff = n / (copy_val(cal_fetch_db, "FETCH_SIZE") * 1024.0)
    wf = n / (copy_val(cal_write_db, "WRITE_SIZE") * 1024.0)
    fe = _per_class(_pmc_rows(fetch_db), "FETCH_SIZE")
    wr = _per_class(_pmc_rows(write_db), "WRITE_SIZE")
    kern = {}
    for cls in fe:
        if cls in wr:
            fb, wb = fe[cls] * 1024.0 * ff, wr[cls] * 1024.0 * wf
            kern[cls] = {"fetch_kib": fe[cls], "write_kib": wr[cls], "read_bytes": fb, "write_bytes": wb,
                         "hbm_bytes_per_launch": fb + wb}
    data = {"source_hash": kernel_source_hash(), "workload": workload,
            "calibration": {"copy_bytes": n, "fetch_factor": ff, "write_factor": wf},
            "kernels": {mode: kern}, "commands": commands}
    with open(out, "w") as fh:
        json.dump(data, fh, indent=1)
    print(json.dumps(data), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--modes", default="fp32,fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--inner", default="galerkin1", choices=["galerkin1", "cocg"],
                    help="inner method of every periodic solve (default: the one-step Galerkin V-cycle)")
    ap.add_argument("--inner-iters", type=int, default=1, help="COCG steps per outer step (at most)")
    ap.add_argument("--inner-rtol", type=float, default=0.0, help="COCG per-frequency relative tolerance")
    ap.add_argument("--paper-stop", action="store_true",
                    help="the paper's protocol: start from the static solution, stop at --tol relative to its "
                         "residual (tab:runtime: 1e-4)")
    ap.add_argument("--cycle", default="default", choices=["default", "v11", "v01"],
                    help="multigrid cycle (default: V(0,1) with the Galerkin step, V(1,1) with COCG)")
    ap.add_argument("--no-batching", action="store_true", help="skip the batching sub-record")
    ap.add_argument("--no-oracle-error", action="store_true", help="skip the error against the oracle solution")
    ap.add_argument("--c4-modes", default="fp32,fp64", help="batching: modes (FP32+refinement first)")
    ap.add_argument("--no-plain", action="store_true", help="batching: skip the instance-by-instance FP64 run")
    ap.add_argument("--no-batch-roofline", action="store_true", help="batching: skip the per-kernel event pass")
    ap.add_argument("--trace-gap", type=float, default=0.0,
                    help="batching: idle seconds before the timed solves (marks them in a kernel trace)")
    ap.add_argument("--trace-idle", default="", metavar="KERNEL_TRACE_CSV",
                    help="only summarise a rocprofv3 kernel trace (csv): device busy and idle time of the "
                         "window after the last gap of at least 0.5 s")
    ap.add_argument("--c4-steps", type=int, default=2, help="batching: timed steps")
    ap.add_argument("--c4-warmup", type=int, default=1, help="batching: warmup steps")
    ap.add_argument("--streams", type=int, default=4, help="batching: host threads / HIP streams of the work list")
    ap.add_argument("--no-graph", action="store_true", help="batching: eager launches instead of graph replay")
    ap.add_argument("--tuning", default=os.path.join(ROOT, "paper_2502_21013_amd", "tuning_mi355x.json"),
                    help="autotuner table (JSON) to apply ('' for the library defaults)")
    ap.add_argument("--max-outer", type=int, default=2000,
                    help="cap on outer steps per solve; below the count needed for 1e-8 the run is a "
                         "profiling run (marked in the output), not a metric measurement")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration under rocprofv3 --pmc)")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH_DB", "WRITE_DB", "COPY_FETCH_DB", "COPY_WRITE_DB"),
                    help="write the HBM traffic table (--pmc-out) from four rocprofv3 --pmc databases")
    ap.add_argument("--pmc-out", default=os.path.join(ROOT, "profiles", "pmc_counters.json"))
    ap.add_argument("--pmc-commands", default="", help="the profiling commands, recorded in the table")
    args = ap.parse_args()
    if args.trace_idle:
        trace_idle(args.trace_idle)
        return
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary, workload=args.workload, mode=args.modes.split(",")[0], out=args.pmc_out,
                    commands=args.pmc_commands)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the multi-GPU sharding of this "
              "solver is a design note, not an implementation", file=sys.stderr)
        sys.exit(2)

    # CPU baselines first, in worker processes started before anything touches the GPU
    cpu = cpu4 = None
    want_batch = args.workload == "c4" or (args.workload == "c3" and not args.no_batching)
    if not args.no_cpu_baseline and not args.calibrate_copy:
        if args.workload != "c4":
            log("cpu baseline (oracle on a bounded sample, one copy per host core)")
            kind = args.workload if args.workload in ("tr", "c5") else "c3"
            cpu = cpu_baseline(kind, args.seed, N=32 if kind == "c5" else 64)
            log(f"cpu baseline {cpu['value']:.1f} DoFs/s on {cpu['cores']} cores")
        if want_batch:
            cpu4 = cpu_baseline("c4", args.seed)
            log(f"batching cpu baseline {cpu4['value']:.1f} DoFs/s on {cpu4['cores']} cores")

    import torch
    import paper_2502_21013_amd as P
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        copy_calibration()
        return
    P.library()
    if args.workload == "c4":
        main_many(args, P, cpu4)
        return
    if args.workload == "c5":
        main_adjoint(args, P, cpu)
        return
    import workloads as W
    prob, desc = workload(args.workload, args.seed)
    log(f"workload {args.workload}: {desc}, {prob.st_dofs} space-time DoFs")

    modes = [m.strip() for m in args.modes.split(",") if m.strip()]
    from paper_2502_21013_amd import autotune as AT
    from paper_2502_21013_amd.batch import tune_key
    table = AT.load_table(args.tuning) if args.tuning else {}
    inner = {"inner": args.inner, "inner_iters": args.inner_iters, "inner_rtol": args.inner_rtol, "cycle": args.cycle}
    extra = {}
    if prob.regions is not None:
        extra["region"] = torch.from_numpy(W.region_ids(prob)).to("cuda:0")
    if args.paper_stop:
        # Sec. 4: start from the static solution (sigma = 0) and stop relative to its residual
        extra.update(init_static=True, stop_relative_initial=True)
    res = {}
    for m in modes:
        tuned = table.get(tune_key(prob, 1, m))
        if tuned:
            log(f"{m}: tuned setting {tuned}")
        res[m] = run_mode(P, prob, m, args.steps, args.warmup, args.tol, args.max_outer, tuned, inner, extra)
        res[m]["tuned"] = tuned
        log(f"{m}: {res[m]['ms_per_step']:.1f} ms per solve")
    errors = {}
    if "fp32" in res and "fp64" in res:
        a, b = res["fp32"]["U"], res["fp64"]["U"]
        errors["fp32_vs_fp64_rel_l2"] = float((a - b).norm() / b.norm())
        log(f"rel L2 (FP32+refine vs FP64) {errors['fp32_vs_fp64_rel_l2']:.3e}")
    for m in res:
        res[m].pop("U")
    torch.cuda.empty_cache()
    if args.workload == "c3" and not args.no_oracle_error:
        ev = error_vs_oracle(P, args.seed)
        if ev:
            errors["vs_oracle_coarsened_copy"] = ev
            log(f"vs oracle (512^2 x 256): fp32 {ev['fp32']['rel_l2_sampled_slices']:.3e}, "
                f"fp64 {ev['fp64']['rel_l2_sampled_slices']:.3e}")

    primary = modes[0]
    r0 = res[primary]
    elem = 8 if primary == "fp32" else 16
    ab = algorithmic_bytes(prob, elem)
    def per_kernel(ms, cnt):
        out = {}
        for name, b in ab.items():
            if name in ms:
                avg_ms = ms[name] / cnt[name]
                out[name] = {"avg_ms": avg_ms, "launches": cnt[name], "total_ms": ms[name], "alg_bytes": b,
                             "achieved_gbs": b / (avg_ms * 1e-3) / 1e9}
        return out
    kern = per_kernel(r0["kernel_ms"], r0["kernel_launches"])              # timed region
    kern_pass = per_kernel(r0["kernel_ms_pass"], r0["kernel_launches_pass"])  # per-kernel pass
    roofline = None
    if kern:
        dom = max(kern, key=lambda k: kern[k]["total_ms"])
        dk = kern[dom]
        traffic = load_traffic(dom, primary, args.workload)
        copy_gbs = copy_bandwidth()
        roofline = {"bound": "hbm", "achieved": round(dk["achieved_gbs"], 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(dk["achieved_gbs"] / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "kernel": dom, "alg_bytes_per_launch": dk["alg_bytes"], "avg_launch_ms": round(dk["avg_ms"], 4),
                    "copy_measured_gbs": copy_gbs, "frac_of_copy": round(dk["achieved_gbs"] / copy_gbs, 4)}

    batching = None
    if want_batch:
        batching = batching_record(args, P, cpu4)

    value = prob.st_dofs / (r0["ms_per_step"] * 1e-3)
    out = {
        "metric": "space-time DoFs/s to rel. residual 1e-8 (FP32+refine vs FP64); % HBM peak",
        "value": value,
        "unit": "space-time DoFs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r0["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if primary == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "n": prob.n, "N": prob.N, "seed": args.seed, "st_dofs": prob.st_dofs,
                   "tol": args.tol, "mode": "fp32_refine" if primary == "fp32" else "fp64",
                   "inner": inner},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "modes": {m: {"value": prob.st_dofs / (res[m]["ms_per_step"] * 1e-3), "ms_per_step": res[m]["ms_per_step"],
                      "median_solve_ms_device": statistics.median(res[m]["solve_ms_device"]),
                      "solve_ms_device": [round(x, 2) for x in res[m]["solve_ms_device"]],
                      "outer_iters": res[m]["outer_iters"], "rel_residual": res[m]["rel_residual"],
                      **({"static_start_iters": res[m]["init_iters"]} if args.paper_stop else {}),
                      "tuned": res[m]["tuned"]} for m in modes},
        "errors": errors,
        "kernels": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kern.items()},
        "kernels_per_kernel_pass": {k: {kk: (round(vv, 5) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                                    for k, v in kern_pass.items()},
        "kernel_ms_all": {k: round(v, 3) for k, v in r0["kernel_ms_pass"].items()},
        "timing_note": "the timed solves bracket only the two kernel classes of `kernels` with HIP events; "
                       "`kernels_per_kernel_pass` and `kernel_ms_all` come from one untimed solve before "
                       "them with every launch bracketed",
        "batching": batching,
        "paper_context": PAPER_CONTEXT,
    }
    if args.max_outer < 2000:
        out["profiling_run"] = f"outer steps capped at {args.max_outer}: not a metric measurement"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
