#!/usr/bin/env python3
"""Write the oracle's periodic solution of a seeded problem at a size where only the
period-sweep solver (oracle B) is feasible, for the full-size parity tests.

Calls only the oracle (``oracle.periodic``: residual of eq. (disc1), fixed-point iteration of
eqs. (iter1)-(iter2) with an exact inner solve by sparse LU of M/tau + Khat and period sweeps)
and the seeded problem descriptions of ``workloads``. Nothing here comes from the GPU path.

Stored (npz, float64):
  slices       U on the time slices ``slice_idx`` (full grid, zero boundary), on every
               ``stride``-th node in each direction (row-major over the sampled grid)
  slice_idx    which slices (slice j holds u^{j+1})
  stride       node sampling stride
  u_sq_sum     sum of U^2 over all nodes and slices
  u_sum        sum of U over all nodes and slices
  rel_hist     relative residual ||F - A(U^k)|| / ||F|| at every step
  khat_steps   ||U^{k+1} - U^k||_Khat of every step
  meta         JSON: problem, tolerance, steps, host time, host threads, command

Usage:
  python tests/golden/make_oracle_solutions.py --n 256 --N 256 --seed 0 --tol 1e-12 \
      --out tests/golden/oracle_c2_seed0_n256_N256.npz
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import fem, periodic as pp  # noqa: E402


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, required=True)
    ap.add_argument("--N", type=int, required=True)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tol", type=float, default=1e-12)
    ap.add_argument("--stride", type=int, default=1)
    ap.add_argument("--slices", default="0,q,h,l", help="slice indices; q = N/4-1, h = N/2-1, l = N-1")
    ap.add_argument("--out", required=True)
    ap.add_argument("--checkpoint", default="", help="file to keep the iterate in every 10 steps")
    args = ap.parse_args()

    # the metric workload's materials and source (seeded J0 and iron jitter) on this grid
    p = W.with_size(W.config3(args.seed), args.n, args.N)
    t_start = time.perf_counter()
    d = fem.discretise(p)
    F = pp.load_series(d)
    lin = pp.PeriodSweepLU(d)
    U0 = None
    if args.checkpoint and os.path.exists(args.checkpoint):
        U0 = np.load(args.checkpoint)
        print(f"resuming from {args.checkpoint}", flush=True)

    def progress(k, rel, U):
        print(f"step {k}: rel {rel:.3e} ({time.perf_counter() - t_start:.0f} s)", flush=True)
        if args.checkpoint and k > 0 and k % 10 == 0:
            np.save(args.checkpoint, U)

    r = pp.fixed_point(d, tol=args.tol, max_iter=5000, F=F, lin=lin, U0=U0, callback=progress)
    wall = time.perf_counter() - t_start
    if not r.converged:
        raise SystemExit(f"oracle did not reach tol {args.tol}: rel {r.rel[-1]}")
    U, rels, steps, k, rel = r.U, r.rel, r.khat_step, r.iters, r.rel[-1]

    N, n = args.N, args.n
    idx = []
    for t in args.slices.split(","):
        idx.append({"q": N // 4 - 1, "h": N // 2 - 1, "l": N - 1}.get(t, None) if t in "qhl" else int(t))
    full = pp.to_full(d, U)                                    # (N, n+1, n+1)
    s = args.stride
    sl = np.stack([full[j, ::s, ::s] for j in idx])
    meta = {
        "problem": {"n": n, "N": N, "seed": args.seed, "J0": p.J0, "nu_rect": p.nu_rect.as_tuple(),
                    "workload": "metric materials and source (seeded J0, iron jitter) on this grid"},
        "solver": "oracle B: fixed point (eqs. (iter1)-(iter2)), Khat = nu_max S, exact inner solve by "
                  "sparse LU of M/tau + Khat with period sweeps",
        "tol": args.tol, "steps": k, "rel_final": rel, "host_seconds": wall,
        "host_threads": 1, "host": platform.processor() or platform.machine(), "cpu_count": os.cpu_count(),
        "command": " ".join(["python", "tests/golden/make_oracle_solutions.py"] + sys.argv[1:]),
    }
    np.savez_compressed(args.out, slices=sl, slice_idx=np.array(idx), stride=np.array(s),
                        u_sq_sum=np.array(float(np.sum(U * U))), u_sum=np.array(float(np.sum(U))),
                        rel_hist=np.array(rels), khat_steps=np.array(steps), meta=np.array(json.dumps(meta)))
    print(json.dumps(meta), flush=True)


if __name__ == "__main__":
    main()
