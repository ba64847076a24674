"""Many problems of uneven size on one GPU.

Problems that share the grid, the period, the conductivity and nu_max are stacked into
batch plans (pt_plan_create_batch; a power of two instances each, so a group of 5 becomes
batches of 4 and 1). All batch plans are then solved by the native work-list runner
pt_solve_many: a few host threads, each owning one HIP stream, take the next plan in
order of decreasing cost (longest-processing-time-first), so the small plans fill the
device while the large ones run. With graph=True each plan replays its outer steps from
a captured HIP graph.

Only argument marshalling happens here; the solves run in the HIP library.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

from . import _lib as L
from . import BatchPlan, PTError, SolveStats, _StatsBuf


def share_key(p) -> Tuple:
    """Problems with equal keys can share one batch plan (same M, Khat, hierarchy)."""
    r = p.sigma_rect
    rect = tuple(r.as_tuple()) if hasattr(r, "as_tuple") else tuple(r)
    return (int(p.n), int(p.N), float(p.T), float(p.sigma_in), rect, float(p.nu_max))


def pow2_split(count: int, max_batch: int) -> List[int]:
    """Sizes of the batches a group of `count` is cut into: powers of two, largest first,
    none above max_batch (itself a power of two)."""
    if max_batch < 1 or max_batch & (max_batch - 1):
        raise ValueError("max_batch must be a power of two")
    out = []
    while count > 0:
        b = min(max_batch, 1 << (count.bit_length() - 1))
        out.append(b)
        count -= b
    return out


def plan_groups(problems: Sequence, max_batch: int = 64, max_slots: int = 65536) -> List[List[int]]:
    """Indices of the problems of each batch plan, in order of decreasing cost (nodes x N
    per outer step). Within a group the input order is kept."""
    groups: Dict[Tuple, List[int]] = {}
    for i, p in enumerate(problems):
        groups.setdefault(share_key(p), []).append(i)
    batches = []
    for key, idx in groups.items():
        N = key[1]
        cap = max_batch
        while cap > 1 and cap * (N // 2) > max_slots:
            cap //= 2
        pos = 0
        for b in pow2_split(len(idx), cap):
            batches.append(idx[pos:pos + b])
            pos += b

    def cost(ix):
        p = problems[ix[0]]
        return (p.n + 1) ** 2 * p.N * len(ix)

    batches.sort(key=cost, reverse=True)
    return batches


@dataclass
class ManyResult:
    U: List            # per problem: device tensor [N, n+1, n+1] (a view into its batch's field)
    stats: List[SolveStats]
    status: int
    batches: List[List[int]]


class ManySolver:
    """Plans, workspaces and output fields for a fixed list of problems; solve() may be
    called repeatedly (the workspaces and captured graphs are reused)."""

    def __init__(self, problems: Sequence, *, precision="fp64", tol=1e-8, max_outer=1000, check_every=1,
                 graph=True, nstreams=4, max_batch=64, tuning: Optional[Dict] = None, **opts):
        import torch
        self.problems = list(problems)
        self.lib = L.load()
        self.batches = plan_groups(self.problems, max_batch=max_batch)
        self.plans: List[BatchPlan] = []
        for ix in self.batches:
            kw = dict(opts)
            if tuning is not None:
                kw.update(tuning.get(tune_key(self.problems[ix[0]], len(ix), precision), {}))
            self.plans.append(BatchPlan([self.problems[i] for i in ix], precision=precision, tol=tol,
                                        max_outer=max_outer, check_every=check_every, graph=graph, **kw))
        self.fields = [pl.new_time_field() for pl in self.plans]
        self.ws = [pl.workspace() for pl in self.plans]
        self.streams = [torch.cuda.Stream() for _ in range(max(1, int(nstreams)))]
        torch.cuda.synchronize()
        self.total_st_dofs = sum(p.st_dofs for p in self.problems)

    def solve(self, history_cap: int = 0, raise_on_error: bool = True) -> ManyResult:
        import torch
        n = len(self.plans)
        plans = (C.c_void_p * n)(*[pl._h.value for pl in self.plans])
        wsp = (C.c_void_p * n)(*[w[0].value for w in self.ws])
        wsb = (C.c_size_t * n)(*[w[1].value for w in self.ws])
        us = (C.c_void_p * n)(*[f.data_ptr() for f in self.fields])
        bufs, arrays = [], []
        for pl in self.plans:
            bb = [_StatsBuf(max(1, history_cap)) for _ in range(pl.count)]
            sa = (L.Stats * pl.count)()
            for b, s in zip(bb, sa):
                b.fill(s)
            bufs.append(bb)
            arrays.append(sa)
        sp = (C.POINTER(L.Stats) * n)(*[C.cast(a, C.POINTER(L.Stats)) for a in arrays])
        status = (C.c_int32 * n)()
        streams = (C.c_void_p * len(self.streams))(*[s.cuda_stream for s in self.streams])
        torch.cuda.synchronize()
        st = self.lib.pt_solve_many(n, plans, wsp, wsb, us, sp, status, streams, len(self.streams))
        if raise_on_error and st != L.PT_OK:
            raise PTError(st, "pt_solve_many")
        U = [None] * len(self.problems)
        stats = [None] * len(self.problems)
        for k, ix in enumerate(self.batches):
            for b, i in enumerate(ix):
                U[i] = self.fields[k][b]
                stats[i] = bufs[k][b].result(self.lib, status[k], arrays[k][b])
        return ManyResult(U=U, stats=stats, status=st, batches=self.batches)

    def close(self):
        for pl in self.plans:
            pl.close()


def tune_key(p, count, precision) -> str:
    """Key of a tuning table entry: grid, period, batch size and precision."""
    return f"n{p.n}_N{p.N}_B{count}_{precision}"
