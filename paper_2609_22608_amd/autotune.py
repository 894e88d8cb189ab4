"""Launch-mapping autotuner for the planner's kernels.

The kNN scan splits the tree into node chunks so that enough wavefronts run
to fill the 256 compute units; how many, and how small a chunk may get, is a
trade between occupancy and the cost of merging partial lists, and the best
point moves with the tree size, the batch size and (for a batched round) the
number of problems.  The edge search has two exact modes (plain ascending
scan and endpoint-screened scan) whose ratio moves with the workload's
feasibility mix, and the screened modes three exact forms (one kernel; a
triage kernel before the search of the open edges; the same with the open
edges sorted longest-first) whose ratio moves with the number of edges.  This module times the candidates on the device with HIP
events on the launching stream, keeps the fastest, and caches the choice
per shape in a JSON file so later runs skip the search.

Every candidate computes the same result (the mapping changes only the
order of independent work; the merge is exact), so tuning is safe at any
time; the tests check that results do not depend on the tuning.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass

import torch

from . import fn

# (target wavefronts, minimum chunk of nodes per wavefront)
KNN_CANDIDATES = ((1024, 256), (2048, 256), (2048, 512), (3072, 1024), (4096, 512),
                  (4096, 1024), (6144, 1024), (8192, 512), (8192, 1024), (16384, 1024))
# the matrix-core form runs 16 queries per wavefront (and at most 4096
# wavefronts): fewer wavefronts for the same split
KNN_CANDIDATES_MFMA = ((512, 512), (1024, 512), (2048, 512), (2048, 1024), (4096, 512),
                       (4096, 1024))
# kNN scan forms: 1 = VALU keys, per-wavefront node loads; 2 = VALU keys,
# workgroup node tiles in LDS; 3 = matrix-core keys
KNN_FORMS = (1, 2, 3)
# edge forms of the screened searches: 1 = one kernel; 2 = triage, then the
# search of the open edges; 3 = the same, open edges longest-first
EDGE_FORMS = (1, 2, 3)


def knn_grid(candidates=None):
    """(target wavefronts, minimum chunk, form) triples the tuner times."""
    for form in KNN_FORMS:
        cl = candidates if candidates is not None else (
            KNN_CANDIDATES_MFMA if form == 3 else KNN_CANDIDATES)
        for tw, mc in cl:
            yield tw, mc, form


@dataclass
class Choice:
    knn_target_waves: int
    knn_min_chunk: int
    mode: int
    ms: float
    knn_form: int = 0
    edge_form: int = 0  # search form of edge_time_batch (tune_edge); 0 = not tuned

    def as_dict(self):
        return dict(knn_target_waves=self.knn_target_waves, knn_min_chunk=self.knn_min_chunk,
                    knn_form=self.knn_form, mode=self.mode, ms=self.ms, edge_form=self.edge_form)


class Cache:
    """JSON cache {key: choice}; key names the shape, the device and the
    library version so a rebuilt library or another card retunes."""

    def __init__(self, path: str | None):
        self.path = path
        self.data = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.data = json.load(f)

    def get(self, key):
        d = self.data.get(key)
        return None if d is None else Choice(**d)

    def put(self, key, ch: Choice):
        self.data[key] = ch.as_dict()
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.data, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def _device_tag():
    # architecture, compute units and library version (the marketing name is
    # not reported under every tool, e.g. a profiler)
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{getattr(p, 'gcnArchName', '')}|cu{p.multi_processor_count}|{fn.version()}"


def _time(run, reps, setup=None):
    """Median device time of run() over reps calls (events on the current
    stream); setup() runs before each call, outside the timed events."""
    s = torch.cuda.current_stream()
    ts = []
    for r in range(reps + 1):
        if setup:
            setup()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        run()
        e1.record(s)
        torch.cuda.synchronize()
        if r:  # the first call warms up
            ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def tune_knn(ctx: fn.Context, tree, ld, n_nodes, cand, k, reps=5, cache: Cache | None = None,
             candidates=None):
    """Fastest kNN mapping for one (tree, batch, k); leaves it set on ctx."""
    B = cand.shape[0]
    key = f"knn|n{n_nodes}|B{B}|k{k}|{_device_tag()}"
    hit = cache.get(key) if cache else None
    if hit is not None:
        ctx.set_tuning(hit.knn_target_waves, hit.knn_min_chunk, hit.knn_form)
        return hit, {}
    idx = torch.empty((B, k), dtype=torch.int32, device=cand.device)
    times = {}
    for tw, mc, form in knn_grid(candidates):
        ctx.set_tuning(tw, mc, form)
        times[(tw, mc, form)] = _time(lambda: ctx.plan_knn(tree, ld, n_nodes, cand, k,
                                                           out_idx=idx, want_d2=False), reps)
    (tw, mc, form), ms = min(times.items(), key=lambda kv: kv[1])
    ch = Choice(tw, mc, -1, ms, form)
    ctx.set_tuning(tw, mc, form)
    if cache:
        cache.put(key, ch)
    return ch, {f"{a}/{b}/{f}": v for (a, b, f), v in times.items()}


def tune_edge(ctx: fn.Context, tree, ld, n_nodes, cand, nbr, grid, samples, obs=None,
              mode=fn.SEARCH_SCREEN, reps=5, cache: Cache | None = None, win_lo=None, win_half=4):
    """Fastest edge form of edge_time_batch for one shape and search mode: 1
    (one kernel, a wavefront per edge), 2 (the triage of every edge, then the
    search of the open ones) or 3 (as 2, the open edges in descending order
    of their open-slot count); all give identical results.  Leaves it set on
    ctx (the kNN mapping is kept)."""
    B, k = nbr.shape
    n_obs = 0 if obs is None else int(obs.shape[0])
    key = (f"edge|n{n_nodes}|B{B}|k{k}|nt{grid.shape[0]}|S{samples}|o{n_obs}|m{mode}|"
           f"{_device_tag()}")
    hit = cache.get(key) if cache else None
    if hit is not None:
        ctx.set_tuning(edge_form=hit.edge_form)
        return hit, {}
    E = B * k
    d = cand.device
    out = dict(j=torch.empty(E, dtype=torch.int16, device=d),
               status=torch.empty(E, dtype=torch.int16, device=d),
               margin=torch.empty(E, dtype=torch.float32, device=d), rho=None, work=None,
               screened=None)
    kw = dict(win_lo=win_lo, win_half=win_half) if mode == fn.SEARCH_WINDOW else {}
    times = {}
    for form in EDGE_FORMS:
        ctx.set_tuning(edge_form=form)
        times[form] = _time(lambda: ctx.edge_time_batch(tree, ld, n_nodes, cand, nbr, grid,
                                                        samples, obs, mode=mode, out=out, **kw),
                            reps)
    form, ms = min(times.items(), key=lambda kv: kv[1])
    ch = Choice(0, 0, mode, ms, 0, form)
    ctx.set_tuning(edge_form=form)
    if cache:
        cache.put(key, ch)
    return ch, {f"edge_form {f}": v for f, v in times.items()}


def tune_batch(bt: fn.Batch, reps=3, cache: Cache | None = None, candidates=None,
               modes=(fn.SEARCH_PLAIN, fn.SEARCH_SCREEN)):
    """Fastest (kNN mapping, search mode, edge form) for a prepared batched
    round: every kNN mapping in each mode with the one-kernel search, then
    the ordered two-phase search (edge form 3) with the screened mode's best
    mapping.

    Each timing restores the initial trees first, so every candidate times
    the same round.  Leaves the winner prepared on ``bt``."""
    sig = ";".join(f"{P['n0']}x{P['B']}o{P['n_obs']}" for P in bt.problems)
    key = f"batch|{sig}|k{bt.k}|nt{bt.grid.shape[0]}|S{bt.samples}|{_device_tag()}"
    hit = cache.get(key) if cache else None
    if hit is not None:
        bt.ctx.set_tuning(hit.knn_target_waves, hit.knn_min_chunk, hit.knn_form,
                          edge_form=hit.edge_form)
        bt.mode = hit.mode
        bt.prepare()
        return hit, {}

    def run(tw, mc, mode, form, ef):
        bt.ctx.set_tuning(tw, mc, form, edge_form=ef)
        bt.mode = mode
        bt.prepare()
        times[(tw, mc, mode, form, ef)] = _time(bt.launch, reps, setup=bt.reset_trees)

    times = {}
    for mode in modes:
        for tw, mc, form in knn_grid(candidates):
            run(tw, mc, mode, form, 1)
    screened = {kk: v for kk, v in times.items() if kk[2] != fn.SEARCH_PLAIN}
    if screened:
        tw, mc, mode, form, _ = min(screened.items(), key=lambda kv: kv[1])[0]
        run(tw, mc, mode, form, 3)
    (tw, mc, mode, form, ef), ms = min(times.items(), key=lambda kv: kv[1])
    ch = Choice(tw, mc, mode, ms, form, ef)
    bt.ctx.set_tuning(tw, mc, form, edge_form=ef)
    bt.mode = mode
    bt.prepare()
    bt.reset_trees()
    if cache:
        cache.put(key, ch)
    return ch, {f"{a}/{b}/{'plain' if m == fn.SEARCH_PLAIN else 'screen'}/{f}/e{e}": v
                for (a, b, m, f, e), v in times.items()}
