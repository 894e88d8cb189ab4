"""Benchmark: validated edges/s of the edge timing and validation step.

One step = one pass of the hot path over one batch: brute-force kNN parents
for every candidate, then minimum-time search + post-checks of every
(candidate, parent) edge.  Inputs are generated once, copied to HBM, and
stay resident; the timed region is bracketed by device synchronisation and
HIP events on the stream the library launches on.

Prints one JSON line (see the project's benchmark contract).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "validated edges/s (7-DOF, 64 T x 32 samples); MLP-window vs exact speedup"
PEAK_FP32 = 157.3e12  # MI355X FP32 vector peak (packed), FLOP/s

# Algorithmic FLOP per unit in the kernels' formulation (FMA = 2, each
# transcendental or reciprocal = 1); the design notes derive every count.
# One evaluation point of Eq. (4)-(7): cubic 169, sin/cos 21, RNEA 1,005,
# armature 14, friction 56, ratios and power 30.
F_EVAL = 1295
# One slot screened from the endpoint models and the edge's coefficients:
# the reciprocal of T and 1/T^2 (2), both endpoint torques by two FMAs per
# joint (56), ratios and power (59).
F_SCREEN = 117
# The coefficients of one screened edge: 28 products of 7 terms with their
# operands (6 dq: 3 per term; 6 qd0 + 2 d2 or 6 qd0 + 4 d2: 5 per term).
F_SCREEN_EDGE = 784
# One endpoint model (per state): 8 lanes x (sin/cos 21 + rigid RNEA 1,005)
# + armature 7 + friction 56.
F_MODEL = 8271
# Post-checks of one edge at its result: velocity taper and position
# extrema, 140 per joint; clearance per sample: cubic position 98, sin/cos
# 21, the frame chain 252, per sphere 19 + 13 per obstacle.
F_JOINTS = 980


# One row of surrogate inference: 2 x (28 x 256 + 2 x 256 x 256 + 256 x 2).
F_MLP_ROW = 277504
# One (query, node) pair of the kNN scan: 14 differences and 14 squares
# summed (FMA = 2).
F_KNN_PAIR = 42
PEAK_BF16 = 2500e12  # MI355X dense BF16 matrix peak, FLOP/s
# Initial (cosine-decayed) learning rate of the surrogate's training: from
# 1e-3 to 1e-2 at minibatch 4,096 the held-out window misses fall to a
# plateau from 3e-3 on (16.4% -> 13.4% of feasible edges).
LR_SURROGATE = 3e-3
# One controller step: Eq. (9) and the taper bounds 7 x 20, sin/cos 21,
# rigid-body recursion 1,005, armature 14, friction 56, clips and power 7 x 8.
F_CONTROL = 1252
# HBM bytes of one controller step: q, qd, the previous torque, the
# rendezvous state (7 floats each) and the horizon in; torque and
# acceleration (7 floats each) and a 2-byte status out.
B_CONTROL = 4 * (5 * 7 + 1) + 4 * 2 * 7 + 2
PEAK_HBM = 8.0e12  # MI355X HBM3E, bytes/s


def f_clear(S, n_obs, n_sph):
    """Clearance of one edge (evaluated only when its limit checks pass)."""
    return S * (371 + n_sph * (19 + 13 * n_obs)) if n_obs > 0 else 0


WORKLOADS = {
    "iteration": "one planning iteration: 16,384-node tree, 4,096 candidates (half goal), k=8, "
                 "64 T x 32 samples, 5 obstacles, 7-DOF arm",
    "stress": "stress: 262,144-node tree, 65,536 candidates (30% goal), k=16, 128 T over "
              "0.01-1.2 s x 64 samples, 20 obstacles, 7-DOF arm",
}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--seed", type=int, default=101)
    p.add_argument("--modes", default="plain,screen,window")
    p.add_argument("--surrogate", default=None, help="checkpoint to load instead of training")
    p.add_argument("--save-surrogate", default=None, help="write the trained network here")
    p.add_argument("--train-batches", type=int, default=306,
                   help="one-iteration batches labelled for the surrogate (306 x 32,768 = "
                        "10.0 M edges)")
    p.add_argument("--train-epochs", type=int, default=20)
    p.add_argument("--half", type=int, default=4)
    p.add_argument("--workload", default="iteration", choices=sorted(WORKLOADS))
    p.add_argument("--cpu-sample", type=int, default=None,
                   help="candidates in the CPU oracle sample (default: all for the one-iteration "
                        "workload, 1,024 for the stress workload)")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--profile", action="store_true", help="few steps, no CPU leg (under rocprofv3)")
    p.add_argument("--batch-problems", type=int, default=32,
                   help="problems in the batched-round form (0 skips it)")
    p.add_argument("--no-tune", action="store_true", help="default launch mappings (no autotuning)")
    p.add_argument("--tune-cache", default=None,
                   help="JSON cache of tuned launch mappings (read and written)")
    p.add_argument("--edge-form", type=int, default=0, choices=(0, 1, 2, 3),
                   help="screened searches: 0 library default, 1 one kernel, 2 triage + search "
                        "of the open edges, 3 the same longest-first (fn_tuning.edge_form)")
    return p.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_2609_22608_amd import fn, workload as W

    if args.profile:
        args.steps, args.warmup, args.no_cpu = min(args.steps, 5), 1, True
    if args.workload != "iteration":
        args.batch_problems = 0
    sh = W.CONFIGS[args.workload]
    wl = W.make_workload(sh, seed=args.seed)
    E = sh.batch * sh.k
    ctx = fn.Context(wl["arm"], sh.n_nodes, sh.batch, sh.k)
    tree, ld, n = fn.tree_soa(wl["tree_x"])
    cand = fn.dev(wl["cand"]["x"])
    grid = fn.dev(wl["grid"])
    obs = fn.dev(wl["obs"])
    idx = torch.empty((sh.batch, sh.k), dtype=torch.int32, device="cuda")
    out = dict(j=torch.empty(E, dtype=torch.int16, device="cuda"),
               status=torch.empty(E, dtype=torch.int16, device="cuda"),
               margin=torch.empty(E, dtype=torch.float32, device="cuda"),
               rho=None, work=torch.empty(E, dtype=torch.int32, device="cuda"),
               screened=torch.empty(E, dtype=torch.int16, device="cuda"))
    stream = torch.cuda.current_stream()
    if args.edge_form:
        ctx.set_tuning(edge_form=args.edge_form)
    knn_tuning = None
    if not args.no_tune:
        # launch mapping of the kNN scan for this shape (outside the timed region)
        from paper_2609_22608_amd import autotune

        ch, _ = autotune.tune_knn(ctx, tree, ld, n, cand, sh.k, reps=3,
                                  cache=autotune.Cache(args.tune_cache))
        knn_tuning = ch.as_dict()
    modes = {"plain": fn.SEARCH_PLAIN, "screen": fn.SEARCH_SCREEN, "window": fn.SEARCH_WINDOW}
    wanted = args.modes.split(",")
    edge_tuning = None
    if not args.no_tune and not args.edge_form and ("screen" in wanted or "window" in wanted):
        # the screened searches' form (one kernel, or triage then search) for
        # this shape, timed on the screened search (outside the timed region)
        from paper_2609_22608_amd import autotune

        ctx.plan_knn(tree, ld, n, cand, sh.k, out_idx=idx, want_d2=False)
        ch, _ = autotune.tune_edge(ctx, tree, ld, n, cand, idx, grid, sh.samples, obs,
                                   mode=fn.SEARCH_SCREEN, reps=3,
                                   cache=autotune.Cache(args.tune_cache))
        edge_tuning = {"edge_form": ch.edge_form, "ms": ch.ms}
    # the screened searches' form, always set explicitly so that the line
    # names the kernels it timed (untuned: the ordered two-phase form)
    edge_form = args.edge_form or (edge_tuning["edge_form"] if edge_tuning else 3)
    ctx.set_tuning(edge_form=edge_form)
    surrogate_info = None
    net = None
    if "window" in wanted:
        # trained on one-iteration-shaped edges whatever the workload
        net, surrogate_info = surrogate(args, ctx, wl["arm"], W.CONFIGS["iteration"], fn, W,
                                        torch)
        if args.save_surrogate:
            net.save(args.save_surrogate)
    win = torch.empty(E, dtype=torch.int16, device="cuda")
    forms = {}
    for name in wanted:
        mode = modes[name]

        def step(ev=None):
            # ev: events after the kNN, before the search and at the end (the
            # breakdown pass only; the timed steps carry no events of their own)
            ctx.plan_knn(tree, ld, n, cand, sh.k, out_idx=idx, want_d2=False)
            if ev:
                ev[0].record(stream)
            if mode == fn.SEARCH_WINDOW:
                # edge rows gathered inside the inference kernel
                net.window(tree, ld, n, cand, idx, grid, half=args.half, win_lo=win)
                if ev:
                    ev[2].record(stream)
                ctx.edge_time_batch(tree, ld, n, cand, idx, grid, sh.samples, obs, mode=mode,
                                    win_lo=win, win_half=args.half, out=out)
            else:
                if ev:
                    ev[2].record(stream)
                ctx.edge_time_batch(tree, ld, n, cand, idx, grid, sh.samples, obs, mode=mode,
                                    out=out)
            if ev:
                ev[1].record(stream)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        # timed steps; the library's own event pair brackets the search kernel
        ctx.kernel_timing(True)
        ctx.kernel_times()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        t0.record(stream)
        for _ in range(args.steps):
            step()
        t1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        k_ms = ctx.kernel_times()
        ctx.kernel_timing(False)
        ms = t0.elapsed_time(t1) / args.steps
        # breakdown (untimed): a few more steps with events inside
        edge_ms = []
        for _ in range(min(args.steps, 5)):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            step(ev)
            edge_ms.append(ev)
        torch.cuda.synchronize()
        e_ms = float(np.mean([a[2].elapsed_time(a[1]) for a in edge_ms]))
        kern_ms = float(np.mean(k_ms))
        work = int(out["work"].sum().item())
        scr = int(out["screened"].sum().item())
        st = out["status"].cpu().numpy().astype(np.uint16)
        jj = out["j"].cpu().numpy()
        post = (jj >= 0) & ((st & fn.S_RECHECK64) == 0)
        n_post = int(post.sum())
        # the clearance runs only where the limit checks passed
        n_clear = int((post & ((st & (fn.S_VEL | fn.S_POS)) == 0)).sum())
        n_sph = len(wl["arm"]["sph"])
        n_scr_edges = int((out["screened"] > 0).sum().item())
        flop = (work * F_EVAL + scr * F_SCREEN + n_scr_edges * F_SCREEN_EDGE + n_post * F_JOINTS
                + n_clear * f_clear(sh.samples, sh.n_obs, n_sph))
        f = dict(edges_per_s=E / (ms * 1e-3), ms_per_step=ms, edge_search_ms=e_ms,
                 search_span_ms=kern_ms, evaluations=work, screened_slots=scr,
                 screened_edges=n_scr_edges,
                 post_checked=n_post, clearance_checked=n_clear, kernel_gflop=flop / 1e9,
                 wall_s=wall,
                 fp32_tflops=flop / (kern_ms * 1e-3) / 1e12,
                 model_states=(E + sh.batch) if mode != fn.SEARCH_PLAIN else 0,
                 edge_form=edge_form if mode != fn.SEARCH_PLAIN else 1,
                 recheck64=int(((st & fn.S_RECHECK64) > 0).sum()))
        if mode == fn.SEARCH_WINDOW:
            pre = float(np.mean([a[0].elapsed_time(a[2]) for a in edge_ms]))
            f.update(features_infer_ms=pre)
            f.update(window_stats(args, ctx, net, tree, ld, n, cand, idx, grid, sh, obs, out, fn,
                                  torch))
        f["roofline"] = {"bound": "alu", "achieved": f["fp32_tflops"], "peak": PEAK_FP32 / 1e12,
                         "unit": "TFLOP/s", "frac": f["fp32_tflops"] * 1e12 / PEAK_FP32}
        forms[name] = f
    best = min(forms, key=lambda k: forms[k]["ms_per_step"])
    speed = {}
    if "window" in forms and "plain" in forms:
        speed["window_vs_plain"] = forms["window"]["edges_per_s"] / forms["plain"]["edges_per_s"]
    if "window" in forms and "screen" in forms:
        speed["window_vs_screen"] = forms["window"]["edges_per_s"] / forms["screen"]["edges_per_s"]
    bf = forms[best]
    res = {
        "metric": METRIC,
        "value": bf["edges_per_s"],
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": bf["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "search": best, "edges": E,
                   "seed": args.seed, "knn_tuning": knn_tuning, "edge_tuning": edge_tuning},
        "diagnostics": diagnostics(out, sh, fn),  # decisions are the same in every form
        "forms": forms,
        "speedup": speed,
        "surrogate": surrogate_info,
        "roofline": {"bound": "alu", "kernel": EDGE_SPAN_KERNELS[bf["edge_form"]],
                     "form": best, "edge_form": bf["edge_form"], "achieved": bf["fp32_tflops"],
                     "peak": PEAK_FP32 / 1e12,
                     "unit": "TFLOP/s", "frac": bf["fp32_tflops"] * 1e12 / PEAK_FP32,
                     "traffic": traffic_bytes("edge_search", f"{best}/{bf['edge_form']}"),
                     "kernel_ms": bf["search_span_ms"],
                     "flop_per_launch": bf["kernel_gflop"] * 1e9,
                     "flop_model": {"eval": F_EVAL, "screened_slot": F_SCREEN,
                                    "screened_edge": F_SCREEN_EDGE,
                                    "post_checked_edge": F_JOINTS,
                                    "clearance_edge": f_clear(sh.samples, sh.n_obs,
                                                              len(wl["arm"]["sph"])),
                                    "model_state": F_MODEL},
                     "units": {"evaluations": bf["evaluations"],
                               "screened_slots": bf["screened_slots"],
                               "screened_edges": bf["screened_edges"],
                               "post_checked_edges": bf["post_checked"],
                               "clearance_checked_edges": bf["clearance_checked"]}},
    }
    res["roofline_other"] = other_rooflines(args, ctx, net, tree, ld, n, cand, idx, grid, sh,
                                            win, fn, torch)
    res["refine"] = refine_stats(args, ctx, wl, tree, ld, n, cand, idx, grid, sh, obs, out, fn,
                                 torch)
    res["controller"] = controller_stats(args, ctx, wl, fn, W, torch)
    if args.batch_problems > 0:
        res["batched_round"] = batched_round(args, fn, W, torch)
    res["planning_cycle"] = planning_cycle(args, fn, W, torch)
    if args.profile:
        # a plain device copy of known size (256 MiB) for calibrating the
        # HBM traffic counters
        a = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
    if not args.no_cpu:
        n_cpu = args.cpu_sample or (sh.batch if args.workload == "iteration" else 1024)
        res["cpu_baseline"] = cpu_baseline(wl, min(n_cpu, sh.batch))
    print(json.dumps(res), flush=True)
    ctx.close()


def window_stats(args, ctx, net, tree, ld, n, cand, idx, grid, sh, obs, out, fn, torch):
    """Window outcome of the timed window runs (out holds the last one) and
    what the network gains: the same exact search with the window placed at
    the first slot the endpoint screen leaves open (no network), and the
    network's raw window before that lower bound is applied."""
    jj = out["j"].cpu().numpy().astype(np.int64)
    st = out["status"].cpu().numpy().astype(np.uint16)
    feas = jj >= 0
    miss = (st & fn.S_WIN_MISS) > 0
    y, w_net = net.window(tree, ld, n, cand, idx, grid, half=args.half, want_out=True)
    E = jj.size
    base = ctx.edge_time_batch(tree, ld, n, cand, idx, grid, sh.samples, obs,
                               mode=fn.SEARCH_WINDOW,
                               win_lo=torch.zeros(E, dtype=torch.int16, device="cuda"),
                               win_half=args.half, want_rho=False)
    torch.cuda.synchronize()
    jb = base["j"].cpu().numpy().astype(np.int64)
    sb = base["status"].cpu().numpy().astype(np.uint16)
    assert np.array_equal(jb, jj), "window placement changed a result"
    miss_base = (sb & fn.S_WIN_MISS) > 0
    lo = w_net.cpu().numpy().astype(np.int64)
    raw_hit = feas & (jj >= lo) & (jj <= lo + 2 * args.half)
    lg = np.log(grid.cpu().numpy().astype(np.float64))
    yy = y.cpu().numpy().astype(np.float64)
    lt_hat = 0.5 * (lg[0] + lg[-1]) + 0.5 * (lg[-1] - lg[0]) * yy[:, 0]
    err = np.abs(lt_hat[feas] - lg[jj[feas]])
    nf = max(1, int(feas.sum()))
    return dict(
        miss_rate_feasible=float(miss[feas].sum() / nf),
        miss_rate_all=float(miss.mean()),
        below_window_rate=float(((st & fn.S_WIN_BELOW) > 0).mean()),
        miss_rate_feasible_raw_network_window=float(1.0 - raw_hit.sum() / nf),
        miss_rate_feasible_without_network=float(miss_base[feas].sum() / nf),
        logT_abs_err_median=float(np.median(err)) if err.size else None,
        logT_abs_err_p90=float(np.quantile(err, 0.9)) if err.size else None,
        bin_width_logT=float((lg[-1] - lg[0]) / (len(lg) - 1)),
        predicted_infeasible_frac=float((yy[:, 1] < 0.0).mean()))


def other_rooflines(args, ctx, net, tree, ld, n, cand, idx, grid, sh, win, fn, torch):
    """Rooflines of the kNN call (scan + merge; FP32 VALU) and of the fused
    surrogate inference kernel with its edge-row gather (surrogate_window;
    BF16 matrix cores), each timed alone with HIP events on the stream the
    library launches on."""
    stream = torch.cuda.current_stream()

    def time_it(call, reps):
        for _ in range(2):
            call()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            call()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    reps = max(5, args.steps)
    res = {}
    # the scan form the tuner picked (0: chosen by tree size, which is the
    # per-wavefront form 1 at or below 65,536 nodes and matrix cores above)
    ctx_knn_form = getattr(ctx, "tuned_knn_form", 0) or (3 if n > 65536 else 1)
    ms = time_it(lambda: ctx.plan_knn(tree, ld, n, cand, sh.k, out_idx=idx, want_d2=False), reps)
    flop = float(sh.batch) * n * F_KNN_PAIR
    res["plan_knn"] = {"bound": "alu", "achieved": flop / (ms * 1e-3) / 1e12,
                       "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                       "frac": flop / (ms * 1e-3) / PEAK_FP32, "ms": ms,
                       "pairs": sh.batch * n, "flop_per_pair": F_KNN_PAIR,
                       "knn_form": ctx_knn_form,
                       "traffic": traffic_bytes("knn_scan_mfma" if ctx_knn_form == 3 else "knn_scan",
                                                str(ctx_knn_form))}
    if net is not None:
        E = idx.numel()
        ms = time_it(lambda: net.window(tree, ld, n, cand, idx, grid, half=args.half, win_lo=win),
                     reps)
        flop = float(E) * F_MLP_ROW
        res["mlp_infer_fused"] = {"bound": "mfma", "achieved": flop / (ms * 1e-3) / 1e12,
                                  "peak": PEAK_BF16 / 1e12, "unit": "TFLOP/s",
                                  "frac": flop / (ms * 1e-3) / PEAK_BF16, "ms": ms, "rows": E,
                                  "flop_per_row": F_MLP_ROW}
    return res


# Kernels between the library's timing events of one screened search, per
# edge form (the endpoint models before and the FP64 stage after them are
# outside the span)
EDGE_SPAN_KERNELS = {
    1: "edge_time_kernel",
    2: "edge_triage_kernel + edge_search_open_kernel",
    3: "edge_triage_kernel + tri_hist_kernel + tri_scatter_kernel + edge_search_open_kernel "
       "(ordered)",
}


# Sources each counter record depends on: a stored traffic figure applies
# only to the kernel code it was measured on.
KERNEL_SOURCES = {
    # the kernels of the timed edge-search span (EDGE_SPAN_KERNELS)
    "edge_search": ("fn_internal.h", "fn_ctx.h", "fn_edge.h", "fn_edge.hip"),
    "knn_scan": ("fn_internal.h", "fn_ctx.h", "fn_knn.h", "fn_knn.hip"),
    # the matrix-core form's record (stress shape): same sources
    "knn_scan_mfma": ("fn_internal.h", "fn_ctx.h", "fn_knn.h", "fn_knn.hip"),
}


def refine_stats(args, ctx, wl, tree, ld, n, cand, idx, grid, sh, obs, out, fn, torch):
    """Multi-round N-ary refinement below the grid result of every edge of
    the step (N = 3, eps = 1e-4 s), timed alone with HIP events: refined
    edges/s, its FP32 rate, and how far below the grid slot the refined
    minimum feasible time lies."""
    stream = torch.cuda.current_stream()
    j = out["j"].clone()
    n_ary, eps = 3, 1e-4

    def call():
        return ctx.edge_refine(tree, ld, n, cand, idx, j, grid, sh.samples, n_ary=n_ary, eps=eps,
                               obs=obs)

    for _ in range(2):
        r = call()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = max(5, args.steps)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        r = call()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    jj = j.cpu().numpy().astype(np.int64)
    f = jj >= 0
    T = r["T"].cpu().numpy().astype(np.float64)
    g = wl["grid"].astype(np.float64)
    gain = (g[jj[f]] - T[f]) / g[jj[f]]
    st = r["status"].cpu().numpy().astype(np.uint16)
    n_post = int(f.sum())
    n_clear = int((f & ((st & (fn.S_VEL | fn.S_POS)) == 0)).sum())
    work = int(r["work"].sum().item())
    flop = (work * F_EVAL + n_post * F_JOINTS
            + n_clear * f_clear(sh.samples, sh.n_obs, len(wl["arm"]["sph"])))
    return {"n_ary": n_ary, "eps_s": eps, "ms": ms, "edges": int(jj.size),
            "refined_edges": n_post, "refined_edges_per_s": n_post / (ms * 1e-3),
            "rounds_mean": float(r["rounds"].float()[torch.as_tensor(f).cuda()].mean().item()),
            "evaluations": work, "fp32_tflops": flop / (ms * 1e-3) / 1e12,
            "frac": flop / (ms * 1e-3) / PEAK_FP32,
            "T_below_grid_rel_median": float(np.median(gain)) if gain.size else None,
            "T_below_grid_rel_max": float(np.max(gain)) if gain.size else None,
            "final_ok_frac_refined": float((f & ((st & (fn.S_VEL | fn.S_POS | fn.S_COLL)) == 0)).sum()
                                           / max(1, n_post))}


def controller_stats(args, ctx, wl, fn, W, torch, n=1 << 20):
    """One step of the tracking controller of Eq. (9) for 1,048,576 seeded
    instances (states in the limits, rendezvous states, horizons U[0.02,
    0.8] s, previous torques within 80% of the limits), timed alone."""
    arm = wl["arm"]
    rng = np.random.default_rng(7)
    x = W.uniform_states(arm, n, rng, qd_scale=1.0)
    g = W.uniform_states(arm, n, rng, qd_scale=0.5)
    dev = lambda a: fn.dev(np.asarray(a, np.float32))  # noqa: E731
    q, qd, qg, qdg = dev(x[:, :7]), dev(x[:, 7:]), dev(g[:, :7]), dev(g[:, 7:])
    tp = dev(rng.uniform(-0.8, 0.8, (n, 7)) * arm["taumax"])
    T = dev(rng.uniform(0.02, 0.8, n))
    slew = np.full(7, 1000.0)
    stream = torch.cuda.current_stream()
    for _ in range(2):
        tau, qdd, st = fn.control(ctx, q, qd, tp, qg, qdg, T, 1e-3, slew)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = max(5, args.steps)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        fn.control(ctx, q, qd, tp, qg, qdg, T, 1e-3, slew)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    stn = st.cpu().numpy().astype(np.uint16)
    return {"instances": n, "ms": ms, "instances_per_s": n / (ms * 1e-3),
            "fp32_tflops": n * F_CONTROL / (ms * 1e-3) / 1e12,
            "frac": n * F_CONTROL / (ms * 1e-3) / PEAK_FP32, "flop_per_instance": F_CONTROL,
            "hbm": {"bytes_per_instance": B_CONTROL,
                    "achieved_gbs": n * B_CONTROL / (ms * 1e-3) / 1e9,
                    "frac": n * B_CONTROL / (ms * 1e-3) / PEAK_HBM},
            "clipped": {name: float(((stn & b) > 0).mean()) for name, b in
                        (("acc", fn.C_ACC), ("slew", fn.C_SLEW), ("torque", fn.C_TORQUE),
                         ("power", fn.C_POWER))}}


def kernel_source_hash(kernel="edge_search"):
    """Hash of the code a kernel is built from (comments and blank lines
    dropped)."""
    import hashlib
    import re

    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2609_22608_amd", "csrc")
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(d, name)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        lines = (re.sub(r"//.*", "", ln).rstrip() for ln in text.splitlines())
        h.update("\n".join(ln for ln in lines if ln).encode())
    return h.hexdigest()[:16]


def traffic_bytes(kernel, form):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    rec = t.get(kernel, {})
    if rec.get("source_hash") != kernel_source_hash(kernel) or rec.get("form") != form:
        return None
    return rec.get("bytes_per_launch")


def batched_round(args, fn, W, torch):
    """One round of Algorithm 1 for many uneven problems, replayed as one
    HIP graph: kNN parents, edge search (free) or fixed-duration check
    (goal), attachment to the cheapest valid parent, risk of the new goal
    nodes.  Trees are restored between replays, outside the timed events,
    so every timed replay does the same round."""
    from paper_2609_22608_amd import autotune

    n_p = args.batch_problems
    arm, probs = W.make_problem_set(n_p, seed=args.seed, nodes=(1024, 65536), batch=(256, 8192))
    k = probs[0]["shape"].k
    sumB = sum(p["shape"].batch for p in probs)
    E = sumB * k
    pairs = sum(p["shape"].batch * p["shape"].n_nodes for p in probs)
    ctx = fn.Context(arm, max(p["shape"].n_nodes + p["shape"].batch for p in probs), sumB, k,
                     max_edges=E, max_problems=n_p)
    grid = fn.dev(probs[0]["grid"])
    bt = fn.Batch(ctx, grid, probs[0]["shape"].samples, k, mode=fn.SEARCH_SCREEN)
    for wl in probs:
        bt.add_problem(wl["tree_x"], wl["tree_t"], wl["cand"], wl["obs"],
                       capacity=wl["shape"].n_nodes + wl["shape"].batch)
    bt.prepare()
    tuned = None
    if not args.no_tune:
        ch, _ = autotune.tune_batch(bt, reps=2, cache=autotune.Cache(args.tune_cache))
        tuned = ch.as_dict()
    stream = torch.cuda.current_stream()

    def timed(run, steps):
        ts = []
        for _ in range(steps):
            bt.reset_trees()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            run()
            e1.record(stream)
            ts.append((e0, e1))
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ts]))

    for _ in range(args.warmup):
        bt.reset_trees()
        bt.launch()
    ms_eager = timed(bt.launch, args.steps)
    cap = torch.cuda.Stream()
    torch.cuda.synchronize()
    bt.capture(cap)
    for _ in range(args.warmup):
        bt.reset_trees()
        bt.replay()
    ms_graph = timed(bt.replay, args.steps)
    attached = sum(int((P["out_node"] >= 0).sum().item()) for P in bt.problems)
    goals = sum(int(torch.isfinite(P["out_J"]).sum().item()) for P in bt.problems)
    res = dict(problems=n_p, candidates=sumB, edges=E, knn_pairs=pairs,
               ms_graph=ms_graph, ms_eager=ms_eager, edges_per_s=E / (ms_graph * 1e-3),
               attached=attached, goal_nodes_scored=goals, tuning=tuned,
               workload=f"{n_p} problems, tree sizes log-uniform 1,024-65,536, candidates "
                        f"log-uniform 256-8,192 (half goal), k={k}, 64 T x 32 samples, "
                        f"0-5 obstacles, seed {args.seed}")
    ctx.close()
    return res


def planning_cycle(args, fn, W, torch, V_TIP=4.0):
    """Whole planning cycles of Algorithm 1 in the paper's configuration
    (A = 2 anytime iterations of R = 2 rounds, B = 128 candidates, M = 4
    parents), each starting from the root alone, as one HIP graph: per round
    kNN, edge search below t_best (free) or the check at t_req - t(p)
    (goal), attachment, risk of goal nodes and the incumbent; Prune by
    Eq. (8) after each iteration.  One problem (latency) and 32 problems
    (throughput), 64 T x 32 samples, 5 obstacles, V_tip 4 m/s.  Trees and
    incumbents are restored between replays, outside the timed events."""
    arm = W.make_arm(0)
    blade = W.blade_midpoint(arm)
    out = {"config": "A=2, R=2, B=128 (half goals), M=4, 64 T x 32 samples, 5 obstacle spheres, "
                     "root-only tree at the start of every cycle (root at rest, goal poses within "
                     "0.8 rad of it, arrivals in the flight's reach window), V_tip 4 m/s, blade "
                     "point at the middle of the 0.30 m edge",
           "paper_solve_ms": {"value": 12.0, "note": "median solve time of the whole planner "
                                                     "(sampling included), RTX 4090 + JAX; "
                                                     "context only"}}
    stream = torch.cuda.current_stream()
    for n_p in (1, 32):
        probs = [W.make_cycle_problem(arm, args.seed + p, 1, 128, k=4, rounds=4, n_obs=5, n_t=64,
                                      samples=32, with_goal_parents=False, root_at_rest=True,
                                      goal_spread=0.8) for p in range(n_p)]
        ctx = fn.Context(arm, 1024, 128 * n_p, 4, max_edges=512 * n_p, max_problems=n_p)
        bt = fn.Batch(ctx, fn.dev(probs[0]["grid"]), 32, 4, mode=fn.SEARCH_SCREEN)
        for c in probs:
            bt.add_problem(c["tree_x"], c["tree_t"], c["rounds"], c["obs"], capacity=516,
                           flight=c["flight"])
        # both searches of a batched round (one kernel; triage, sort and the
        # ordered search): the same cycle, the faster one reported
        by_form = {}
        for ef in (1, 3):
            ctx.set_tuning(edge_form=ef)
            bt.prepare()
            cap = torch.cuda.Stream()
            torch.cuda.synchronize()
            bt.capture_cycle(cap, 2, 2, V_TIP, blade)
            for _ in range(args.warmup):
                bt.reset_trees()
                bt.replay()
            ts = []
            for _ in range(max(5, args.steps)):
                bt.reset_trees()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                bt.replay()
                e1.record(stream)
                ts.append((e0, e1))
            torch.cuda.synchronize()
            by_form[ef] = float(np.median([a.elapsed_time(b) for a, b in ts]))
        ef_best = min(by_form, key=by_form.get)
        ms = by_form[ef_best]
        inc = np.stack([P["incumbent"].cpu().numpy() for P in bt.problems])
        nodes = [int(P["n_nodes"].item()) for P in bt.problems]
        out[f"problems_{n_p}"] = {
            "ms_per_cycle": ms, "cycles_per_s": n_p / (ms * 1e-3), "edge_form": ef_best,
            "ms_per_cycle_by_edge_form": by_form,
            "edges_per_cycle": 4 * 128 * 4 * n_p,
            "found": int((inc[:, 1] >= 0).sum()),
            "J_best_median": (float(np.median(inc[inc[:, 1] >= 0, 0]))
                              if (inc[:, 1] >= 0).any() else None),
            "nodes_after_cycle_median": float(np.median(nodes))}
        ctx.close()
    return out


def surrogate(args, ctx, arm, sh, fn, W, torch):
    """The T-window network: loaded from a checkpoint, or trained here to the
    recipe (one-iteration batches with seeds disjoint from the benchmark's,
    labelled by the exact search, 20 epochs of minibatch 4,096, Adam with a
    cosine-decayed learning rate from 3e-3) by the library's own kernels."""
    if args.surrogate and os.path.exists(args.surrogate):
        return fn.Surrogate.load(ctx, args.surrogate), {"checkpoint": args.surrogate}
    from paper_2609_22608_amd import train_surrogate as TS

    t0 = time.perf_counter()
    X, y, grid = TS.label_batches(ctx, arm, sh, range(1000, 1000 + args.train_batches), fn,
                                  torch, W)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    net = fn.Surrogate(ctx, seed=1)
    t1 = time.perf_counter()
    losses = net.train(X, y, grid, epochs=args.train_epochs, batch=4096, lr=LR_SURROGATE)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    L = losses.cpu().numpy()
    rows = X.shape[0] // 4096 * 4096 * args.train_epochs
    info = {"train_edges": int(X.shape[0]), "epochs": args.train_epochs,
            "seeds": f"1000..{999 + args.train_batches}",
            "feasible_frac": float((y >= 0).float().mean().item()),
            "lr": LR_SURROGATE,
            "loss_first_last": [float(L[0, 0]), float(L[-1, 0])],
            "label_s": t_data, "train_s": t_train,
            "train_bf16_tflops": rows * 3 * F_MLP_ROW / t_train / 1e12}
    del X, y
    return net, info


def diagnostics(o, sh, fn):
    """Outcome mix of the workload's edges (from the library's results)."""
    j = o["j"].cpu().numpy().astype(np.int64)
    st = o["status"].cpu().numpy().astype(np.uint16)
    feas = j >= 0
    ok = feas & ((st & (fn.S_VEL | fn.S_POS | fn.S_COLL)) == 0)
    hist = np.bincount(j[feas], minlength=sh.n_t).tolist() if feas.any() else [0] * sh.n_t
    q = np.quantile(j[feas], [0.1, 0.5, 0.9]).tolist() if feas.any() else None
    return {"edges": int(len(j)), "feasible_frac": float(feas.mean()),
            "final_ok_frac": float(ok.mean()),
            "vel_fail_frac": float(((st & fn.S_VEL) > 0).mean()),
            "pos_fail_frac": float(((st & fn.S_POS) > 0).mean()),
            "coll_fail_frac": float(((st & fn.S_COLL) > 0).mean()),
            "recheck64_frac": float(((st & fn.S_RECHECK64) > 0).mean()),
            "no_parent_frac": float(((st & fn.S_NO_PARENT) > 0).mean()),
            "j_star_p10_p50_p90": q, "j_star_hist": hist}


def cpu_baseline(wl, n_queries):
    """The FP64 oracle on the host cores: kNN + plain search of a bounded
    sample of the same workload's candidates, on all usable cores (up to 16)
    and on one thread (a smaller sample)."""
    import oracle as O

    sh = wl["shape"]
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(sh.batch, n_queries, replace=False))
    A = O.make_oarm(wl["arm"])
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    threads = max(1, min(threads, 16))
    chunks = np.array_split(rows, threads * 4)

    def job(r):
        idx, _ = O.plan_knn(wl["tree_x"], wl["cand"]["x"][r], sh.k)
        x0, x1, ok = O.edges_of(wl["tree_x"], wl["cand"]["x"][r], idx)
        O.edge_time(A, x0, x1, wl["grid"], sh.samples, wl["obs"], parent_ok=ok, scan=1)
        return len(x0)

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        edges = sum(ex.map(job, chunks))
    dt = time.perf_counter() - t0
    one = rows[: max(1, len(rows) // (4 * threads))]
    t1 = time.perf_counter()
    e1 = job(one)
    dt1 = time.perf_counter() - t1
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": edges / dt, "unit": "edges/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_queries} of {sh.batch} candidates ({edges} edges), kNN over the full "
                      f"{sh.n_nodes}-node tree + plain ascending search, FP64, {dt:.1f} s wall",
            "one_thread": {"value": e1 / dt1, "sample": f"{len(one)} candidates ({e1} edges), "
                                                         f"{dt1:.1f} s"},
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
            "nproc": os.cpu_count(), "cpu": cpu}


if __name__ == "__main__":
    main()
