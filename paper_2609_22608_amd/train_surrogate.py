"""Train and evaluate the learned T-window surrogate.

Recipe: one-iteration-shaped batches (16,384-node tree, 4,096 candidates of
which half are goal samples, k = 8, 64 durations over 0.02-1.0 s, 32 samples,
5 obstacles) are labelled by the exact search on the GPU; the network is
trained on their edges with the library's own forward / backward / Adam
kernels; held-out batches (seeds >= 1e6) measure the window miss rate, the
log-T error and the throughput of plain, screened and windowed search (all
three checked equal edge by edge).

    python -m paper_2609_22608_amd.train_surrogate --edges 10000000 --epochs 20 \
        --save surrogate.bin --report report.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def log(msg):
    print(f"[train_surrogate {time.strftime('%H:%M:%S')}] {msg}", flush=True)


def label_batches(ctx, arm, sh, seeds, fn, torch, W, workers=8):
    """Edge features and exact slot labels of the given workload seeds.  Host
    processes (spawned; they import numpy only and never touch the GPU) draw
    upcoming workloads, at most 2 x workers ahead, while the GPU labels the
    current one."""
    import collections
    import concurrent.futures as cf
    import multiprocessing as mp

    grid = fn.dev(W.t_grid(sh.n_t, sh.t_min, sh.t_max))
    Xs, ys = [], []
    seeds = list(seeds)
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        pending = collections.deque()
        nxt = 0
        for i in range(len(seeds)):
            while nxt < len(seeds) and len(pending) < 2 * workers:
                pending.append(ex.submit(W.make_workload, sh, seeds[nxt], 0, arm))
                nxt += 1
            _label_one(ctx, sh, pending.popleft().result(), grid, fn, Xs, ys)
            if (i + 1) % 50 == 0:
                log(f"labelled {i + 1}/{len(seeds)} batches")
    return torch.cat(Xs), torch.cat(ys), grid


def _label_one(ctx, sh, wl, grid, fn, Xs, ys):
    """Appends one workload's edge features and exact slot labels."""
    tree, ld, n = fn.tree_soa(wl["tree_x"])
    cand = fn.dev(wl["cand"]["x"])
    idx, _ = ctx.plan_knn(tree, ld, n, cand, sh.k, want_d2=False)
    out = ctx.edge_time_batch(tree, ld, n, cand, idx, grid, sh.samples, fn.dev(wl["obs"]),
                              mode=fn.SEARCH_SCREEN, want_rho=False, want_work=False)
    Xs.append(fn.edge_features(ctx, tree, ld, n, cand, idx))
    ys.append(out["j"].clone())


def evaluate(ctx, net, arm, sh, seeds, fn, torch, W, half=4, logit_min=0.0, reps=5):
    grid_np = W.t_grid(sh.n_t, sh.t_min, sh.t_max)
    grid = fn.dev(grid_np)
    lg = np.log(grid_np.astype(np.float64))
    stats = dict(edges=0, feasible=0, miss_feasible=0, miss_all=0, below=0, pred_infeasible=0,
                 true_infeasible=0, logT_abs_err=[], mismatches=0,
                 work={"plain": 0, "screen": 0, "window": 0},
                 ms={"plain": [], "screen": [], "window": []})
    stream = torch.cuda.current_stream()
    for seed in seeds:
        wl = W.make_workload(sh, seed=seed, arm=arm)
        tree, ld, n = fn.tree_soa(wl["tree_x"])
        cand = fn.dev(wl["cand"]["x"])
        obs = fn.dev(wl["obs"])
        idx, _ = ctx.plan_knn(tree, ld, n, cand, sh.k, want_d2=False)
        outs = {}
        for name, mode in (("plain", fn.SEARCH_PLAIN), ("screen", fn.SEARCH_SCREEN),
                           ("window", fn.SEARCH_WINDOW)):
            for r in range(reps + 1):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                pred = None
                if mode == fn.SEARCH_WINDOW:
                    feats = fn.edge_features(ctx, tree, ld, n, cand, idx)
                    pred, win = net.infer(feats, grid, half=half, logit_min=logit_min)
                    o = ctx.edge_time_batch(tree, ld, n, cand, idx, grid, sh.samples, obs,
                                            mode=mode, win_lo=win, win_half=half)
                else:
                    o = ctx.edge_time_batch(tree, ld, n, cand, idx, grid, sh.samples, obs,
                                            mode=mode)
                e1.record(stream)
                torch.cuda.synchronize()
                if r > 0:
                    stats["ms"][name].append(e0.elapsed_time(e1))
            outs[name] = (o, pred)
        a = outs["plain"][0]
        jp = a["j"].cpu().numpy().astype(np.int64)
        sp = a["status"].cpu().numpy().astype(np.uint16) & fn.S_DECISION
        for name in ("screen", "window"):
            o = outs[name][0]
            jj = o["j"].cpu().numpy().astype(np.int64)
            ss = o["status"].cpu().numpy().astype(np.uint16) & fn.S_DECISION
            stats["mismatches"] += int(((jj != jp) | (ss != sp)).sum())
        for name in ("plain", "screen", "window"):
            stats["work"][name] += int(outs[name][0]["work"].sum().item())
        ow, pred = outs["window"]
        sw = ow["status"].cpu().numpy().astype(np.uint16)
        feas = jp >= 0
        miss = (sw & fn.S_WIN_MISS) > 0
        stats["edges"] += len(jp)
        stats["feasible"] += int(feas.sum())
        stats["miss_feasible"] += int((miss & feas).sum())
        stats["miss_all"] += int(miss.sum())
        stats["below"] += int(((sw & fn.S_WIN_BELOW) > 0).sum())
        stats["true_infeasible"] += int((~feas).sum())
        y = pred.cpu().numpy().astype(np.float64)
        stats["pred_infeasible"] += int((y[:, 1] < logit_min).sum())
        lt_hat = 0.5 * (lg[0] + lg[-1]) + 0.5 * (lg[-1] - lg[0]) * y[:, 0]
        stats["logT_abs_err"].extend(np.abs(lt_hat[feas] - lg[jp[feas]]).tolist())
    err = np.asarray(stats.pop("logT_abs_err"))
    ms = {k: float(np.median(v)) for k, v in stats.pop("ms").items()}
    E = stats["edges"] / len(seeds)
    res = dict(stats)
    res.update(
        miss_rate_feasible=stats["miss_feasible"] / max(1, stats["feasible"]),
        miss_rate_all=stats["miss_all"] / max(1, stats["edges"]),
        below_window_rate=stats["below"] / max(1, stats["edges"]),
        logT_err_median=float(np.median(err)) if len(err) else None,
        logT_err_p90=float(np.quantile(err, 0.9)) if len(err) else None,
        bin_width_logT=float((lg[-1] - lg[0]) / (len(lg) - 1)),
        edge_call_ms=ms,
        edges_per_s={k: E / (v * 1e-3) for k, v in ms.items()},
    )
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--edges", type=int, default=10_000_000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--eval-batches", type=int, default=8)
    ap.add_argument("--half", type=int, default=4)
    ap.add_argument("--save", default=None)
    ap.add_argument("--report", default=None)
    args = ap.parse_args()
    import torch

    from paper_2609_22608_amd import fn, workload as W

    sh = W.CONFIGS["iteration"]
    arm = W.make_arm(0)
    E = sh.batch * sh.k
    ctx = fn.Context(arm, sh.n_nodes, sh.batch, sh.k, max_edges=E)
    nb = max(1, math.ceil(args.edges / E))
    t0 = time.perf_counter()
    X, y, grid = label_batches(ctx, arm, sh, range(1000, 1000 + nb), fn, torch, W)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    log(f"{X.shape[0]} labelled edges in {t_data:.1f} s; F-feasible "
        f"{(y >= 0).float().mean().item():.3f}")
    net = fn.Surrogate(ctx, seed=1)
    t0 = time.perf_counter()
    losses = net.train(X, y, grid, epochs=args.epochs, batch=args.batch, lr=args.lr)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    L = losses.cpu().numpy()
    log(f"trained {args.epochs} epochs in {t_train:.1f} s; loss {L[0, 0]:.4f} -> {L[-1, 0]:.4f}")
    rows = X.shape[0] // args.batch * args.batch * args.epochs
    flop = rows * 3 * 2 * (28 * 256 + 2 * 256 * 256 + 256 * 2)
    if args.save:
        net.save(args.save)
    del X, y
    ev = evaluate(ctx, net, arm, sh, range(1_000_000, 1_000_000 + args.eval_batches), fn, torch,
                  W, half=args.half)
    log(f"held-out: miss rate {ev['miss_rate_feasible']:.4f} (feasible edges), "
        f"mismatches {ev['mismatches']}, edges/s {ev['edges_per_s']}")
    rep = dict(train_edges=nb * E, epochs=args.epochs, batch=args.batch, lr=args.lr,
               data_s=t_data, train_s=t_train, train_tflops=flop / t_train / 1e12,
               epoch_loss=L.tolist(), eval=ev)
    print(json.dumps(rep), flush=True)
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)
    net.close()
    ctx.close()


if __name__ == "__main__":
    main()
