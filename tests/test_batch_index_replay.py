"""Host replay of the batched round's index arithmetic (no GPU).

The batched search launches one grid over all problems' edges; a wavefront
decodes its global edge id into (problem, local edge) by binary search over
per-problem prefix offsets, and the FP64 stage decodes the global edge id a
queue entry carries the same way.  Per-problem argument blocks hold pointers
pre-offset to the problem's part of the shared scratch (endpoint models of
parents by edge, of candidates by candidate).  This replays that arithmetic,
as the kernels and fn_batch_prepare write it, for every edge of the
benchmark's 32-problem round, asserting that every access the search and the
FP64 stage make lies inside its allocation; and it measures the three misuses
that an earlier, removed variant of the FP64 stage was suspected of (see the
design notes): a global edge id against the pre-offset model pointers, the
models of goal or padded edges (never written), and problem 0's argument
block used for another problem's arrays."""
import numpy as np

from paper_2609_22608_amd import workload as W

MODEL = 56  # floats per endpoint model
N_XCD = 8


def problem_of(off, eg):
    """The kernels' binary search: largest p with off[p] <= eg (n problems)."""
    n = len(off) - 1
    lo = np.zeros_like(eg)
    hi = np.full_like(eg, n - 1)
    while np.any(lo < hi):
        mid = (lo + hi + 1) >> 1
        go = off[mid] <= eg
        lo = np.where(go & (lo < hi), mid, lo)
        hi = np.where(~go & (lo < hi), mid - 1, hi)
    return lo


def xcd_edge(w, k, B):
    s = w // N_XCD
    b = (s // k) * N_XCD + (w % N_XCD)
    return np.where(b < B, b * k + s % k, -1)


def test_batched_round_indices_stay_in_bounds():
    arm, probs = W.make_problem_set(32, 101, nodes=(1024, 65536), batch=(256, 8192))
    k = probs[0]["shape"].k
    Bs = np.array([p["shape"].batch for p in probs], np.int64)
    ns = np.array([p["shape"].n_nodes for p in probs], np.int64)
    ld = ns + Bs  # the benchmark's capacity: n + B, a multiple of 4 after rounding up
    ld = (ld + 3) // 4 * 4
    eo = np.concatenate([[0], np.cumsum(Bs * k)])
    qo = np.concatenate([[0], np.cumsum(Bs)])
    E, sumB = int(eo[-1]), int(qo[-1])
    max_edges, max_batch = E, sumB  # the benchmark's context caps
    # search grid: every global edge exactly once
    grid = (sumB + N_XCD - 1) // N_XCD * N_XCD * k
    eg = xcd_edge(np.arange(grid, dtype=np.int64), k, sumB)
    eg = eg[eg >= 0]
    assert eg.size == E and np.array_equal(np.sort(eg), np.arange(E))
    # decode (search kernel and FP64 stage alike)
    p = problem_of(eo, eg)
    loc = eg - eo[p]
    assert (loc >= 0).all() and (loc < Bs[p] * k).all()
    b = loc // k
    assert (b < Bs[p]).all()
    # endpoint models through the pre-offset per-problem pointers
    me_end = (eo[p] + loc) * MODEL + MODEL
    mc_end = (qo[p] + b) * MODEL + MODEL
    assert me_end.max() <= max_edges * MODEL
    assert mc_end.max() <= max_batch * MODEL
    # queue entries: one per edge at most
    assert E <= max_edges
    # parent rows: any parent index below the problem's node count lies in its tree
    assert (ns <= ld).all()
    # the misuses: (1) a global id against a pre-offset model pointer
    bad_me = ((eo[p] + eg) * MODEL + MODEL) > max_edges * MODEL
    bad_mc = ((qo[p] + eg // k) * MODEL + MODEL) > max_batch * MODEL
    # (3) problem 0's block for problem p: parents of problem p read from
    # problem 0's tree, problem p's local candidate index against problem 0's
    # candidates
    bad_tree = (ns[p] > ld[0])
    bad_cand = b >= Bs[0]
    print(f"{E} edges, {sumB} candidates; global id against the pre-offset parent models "
          f"leaves the buffer for {bad_me.sum()} edges, candidate models for {bad_mc.sum()}; "
          f"problem 0's block: tree reads past its rows possible for {bad_tree.sum()} edges, "
          f"candidate reads past its batch for {bad_cand.sum()}")
    # (2) models of goal and padded edges are never written, but their slots lie
    # inside the buffers like every other edge's (reading them cannot leave an
    # allocation)
    assert bad_me.sum() > 0 and bad_mc.sum() > 0 and bad_tree.sum() > 0 and bad_cand.sum() > 0
