"""Seeded synthetic workloads for the edge-timing path.

This module only draws random numbers and arranges them into the arrays that
both the GPU library and the FP64 checker consume.  It holds none of the
method's arithmetic (no cubic, no dynamics, no limit ratios, no distances):
every array it returns is an *input*.  All floating-point values are rounded
to FP32 once, here, so that both consumers read identical bits (doubles that
are exactly FP32-representable, except the DH twist angles, which are exact
multiples of pi/2 handled as such by both sides).

One exception is documented: goal candidates are placed by an inverse
construction (pick a goal configuration, place the object's flight through a
point of the blade edge), which needs the blade pose.  That pose comes from a
small forward-kinematics routine private to this module
(``_synth_fk``).  It only positions inputs; neither the kernels nor the
checker call it, and no expected value depends on it.

Workload recipes follow the paper's experimental setup (Sec. V: 7-DOF arm,
B candidates x M parents, ballistic flights, obstacles) at the sizes of the
five benchmark shapes used by this project (see ``CONFIGS``).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional

import numpy as np

DOF = 7
STATE = 2 * DOF  # (q, qd)

# Modified-DH twist angles alpha_{i-1} for joints 1..7 (a Panda/FR3-like
# pattern: every twist is 0 or +-pi/2).
ALPHA_7DOF = np.array([0.0, -math.pi / 2, math.pi / 2, math.pi / 2,
                       -math.pi / 2, math.pi / 2, math.pi / 2])

KIND_FREE = 0
KIND_GOAL = 1


def _f32(x):
    """Round to FP32 and return FP64 holding the same value."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# Arm
# ---------------------------------------------------------------------------

def make_arm(seed: int = 0, n_spheres: int = 40, w_max: float = 300.0,
             armature: bool = True, friction: bool = True,
             sphere_r=(0.04, 0.08), alpha=None) -> Dict[str, np.ndarray]:
    """Seeded synthetic 7-DOF revolute arm (modified DH).

    Joint i's frame is Rx(alpha_{i-1}) Tx(a_{i-1}) Rz(q_i) Tz(d_i).  Link
    lengths a, d ~ U[0.05, 0.35] m, masses U[0.5, 4] kg, diagonal inertias
    about the COM U[0.005, 0.05] kg m^2 (resampled until the triangle
    inequality holds), joint limits +-2.8 rad, velocity limits U[2.0, 2.6]
    rad/s and torque limits U[12, 87] N m (both sorted from proximal to
    distal), power limit ``w_max``.  Reflected rotor inertia and the sigmoid
    friction parameters of Eq. (5) are synthetic (the identified values the
    paper adopts are not printed).  ``acc`` is the braking deceleration that
    defines the position-dependent velocity taper.
    """
    rng = np.random.default_rng(seed)
    n = DOF
    alpha = ALPHA_7DOF.copy() if alpha is None else np.asarray(alpha, np.float64)
    a = rng.uniform(0.05, 0.35, n)
    d = rng.uniform(0.05, 0.35, n)
    a[0] = 0.0  # first axis through the base origin
    tool = np.array([0.0, 0.0, 0.10])
    # segment of link i: origin of frame i+1 expressed in frame i
    seg = np.zeros((n, 3))
    for i in range(n - 1):
        seg[i] = (a[i + 1], -math.sin(alpha[i + 1]) * d[i + 1],
                  math.cos(alpha[i + 1]) * d[i + 1])
    seg[n - 1] = tool
    seg = np.where(np.abs(seg) < 1e-12, 0.0, seg)
    m = rng.uniform(0.5, 4.0, n)
    lam = rng.uniform(0.3, 0.7, n)
    rc = lam[:, None] * seg + rng.uniform(-0.02, 0.02, (n, 3))
    inertia = np.zeros((n, 3))
    for i in range(n):
        while True:
            v = rng.uniform(0.005, 0.05, 3)
            if v[0] + v[1] >= v[2] and v[1] + v[2] >= v[0] and v[0] + v[2] >= v[1]:
                inertia[i] = v
                break
    im = np.sort(rng.uniform(0.01, 0.1, n))[::-1] if armature else np.zeros(n)
    psi1 = rng.uniform(0.1, 0.6, n) if friction else np.zeros(n)
    psi2 = rng.uniform(5.0, 50.0, n)
    psi3 = rng.uniform(-0.05, 0.05, n)
    qdmax = np.sort(rng.uniform(2.0, 2.6, n))[::-1]
    taumax = np.sort(rng.uniform(12.0, 87.0, n))[::-1]
    # collision spheres, split over links 1..7 in proportion to segment length
    seglen = np.linalg.norm(seg, axis=1)
    share = seglen / seglen.sum() * n_spheres
    cnt = np.maximum(1, np.floor(share).astype(int))
    while cnt.sum() < n_spheres:
        cnt[np.argmax(share - cnt)] += 1
    while cnt.sum() > n_spheres:
        cnt[np.argmax(cnt)] -= 1
    sph_link, sph = [], []
    for i in range(n):
        for j in range(cnt[i]):
            c = (j + 0.5) / cnt[i] * seg[i]
            sph_link.append(i + 1)
            sph.append([c[0], c[1], c[2], rng.uniform(*sphere_r)])
    arm = dict(
        n=n,
        alpha=alpha,
        a=_f32(a), d=_f32(d), m=_f32(m), rc=_f32(rc), I=_f32(inertia),
        Im=_f32(im), psi1=_f32(psi1), psi2=_f32(psi2), psi3=_f32(psi3),
        qmin=_f32(np.full(n, -2.8)), qmax=_f32(np.full(n, 2.8)),
        qdmax=_f32(qdmax), taumax=_f32(taumax), acc=_f32(np.full(n, 10.0)),
        wmax=float(np.float32(w_max)), g=_f32([0.0, 0.0, -9.81]),
        tool=_f32(tool),
        sph_link=np.asarray(sph_link, np.int32), sph=_f32(np.asarray(sph)),
        # blade (input synthesis only): 0.30 m edge along x7 from the tool
        # point, cutting direction y7
        blade_base=_f32(tool), blade_dir=_f32([1.0, 0.0, 0.0]),
        blade_len=0.30, blade_normal=_f32([0.0, 1.0, 0.0]),
    )
    return arm


def reach(arm) -> float:
    """Sum of link segment lengths (an upper bound of the arm's reach)."""
    tot = abs(arm["d"][0])
    for i in range(1, arm["n"]):
        tot += math.hypot(arm["a"][i], arm["d"][i])
    return float(tot + np.linalg.norm(arm["tool"]))


# ---------------------------------------------------------------------------
# Travel-time grid
# ---------------------------------------------------------------------------

def t_grid(n_t: int, t_min: float, t_max: float) -> np.ndarray:
    """Geometric grid of candidate travel times, endpoints included, FP32."""
    j = np.arange(n_t, dtype=np.float64)
    return _f32(t_min * (t_max / t_min) ** (j / (n_t - 1)))


# ---------------------------------------------------------------------------
# States
# ---------------------------------------------------------------------------

def uniform_states(arm, n: int, rng, qd_scale: float = 0.5) -> np.ndarray:
    """(q, qd) uniform within the joint box, qd within qd_scale * qdmax."""
    q = rng.uniform(arm["qmin"], arm["qmax"], (n, DOF))
    qd = rng.uniform(-qd_scale * arm["qdmax"], qd_scale * arm["qdmax"], (n, DOF))
    return _f32(np.concatenate([q, qd], axis=1))


def make_tree(arm, n: int, seed: int, qd_scale: float = 0.5):
    """Tree nodes: states uniform within the limits (qd scaled), and a
    time-to-come t_n ~ U[0, 0.3] s.  Returns (states [n][14], t [n])."""
    rng = np.random.default_rng([seed, 1])
    x = uniform_states(arm, n, rng, qd_scale)
    t = _f32(rng.uniform(0.0, 0.3, n))
    return x, t


def _dh(alpha, a, d, q):
    """4x4 homogeneous transforms Rx(alpha) Tx(a) Rz(q) Tz(d), batched over q."""
    ca, sa = math.cos(alpha), math.sin(alpha)
    if abs(ca) < 1e-12:
        ca = 0.0
    if abs(sa) < 1e-12:
        sa = 0.0
    cq, sq = np.cos(q), np.sin(q)
    T = np.zeros(q.shape + (4, 4))
    T[..., 0, 0] = cq
    T[..., 0, 1] = -sq
    T[..., 0, 3] = a
    T[..., 1, 0] = sq * ca
    T[..., 1, 1] = cq * ca
    T[..., 1, 2] = -sa
    T[..., 1, 3] = -sa * d
    T[..., 2, 0] = sq * sa
    T[..., 2, 1] = cq * sa
    T[..., 2, 2] = ca
    T[..., 2, 3] = ca * d
    T[..., 3, 3] = 1.0
    return T


def _synth_fk(arm, q):
    """Flange pose (4x4) for configurations q [n][7]; goal synthesis only."""
    T = np.broadcast_to(np.eye(4), q.shape[:-1] + (4, 4)).copy()
    for i in range(arm["n"]):
        T = T @ _dh(arm["alpha"][i], arm["a"][i], arm["d"][i], q[..., i])
    return T


def _blade_point(arm, q, c):
    T = _synth_fk(arm, q)
    local = arm["blade_base"] + (c * arm["blade_len"])[..., None] * arm["blade_dir"]
    return np.einsum("...ij,...j->...i", T[..., :3, :3], local) + T[..., :3, 3], T


def goal_states(arm, n: int, rng, t_arr=(0.2, 0.8), launch=(4.0, 7.0),
                cone_deg: float = 30.0, blade_speed=(0.5, 2.0), g=9.81, q_center=None,
                q_spread: float = 0.8):
    """Goal candidates by inverse construction.

    A goal configuration q_g is drawn in the joint box; the contact point p
    lies on the 0.30 m blade edge; the arrival time is U[t_arr]; the object's
    velocity at arrival points into the blade within ``cone_deg`` of the
    cutting direction and the flight is the ballistic arc of Eq. (1) through
    p with launch speed U[launch]; the blade moves along its cutting
    direction at U[blade_speed] m/s and qd_g = J^+ v_ee.  Samples whose qd_g
    leaves the velocity box, whose contact point is below 5 cm or whose arc
    has no real launch solution are redrawn.  With q_center, q_g is drawn
    within +-q_spread of it (clipped to 0.9 of the joint box) instead.

    Returns (states [n][14], T_req [n], flight dict of per-sample arrays).
    """
    out_x, out_t, fl = [], [], {k: [] for k in ("x0", "v0", "t_fall", "v_rel")}
    gvec = np.array([0.0, 0.0, -g])
    cos_cone = math.cos(math.radians(cone_deg))
    need = n
    while need > 0:
        m = max(64, 2 * need)
        if q_center is None:
            q = rng.uniform(0.9 * arm["qmin"], 0.9 * arm["qmax"], (m, DOF))
        else:
            q = np.clip(np.asarray(q_center, np.float64)[:DOF]
                        + rng.uniform(-q_spread, q_spread, (m, DOF)),
                        0.9 * arm["qmin"], 0.9 * arm["qmax"])
        c = rng.uniform(0.0, 1.0, m)
        p, T = _blade_point(arm, q, c)
        nb = np.einsum("...ij,j->...i", T[..., :3, :3], arm["blade_normal"])
        # positional Jacobian of the contact point by central differences
        J = np.zeros((m, 3, DOF))
        h = 1e-6
        for j in range(DOF):
            dq = np.zeros(DOF)
            dq[j] = h
            pp, _ = _blade_point(arm, q + dq, c)
            pm, _ = _blade_point(arm, q - dq, c)
            J[:, :, j] = (pp - pm) / (2 * h)
        bs = rng.uniform(*blade_speed, m)
        v_ee = bs[:, None] * nb
        qd = np.einsum("nij,nj->ni", np.linalg.pinv(J), v_ee)
        # object velocity direction: cone about -n_b
        ct = rng.uniform(cos_cone, 1.0, m)
        st = np.sqrt(1 - ct * ct)
        ph = rng.uniform(0, 2 * math.pi, m)
        e1 = np.cross(nb, np.array([0.0, 0.0, 1.0]))
        bad = np.linalg.norm(e1, axis=1) < 1e-6
        e1[bad] = np.cross(nb[bad], np.array([1.0, 0.0, 0.0]))
        e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
        e2 = np.cross(nb, e1)
        dirv = -ct[:, None] * nb + st[:, None] * (np.cos(ph)[:, None] * e1 + np.sin(ph)[:, None] * e2)
        ta = rng.uniform(*t_arr, m)
        s = rng.uniform(*launch, m)
        gT = gvec[None, :] * ta[:, None]
        dg = np.einsum("ni,ni->n", dirv, gT)
        disc = dg * dg - np.einsum("ni,ni->n", gT, gT) + s * s
        lam = dg + np.sqrt(np.maximum(disc, 0.0))
        xd_T = lam[:, None] * dirv
        v0 = xd_T - gT
        x0 = p - v0 * ta[:, None] - 0.5 * gvec[None, :] * ta[:, None] ** 2
        # fall time: later root of x_z(t) = 0
        aa, bb, cc = 0.5 * gvec[2], v0[:, 2], x0[:, 2]
        dd = np.maximum(bb * bb - 4 * aa * cc, 0.0)
        t_fall = (-bb - np.sqrt(dd)) / (2 * aa)
        v_rel = np.linalg.norm(v_ee - xd_T, axis=1)
        ok = ((disc > 0) & (lam > 0) & (p[:, 2] > 0.05)
              & np.all(np.abs(qd) <= arm["qdmax"], axis=1) & (t_fall > ta))
        idx = np.nonzero(ok)[0][:need]
        out_x.append(np.concatenate([q[idx], qd[idx]], axis=1))
        out_t.append(ta[idx])
        fl["x0"].append(x0[idx])
        fl["v0"].append(v0[idx])
        fl["t_fall"].append(t_fall[idx])
        fl["v_rel"].append(v_rel[idx])
        need -= len(idx)
    x = _f32(np.concatenate(out_x))
    t = _f32(np.concatenate(out_t))
    flight = {k: _f32(np.concatenate(v)) for k, v in fl.items()}
    return x, t, flight


def chord_states(arm, root, goals, n: int, rng, sigma: float = 0.15, p_uniform: float = 0.2,
                 qd_frac: float = 0.3) -> np.ndarray:
    """Free states of Algorithm 1's ChordSample: a configuration on the
    joint-space chord from the root to a random goal (uniform position along
    it) perturbed by N(0, sigma^2) rad per joint, or, with probability
    p_uniform, uniform over the joint box; clipped to the box.  Velocities
    uniform within +-qd_frac of the joint-velocity limits."""
    q0 = np.asarray(root, np.float64)[:DOF]
    qg = np.asarray(goals, np.float64)[rng.integers(0, len(goals), n), :DOF]
    s = rng.uniform(0, 1, (n, 1))
    q = q0 + s * (qg - q0) + rng.normal(0, sigma, (n, DOF))
    uni = rng.random(n) < p_uniform
    q[uni] = rng.uniform(arm["qmin"], arm["qmax"], (int(uni.sum()), DOF))
    q = np.clip(q, arm["qmin"], arm["qmax"])
    qd = rng.uniform(-qd_frac, qd_frac, (n, DOF)) * arm["qdmax"]
    return np.concatenate([q, qd], 1)


def make_candidates(arm, b: int, goal_frac: float, seed: int, qd_scale: float = 0.5,
                    root=None, t_arr=(0.2, 0.8), goal_spread=None):
    """Candidate batch: a fraction ``goal_frac`` of goal samples (inverse
    construction, first), the rest uniform -- or, when a root state is given
    and there are goals, chord samples (``chord_states``).  Goal arrival
    times are U[t_arr]; with goal_spread (and a root), goal configurations
    lie within +-goal_spread rad of the root's.  Returns a dict
    with ``x`` [b][14], ``kind`` [b] (0 free, 1 goal), ``t_req`` [b] (0 for
    free) and per-goal flight data (x0, v0, t_fall, v_rel; zeros for free
    samples)."""
    rng = np.random.default_rng([seed, 2])
    n_goal = int(round(goal_frac * b))
    xs = np.zeros((b, STATE))
    kind = np.zeros(b, np.int32)
    t_req = np.zeros(b)
    flight = dict(x0=np.zeros((b, 3)), v0=np.zeros((b, 3)), t_fall=np.zeros(b), v_rel=np.zeros(b))
    if n_goal:
        if goal_spread is not None and root is not None:
            xg, tg, fg = goal_states(arm, n_goal, rng, t_arr=t_arr, q_center=root,
                                     q_spread=goal_spread)
        else:
            xg, tg, fg = goal_states(arm, n_goal, rng, t_arr=t_arr)
        xs[:n_goal] = xg
        kind[:n_goal] = KIND_GOAL
        t_req[:n_goal] = tg
        for k in flight:
            flight[k][:n_goal] = fg[k]
    if root is not None and n_goal:
        xs[n_goal:] = chord_states(arm, root, xs[:n_goal], b - n_goal, rng)
    else:
        xs[n_goal:] = uniform_states(arm, b - n_goal, rng, qd_scale)
    return dict(x=_f32(xs), kind=kind, t_req=_f32(t_req),
                flight={k: _f32(v) for k, v in flight.items()})


def make_obstacles(arm, n_obs: int, seed: int, r=(0.05, 0.15)) -> np.ndarray:
    """Obstacle spheres [n_obs][4] = (centre xyz, radius): centres 0.25-0.8 of
    the reach from the base, z >= 0, clear of the base column (links 0-1)."""
    rng = np.random.default_rng([seed, 3])
    R = reach(arm)
    col_r = 0.15 + abs(arm["a"][1])
    col_h = float(arm["d"][0]) + 0.1
    out = []
    while len(out) < n_obs:
        rad = rng.uniform(*r)
        dist = rng.uniform(0.25 * R, 0.8 * R)
        v = rng.normal(size=3)
        v[2] = abs(v[2])
        v /= np.linalg.norm(v)
        cpos = dist * v
        if math.hypot(cpos[0], cpos[1]) < col_r + rad and cpos[2] < col_h + rad:
            continue
        out.append([cpos[0], cpos[1], cpos[2], rad])
    return _f32(np.asarray(out).reshape(n_obs, 4))


def make_capsules(arm, n_caps: int, seed: int, length: float = 0.75, r=(0.03, 0.08)) -> np.ndarray:
    """Obstacle capsules [n_caps][7] = (segment end p0, segment end p1,
    radius): 0.75 m segments (the cluttered workspace of the paper's
    experiments) centred 0.25-0.8 of the reach from the base, z >= 0, random
    direction, radius U[r]; redrawn when the segment comes within 0.15 m of
    the base column."""
    rng = np.random.default_rng([seed, 5])
    R = reach(arm)
    col_r = 0.15 + abs(arm["a"][1])
    col_h = float(arm["d"][0]) + 0.1
    out = []
    while len(out) < n_caps:
        rad = rng.uniform(*r)
        dist = rng.uniform(0.25 * R, 0.8 * R)
        v = rng.normal(size=3)
        v[2] = abs(v[2])
        v /= np.linalg.norm(v)
        c = dist * v
        d = rng.normal(size=3)
        d *= 0.5 * length / np.linalg.norm(d)
        p0, p1 = c - d, c + d
        pts = np.linspace(p0, p1, 16)
        if np.any((np.hypot(pts[:, 0], pts[:, 1]) < col_r + rad) & (pts[:, 2] < col_h + rad)):
            continue
        out.append([*p0, *p1, rad])
    return _f32(np.asarray(out).reshape(n_caps, 7))


def self_pairs_apart(arm, gap: int = 2) -> np.ndarray:
    """Sphere pairs on links at least `gap` apart [n][2] (neighbouring links
    always touch at their joint); a caller prunes these further offline."""
    link = np.asarray(arm["sph_link"])
    return np.array([(a, b) for a in range(len(link)) for b in range(a + 1, len(link))
                     if abs(int(link[b]) - int(link[a])) >= gap], np.int32).reshape(-1, 2)


# ---------------------------------------------------------------------------
# Benchmark shapes
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Shape:
    name: str
    n_nodes: int
    batch: int
    k: int
    n_t: int
    t_min: float
    t_max: float
    samples: int
    n_obs: int
    goal_frac: float
    obs_r: tuple = (0.05, 0.15)
    w_max: float = 300.0


CONFIGS = {
    # plain method, tiny: 256-node tree, 64 uniform candidates, k=4,
    # 32 durations over 0.02-1.0 s, 16 samples, no obstacles
    "tiny": Shape("tiny", 256, 64, 4, 32, 0.02, 1.0, 16, 0, 0.0),
    # one planning iteration: 16,384 nodes, 4,096 candidates (half goal),
    # k=8, 64 durations x 32 samples, 5 obstacles
    "iteration": Shape("iteration", 16384, 4096, 8, 64, 0.02, 1.0, 32, 5, 0.5),
    # stress: 262,144 nodes, 65,536 candidates (30% goal), k=16,
    # 128 durations over 0.01-1.2 s x 64 samples, 20 obstacles
    "stress": Shape("stress", 262144, 65536, 16, 128, 0.01, 1.2, 64, 20, 0.3, (0.03, 0.2)),
}


def make_flight(seed: int, t_arrive=(0.4, 0.7), window: float = 0.25,
                launch_dist=(2.5, 3.5), g: float = 9.81):
    """The tracked object's flight for the planner's outer loop (Eq. (1)): a
    ballistic arc from a launch point 2.5-3.5 m from the base, 1 m high,
    through a workspace point 0.35-0.7 m from the base and 0.2-0.8 m high,
    reached at t* ~ U[t_arrive]; the object counts as within reach for
    [t* - window, t* + window] (t_enter, t_fall).  Values rounded to FP32."""
    rng = np.random.default_rng([seed, 7])
    az = rng.uniform(0, 2 * math.pi)
    rad = rng.uniform(0.35, 0.7)
    target = np.array([rad * math.cos(az), rad * math.sin(az), rng.uniform(0.2, 0.8)])
    la = az + rng.uniform(-0.6, 0.6)
    dist = rng.uniform(*launch_dist)
    x0 = np.array([dist * math.cos(la), dist * math.sin(la), 1.0])
    gv = np.array([0.0, 0.0, -g])
    ts = rng.uniform(*t_arrive)
    v0 = (target - x0 - 0.5 * gv * ts * ts) / ts
    return dict(x0=_f32(x0), v0=_f32(v0), g=_f32(gv), t_enter=float(np.float32(ts - window)),
                t_fall=float(np.float32(ts + window)), target=_f32(target), t_star=float(ts))


def goal_parents(cand, tau: float = 0.1, every: int = 2):
    """Tree nodes that reach every `every`-th goal candidate at constant
    velocity in tau seconds: state (q_g - qd_g tau, qd_g) with time-to-come
    t_req - tau.  Uniform tree nodes almost never reach a goal state within
    the limits; these let the goal branch, its attachment and its score take
    part.  Returns (states [m][14], times [m])."""
    g = np.nonzero(np.asarray(cand["kind"]) == KIND_GOAL)[0][::every]
    xg = np.asarray(cand["x"], np.float64)[g]
    x = np.concatenate([xg[:, :DOF] - xg[:, DOF:] * tau, xg[:, DOF:]], 1)
    t = np.asarray(cand["t_req"], np.float32)[g] - np.float32(tau)
    return _f32(x), _f32(t)


def make_rounds(arm, n_rounds: int, batch: int, goal_frac: float, seed: int, root=None,
                flight=None, goal_spread=None):
    """Candidates of every round of a planning cycle, each round drawn with
    its own seed (seed * 100 + round); free samples on the chord from `root`
    to the round's goals when a root is given; goal arrival times within the
    flight's [t_enter, t_fall] when a flight is given."""
    t_arr = (0.2, 0.8) if flight is None else (flight["t_enter"], flight["t_fall"])
    return [make_candidates(arm, batch, goal_frac, seed * 100 + r, root=root, t_arr=t_arr,
                            goal_spread=goal_spread)
            for r in range(n_rounds)]


def blade_midpoint(arm) -> np.ndarray:
    """The middle of the 0.30 m blade edge in the last link's frame (the
    blade point p_n that pruning reaches for)."""
    return _f32(arm["blade_base"] + 0.5 * arm["blade_len"] * arm["blade_dir"])


def make_cycle_problem(arm, seed: int, n_tree: int, batch: int, k: int = 8, rounds: int = 4,
                       n_obs: int = 2, n_t: int = 32, samples: int = 16,
                       launch_dist=(1.0, 1.6), with_goal_parents: bool = True,
                       root_at_rest: bool = False, goal_spread=None):
    """One planning problem for the anytime loop: a tree of a root (node 0,
    time 0), n_tree - 1 uniform nodes and (unless with_goal_parents is
    False) goal-reaching nodes for every other goal of every round; `rounds`
    candidate rounds of `batch` (half goals arriving within the flight's
    reach window, free samples on the chord from the root); the object's
    flight (launched 1.0-1.6 m from the base by default, so that part of the
    tree can reach it).  root_at_rest: the root waits at rest at a pose within
    +-1 rad of the joint-range centre; goal_spread: goal poses within that
    many rad of the root's."""
    sh = Shape(f"cycle{seed}", n_tree, batch, k, n_t, 0.02, 1.0, samples, n_obs, 0.5)
    wl = make_workload(sh, seed, arm=arm)
    flight = make_flight(seed, launch_dist=launch_dist)
    if root_at_rest:
        rq = np.random.default_rng([seed, 11]).uniform(-1.0, 1.0, DOF)
        wl["tree_x"][0] = _f32(np.concatenate([rq, np.zeros(DOF)]))
    rs = make_rounds(arm, rounds, batch, 0.5, seed, root=wl["tree_x"][0], flight=flight,
                     goal_spread=goal_spread)
    gx, gt = zip(*[goal_parents(c) for c in rs]) if with_goal_parents else ((), ())
    tree_x = np.concatenate([wl["tree_x"]] + list(gx))
    tree_t = np.concatenate([wl["tree_t"]] + list(gt))
    tree_t[0] = 0.0
    return dict(shape=sh, grid=wl["grid"], obs=wl["obs"], samples=samples, k=k, rounds=rs,
                tree_x=tree_x, tree_t=_f32(tree_t), flight=flight)


def make_workload(shape: Shape, seed: int, arm_seed: int = 0, arm=None):
    """Complete seeded input set for one shape."""
    arm = make_arm(arm_seed, w_max=shape.w_max) if arm is None else arm
    tree_x, tree_t = make_tree(arm, shape.n_nodes, seed)
    cand = make_candidates(arm, shape.batch, shape.goal_frac, seed)
    obs = make_obstacles(arm, shape.n_obs, seed, shape.obs_r)
    grid = t_grid(shape.n_t, shape.t_min, shape.t_max)
    return dict(shape=shape, arm=arm, tree_x=tree_x, tree_t=tree_t, cand=cand,
                obs=obs, grid=grid, samples=shape.samples, k=shape.k)


def make_problem_set(n_problems: int, seed: int, arm_seed: int = 0,
                     nodes=(1024, 65536), batch=(256, 8192), k: int = 8,
                     n_t: int = 64, samples: int = 32, max_obs: int = 5,
                     goal_frac: float = 0.5):
    """Many independent planning problems of uneven size: tree sizes and
    batch sizes log-uniform in the given ranges, 0..max_obs obstacles."""
    rng = np.random.default_rng([seed, 4])
    arm = make_arm(arm_seed)
    probs = []
    for p in range(n_problems):
        nn = int(round(math.exp(rng.uniform(math.log(nodes[0]), math.log(nodes[1])))))
        bb = int(round(math.exp(rng.uniform(math.log(batch[0]), math.log(batch[1])))))
        no = int(rng.integers(0, max_obs + 1))
        sh = Shape(f"p{p}", nn, bb, k, n_t, 0.02, 1.0, samples, no, goal_frac)
        probs.append(make_workload(sh, seed * 1000 + p, arm=arm))
    return arm, probs
