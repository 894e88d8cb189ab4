"""FP64 CPU oracle of the edge-timing path (Python side).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg use it to check the GPU library.  The product package never
imports it.  It loads ``liboracle.so`` built from ``oracle.c`` (plain C,
binary64, no contraction) and holds the numpy FP64 MLP oracle in ``mlp.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")
_lock = threading.Lock()
_lib = None

OJ = 8
OSPH = 64

T_RIGID, T_ARMATURE, T_FRICTION, T_GRAVITY = 1, 2, 4, 8
T_ALL = T_RIGID | T_ARMATURE | T_FRICTION | T_GRAVITY

S_NONE, S_VEL, S_POS, S_COLL, S_BAD, S_NOPARENT, S_SELF = 1, 2, 4, 8, 128, 512, 1024
DECISION_BITS = S_NONE | S_VEL | S_POS | S_COLL | S_BAD | S_NOPARENT


def build(force: bool = False) -> str:
    """Compile liboracle.so (gcc, -O2, no contraction, no fast-math)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                               "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class OArm(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("terms", C.c_int32),
        ("alpha", C.c_double * OJ), ("a", C.c_double * OJ), ("d", C.c_double * OJ),
        ("m", C.c_double * OJ), ("rc", (C.c_double * 3) * OJ), ("I", (C.c_double * 3) * OJ),
        ("Im", C.c_double * OJ), ("psi1", C.c_double * OJ), ("psi2", C.c_double * OJ),
        ("psi3", C.c_double * OJ),
        ("qmin", C.c_double * OJ), ("qmax", C.c_double * OJ), ("qdmax", C.c_double * OJ),
        ("taumax", C.c_double * OJ), ("acc", C.c_double * OJ),
        ("wmax", C.c_double), ("g", C.c_double * 3), ("tool", C.c_double * 3),
        ("nsph", C.c_int32), ("sph_link", C.c_int32 * OSPH), ("sph", (C.c_double * 4) * OSPH),
    ]


class OWorld(C.Structure):
    _fields_ = [
        ("sph", C.POINTER(C.c_double)), ("n_sph", C.c_int32),
        ("cap", C.POINTER(C.c_double)), ("n_cap", C.c_int32),
        ("margin", C.c_double),
        ("pairs", C.POINTER(C.c_int32)), ("n_pairs", C.c_int32),
        ("margin_self", C.c_double),
    ]


def make_world(obs=None, caps=None, pairs=None, margin=0.0, margin_self=0.0):
    """The oracle's world: obstacle spheres [n][4], obstacle capsules [m][7]
    = (p0, p1, radius), the clearance margin, and the arm's self-collision
    sphere pairs [p][2] with their margin (fixed-duration check only).
    Returns (struct, arrays to keep alive while it is used)."""
    W = OWorld()
    keep = []
    o = np.zeros((0, 4)) if obs is None else np.ascontiguousarray(obs, np.float64).reshape(-1, 4)
    c = np.zeros((0, 7)) if caps is None else np.ascontiguousarray(caps, np.float64).reshape(-1, 7)
    p = np.zeros((0, 2), np.int32) if pairs is None else \
        np.ascontiguousarray(pairs, np.int32).reshape(-1, 2)
    o, c, p = (np.ascontiguousarray(a) for a in (o, c, p))
    keep += [o, c, p]
    W.sph = o.ctypes.data_as(C.POINTER(C.c_double))
    W.n_sph = len(o)
    W.cap = c.ctypes.data_as(C.POINTER(C.c_double))
    W.n_cap = len(c)
    W.margin = float(margin)
    W.pairs = p.ctypes.data_as(C.POINTER(C.c_int32))
    W.n_pairs = len(p)
    W.margin_self = float(margin_self)
    return W, keep


class ORisk(C.Structure):
    _fields_ = [
        ("gz", C.c_double), ("sigma_mode", C.c_int32),
        ("sp", C.c_double), ("sv", C.c_double), ("sa", C.c_double),
        ("s0", C.c_double), ("s1", C.c_double),
        ("wv", C.c_double), ("vtarget", C.c_double), ("wp", C.c_double), ("wr", C.c_double),
        ("wx", C.c_double), ("r", C.c_double), ("nu0", C.c_double), ("lam", C.c_double),
    ]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(_SO)
            dp = C.POINTER(C.c_double)
            ip = C.POINTER(C.c_int32)
            sp = C.POINTER(C.c_int16)
            up = C.POINTER(C.c_uint16)
            ap = C.POINTER(OArm)
            L.oracle_cubic.argtypes = [C.c_int, dp, dp, C.c_double, C.c_double, dp, dp, dp]
            L.oracle_friction.argtypes = [C.c_double] * 4
            L.oracle_friction.restype = C.c_double
            L.oracle_rnea.argtypes = [ap, dp, dp, dp, dp]
            L.oracle_fk_spheres.argtypes = [ap, dp, dp]
            L.oracle_fk_point.argtypes = [ap, C.c_int, dp, C.c_int, C.c_int, dp, dp]
            L.oracle_slot_rho.argtypes = [ap, dp, dp, C.c_double, C.c_int, dp, dp, dp]
            L.oracle_rho_v.argtypes = [ap, dp, dp, C.c_double]
            L.oracle_rho_v.restype = C.c_double
            L.oracle_rho_q.argtypes = [ap, dp, dp, C.c_double]
            L.oracle_rho_q.restype = C.c_double
            wp = C.POINTER(OWorld)
            L.oracle_rho_c.argtypes = [ap, dp, dp, C.c_double, C.c_int, wp]
            L.oracle_rho_c.restype = C.c_double
            L.oracle_rho_self.argtypes = [ap, dp, dp, C.c_double, C.c_int, wp]
            L.oracle_rho_self.restype = C.c_double
            L.oracle_point_segment.argtypes = [dp, dp, dp]
            L.oracle_point_segment.restype = C.c_double
            L.oracle_edge_time.argtypes = [ap, C.c_int, dp, dp, ip, C.c_int, dp, C.c_int, sp, wp,
                                           C.c_int, sp, up, dp, dp, ip]
            L.oracle_edge_dense.argtypes = [ap, C.c_int, dp, dp, C.c_int, dp, C.c_int, dp]
            L.oracle_edge_nary.argtypes = [ap, C.c_int, dp, dp, C.c_int, dp, C.c_int, C.c_int, sp]
            L.oracle_edge_check.argtypes = [ap, C.c_int, dp, dp, dp, C.c_int, wp, up, dp, dp]
            L.oracle_edge_refine.argtypes = [ap, C.c_int, dp, dp, sp, C.c_int, dp, C.c_int,
                                             C.c_int, C.c_double, wp, dp, dp, up, dp, ip]
            L.oracle_control.argtypes = [ap, C.c_int, dp, dp, dp, dp, dp, dp, C.c_double, dp,
                                         dp, dp, up]
            L.oracle_plan_knn.argtypes = [C.c_int, dp, C.c_int, dp, C.c_int, C.c_int, ip, dp]
            L.oracle_log_phi.argtypes = [C.c_double]
            L.oracle_log_phi.restype = C.c_double
            L.oracle_risk_score.argtypes = [C.POINTER(ORisk), C.c_int, dp, dp, dp, dp, dp, dp]
            _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def make_oarm(arm, terms: int = T_ALL) -> OArm:
    """Pack a workload arm dict into the oracle's own struct."""
    A = OArm()
    n = int(arm["n"])
    A.n = n
    A.terms = terms
    for i in range(n):
        A.alpha[i] = float(arm["alpha"][i])
        A.a[i] = float(arm["a"][i])
        A.d[i] = float(arm["d"][i])
        A.m[i] = float(arm["m"][i])
        for r in range(3):
            A.rc[i][r] = float(arm["rc"][i][r])
            A.I[i][r] = float(arm["I"][i][r])
        for key in ("Im", "psi1", "psi2", "psi3", "qmin", "qmax", "qdmax", "taumax", "acc"):
            getattr(A, key)[i] = float(arm[key][i])
    A.wmax = float(arm["wmax"])
    for r in range(3):
        A.g[r] = float(arm["g"][r])
        A.tool[r] = float(arm["tool"][r])
    ns = len(arm["sph_link"])
    assert ns <= OSPH
    A.nsph = ns
    for k in range(ns):
        A.sph_link[k] = int(arm["sph_link"][k])
        for r in range(4):
            A.sph[k][r] = float(arm["sph"][k][r])
    return A


# ---------------------------------------------------------------------------
# thin wrappers
# ---------------------------------------------------------------------------

def cubic(x0, x1, T, t):
    n = len(x0) // 2
    x0, p0 = _d(x0)
    x1, p1 = _d(x1)
    s, sd, sdd = (np.zeros(n) for _ in range(3))
    lib().oracle_cubic(n, p0, p1, float(T), float(t), _p(s, C.c_double), _p(sd, C.c_double),
                       _p(sdd, C.c_double))
    return s, sd, sdd


def friction(psi1, psi2, psi3, qd):
    return lib().oracle_friction(float(psi1), float(psi2), float(psi3), float(qd))


def rnea(A: OArm, q, qd, qdd):
    q, pq = _d(q)
    qd, pqd = _d(qd)
    qdd, pqdd = _d(qdd)
    tau = np.zeros(A.n)
    lib().oracle_rnea(C.byref(A), pq, pqd, pqdd, _p(tau, C.c_double))
    return tau


def fk_spheres(A: OArm, q):
    q, pq = _d(q)
    c = np.zeros((A.nsph, 3))
    lib().oracle_fk_spheres(C.byref(A), pq, _p(c, C.c_double))
    return c


def fk_point(A: OArm, X, local, link=None):
    """World position of the point `local` of link `link` (default: the last
    link) for the configurations X[:, :n] (rows may carry velocities too)."""
    X, pX = _d(np.atleast_2d(X))
    local, pl = _d(local)
    out = np.zeros((X.shape[0], 3))
    lib().oracle_fk_point(C.byref(A), X.shape[0], pX, X.shape[1], int(A.n if link is None else link),
                          pl, _p(out, C.c_double))
    return out


def slot_rho(A: OArm, x0, x1, T, S, want_tau=False):
    x0, p0 = _d(x0)
    x1, p1 = _d(x1)
    rt, rp = C.c_double(), C.c_double()
    tau = np.zeros((S, A.n)) if want_tau else None
    lib().oracle_slot_rho(C.byref(A), p0, p1, float(T), int(S), C.byref(rt), C.byref(rp),
                          _p(tau, C.c_double) if want_tau else None)
    return (rt.value, rp.value, tau) if want_tau else (rt.value, rp.value)


def rho_v(A, x0, x1, T):
    x0, p0 = _d(x0)
    x1, p1 = _d(x1)
    return lib().oracle_rho_v(C.byref(A), p0, p1, float(T))


def rho_q(A, x0, x1, T):
    x0, p0 = _d(x0)
    x1, p1 = _d(x1)
    return lib().oracle_rho_q(C.byref(A), p0, p1, float(T))


def rho_c(A, x0, x1, T, S, obs=None, margin=0.0, caps=None):
    """Clearance ratio against obstacle spheres and capsules (Sec. IV-E)."""
    x0, p0 = _d(x0)
    x1, p1 = _d(x1)
    W, keep = make_world(obs, caps, None, margin)
    return lib().oracle_rho_c(C.byref(A), p0, p1, float(T), int(S), C.byref(W))


def rho_self(A, x0, x1, T, S, pairs, margin_self=0.0):
    """Clearance ratio of the arm's self-collision sphere pairs."""
    x0, p0 = _d(x0)
    x1, p1 = _d(x1)
    W, keep = make_world(None, None, pairs, 0.0, margin_self)
    return lib().oracle_rho_self(C.byref(A), p0, p1, float(T), int(S), C.byref(W))


def point_segment(c, p0, p1):
    c, pc = _d(c)
    p0, pa = _d(p0)
    p1, pb = _d(p1)
    return lib().oracle_point_segment(pc, pa, pb)


def edge_time(A: OArm, x0, x1, grid, S, obs=None, jmax=None, parent_ok=None, margin=0.0,
              scan=1, caps=None):
    """Plain search (Def. 7 on the grid) + post-checks for every edge.
    scan=1 stops at the first feasible slot, scan=0 evaluates every slot.
    rho[:, 3] (rho_c) is NaN where rho_v or rho_q already fails: Alg. 1
    and-s the clearance in after the limit checks."""
    x0, p0 = _d(x0)
    x1, p1 = _d(x1)
    E = x0.shape[0]
    grid, pg = _d(grid)
    W, keep = make_world(obs, caps, None, margin)
    out_j = np.zeros(E, np.int16)
    out_st = np.zeros(E, np.uint16)
    out_m = np.zeros(E)
    out_rho = np.zeros((E, 4))
    out_ns = np.zeros(E, np.int32)
    jm = None if jmax is None else np.ascontiguousarray(jmax, np.int16)
    pok = None if parent_ok is None else np.ascontiguousarray(parent_ok, np.int32)
    lib().oracle_edge_time(C.byref(A), E, p0, p1, None if pok is None else _p(pok, C.c_int32),
                           len(grid), pg, int(S), None if jm is None else _p(jm, C.c_int16),
                           C.byref(W), int(scan), _p(out_j, C.c_int16),
                           _p(out_st, C.c_uint16), _p(out_m, C.c_double), _p(out_rho, C.c_double),
                           _p(out_ns, C.c_int32))
    return dict(j=out_j, status=out_st, margin=out_m, rho=out_rho, nslots=out_ns)


def edge_dense(A, x0, x1, grid, S):
    x0, p0 = _d(x0)
    x1, p1 = _d(x1)
    grid, pg = _d(grid)
    E = x0.shape[0]
    rho = np.zeros((E, len(grid), 2))
    lib().oracle_edge_dense(C.byref(A), E, p0, p1, len(grid), pg, int(S), _p(rho, C.c_double))
    return rho


def edge_nary(A, x0, x1, grid, S, N):
    x0, p0 = _d(x0)
    x1, p1 = _d(x1)
    grid, pg = _d(grid)
    E = x0.shape[0]
    out = np.zeros(E, np.int16)
    lib().oracle_edge_nary(C.byref(A), E, p0, p1, len(grid), pg, int(S), int(N),
                           _p(out, C.c_int16))
    return out


def edge_check(A, x0, x1, T, S, obs=None, margin=0.0, want_tau=False, caps=None, pairs=None,
               margin_self=0.0):
    """Fixed-duration check; rho[:, 4] is the larger of the obstacle and
    self-collision clearance ratios (S_SELF marks the self part > 1)."""
    x0, p0 = _d(x0)
    x1, p1 = _d(x1)
    T, pT = _d(T)
    E = x0.shape[0]
    W, keep = make_world(obs, caps, pairs, margin, margin_self)
    st = np.zeros(E, np.uint16)
    rho = np.zeros((E, 5))
    tau = np.zeros((E, S, A.n)) if want_tau else None
    lib().oracle_edge_check(C.byref(A), E, p0, p1, pT, int(S), C.byref(W),
                            _p(st, C.c_uint16), _p(rho, C.c_double),
                            _p(tau, C.c_double) if want_tau else None)
    return dict(status=st, rho=rho, tau=tau)


def edge_refine(A, x0, x1, j, grid, S, N, eps, obs=None, margin=0.0, caps=None):
    """N-ary refinement below the grid result j of every edge (Sec. IV-D):
    returns T, the final lower end lo, status, rho4 = (rho_tauP(T), rho_v,
    rho_q, rho_c) and the rounds run."""
    x0, p0 = _d(x0)
    x1, p1 = _d(x1)
    grid, pg = _d(grid)
    E = x0.shape[0]
    jj = np.ascontiguousarray(j, np.int16)
    W, keep = make_world(obs, caps, None, margin)
    T, lo = np.zeros(E), np.zeros(E)
    st = np.zeros(E, np.uint16)
    rho = np.zeros((E, 4))
    rounds = np.zeros(E, np.int32)
    lib().oracle_edge_refine(C.byref(A), E, p0, p1, _p(jj, C.c_int16), len(grid), pg, int(S),
                             int(N), float(eps), C.byref(W), _p(T, C.c_double),
                             _p(lo, C.c_double), _p(st, C.c_uint16), _p(rho, C.c_double),
                             _p(rounds, C.c_int32))
    return dict(T=T, lo=lo, status=st, rho=rho, rounds=rounds)


C_ACC, C_SLEW, C_TORQUE, C_POWER, C_BAD = 1, 2, 4, 8, 128


def control(A, q, qd, tau_prev, qg, qdg, T, dt, slew):
    """One step of the tracking controller of Eq. (9) per instance: returns
    (tau [n][dof], clipped qdd [n][dof], status [n])."""
    arrs = [_d(np.atleast_2d(x)) for x in (q, qd, tau_prev, qg, qdg)]
    n = arrs[0][0].shape[0]
    T, pT = _d(np.broadcast_to(np.asarray(T, np.float64), (n,)))
    slew, ps = _d(slew)
    tau = np.zeros((n, A.n))
    qdd = np.zeros((n, A.n))
    st = np.zeros(n, np.uint16)
    lib().oracle_control(C.byref(A), n, *[p for _, p in arrs], pT, float(dt), ps,
                         _p(tau, C.c_double), _p(qdd, C.c_double), _p(st, C.c_uint16))
    return tau, qdd, st


def plan_knn(nodes, queries, k):
    nodes, pn = _d(nodes)
    queries, pq = _d(queries)
    N, dim = nodes.shape
    B = queries.shape[0]
    idx = np.zeros((B, k), np.int32)
    d2 = np.zeros((B, k))
    lib().oracle_plan_knn(N, pn, B, pq, dim, int(k), _p(idx, C.c_int32), _p(d2, C.c_double))
    return idx, d2


def log_phi(z):
    return lib().oracle_log_phi(float(z))


PAPER_RISK = dict(wv=0.20, vtarget=9.0, wp=8.0, wr=8.0, wx=1.0, r=0.09, nu0=0.90, lam=1.2)


def make_orisk(gz=-9.81, sigma_mode=0, sp=0.0048, sv=0.0186, sa=0.0, s0=0.01, s1=0.05, **w):
    R = ORisk()
    R.gz, R.sigma_mode, R.sp, R.sv, R.sa, R.s0, R.s1 = gz, sigma_mode, sp, sv, sa, s0, s1
    ww = dict(PAPER_RISK)
    ww.update(w)
    for k, v in ww.items():
        setattr(R, k, v)
    return R


def risk_score(R: ORisk, T, v_rel, nu, vz0, t_fall):
    arrs = [_d(x) for x in (T, v_rel, nu, vz0, t_fall)]
    n = len(arrs[0][0])
    out = np.zeros(n)
    lib().oracle_risk_score(C.byref(R), n, *[p for _, p in arrs], _p(out, C.c_double))
    return out


def edges_of(tree_x, cand_x, nbr):
    """Edge endpoint arrays: x0[b*k+i] = tree node nbr[b][i], x1 = candidate b.
    Padded parents (-1) give a zero state and parent_ok = 0."""
    B, k = nbr.shape
    flat = nbr.reshape(-1)
    ok = (flat >= 0).astype(np.int32)
    x0 = np.asarray(tree_x, np.float64)[np.where(flat >= 0, flat, 0)]
    x0[flat < 0] = 0.0
    x1 = np.repeat(np.asarray(cand_x, np.float64), k, axis=0)
    return x0, x1, ok
