"""ctypes binding of libfruitninja.so (include/fruitninja.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch provides device memory and the current stream.  The
library must have been built (``python -m paper_2609_22608_amd.build``);
loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfruitninja.so")

FN_OK, FN_E_ARG, FN_E_SHAPE, FN_E_UNSUPPORTED, FN_E_HIP, FN_E_NOMEM, FN_E_STATE = 0, -1, -2, -3, -4, -5, -6
S_NONE, S_VEL, S_POS, S_COLL, S_RECHECK64, S_WIN_HIT, S_WIN_MISS, S_BAD_INPUT, S_WIN_BELOW, \
    S_NO_PARENT, S_SELF = 1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024
S_DECISION = S_NONE | S_VEL | S_POS | S_COLL | S_BAD_INPUT | S_NO_PARENT
T_RIGID, T_ARMATURE, T_FRICTION, T_GRAVITY, T_ALL = 1, 2, 4, 8, 15
SEARCH_PLAIN, SEARCH_SCREEN, SEARCH_WINDOW = 0, 1, 2
MAX_SPHERES = 64


class FnError(RuntimeError):
    pass


class ArmDesc(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("terms", C.c_int32),
        ("alpha", C.c_double * 7), ("a", C.c_double * 7), ("d", C.c_double * 7),
        ("m", C.c_double * 7), ("rc", (C.c_double * 3) * 7), ("inertia", (C.c_double * 3) * 7),
        ("Im", C.c_double * 7), ("psi1", C.c_double * 7), ("psi2", C.c_double * 7),
        ("psi3", C.c_double * 7),
        ("qmin", C.c_double * 7), ("qmax", C.c_double * 7), ("qdmax", C.c_double * 7),
        ("taumax", C.c_double * 7), ("acc", C.c_double * 7),
        ("wmax", C.c_double), ("g", C.c_double * 3),
        ("n_spheres", C.c_int32), ("sphere_link", C.c_int32 * MAX_SPHERES),
        ("sphere", (C.c_double * 4) * MAX_SPHERES),
    ]


class Caps(C.Structure):
    _fields_ = [("max_nodes", C.c_int32), ("max_batch", C.c_int32), ("max_k", C.c_int32),
                ("max_edges", C.c_int64), ("max_problems", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("knn_target_waves", C.c_int32), ("knn_min_chunk", C.c_int32),
                ("knn_form", C.c_int32), ("edge_form", C.c_int32), ("mlp_rows", C.c_int32)]


class Search(C.Structure):
    _fields_ = [("grid", C.c_void_p), ("n_t", C.c_int32), ("samples", C.c_int32),
                ("mode", C.c_int32), ("win_half", C.c_int32), ("j_max", C.c_void_p),
                ("win_lo", C.c_void_p)]


class Obstacles(C.Structure):
    _fields_ = [("spheres", C.c_void_p), ("n", C.c_int32), ("margin", C.c_float),
                ("capsules", C.c_void_p), ("n_caps", C.c_int32)]


def obstacles(obs=None, margin=0.0, caps=None):
    """fn_obstacles of device tensors: spheres [n][4], capsules [m][7]."""
    return Obstacles(None if obs is None or obs.shape[0] == 0 else C.c_void_p(obs.data_ptr()),
                     0 if obs is None else obs.shape[0], float(margin),
                     None if caps is None or caps.shape[0] == 0 else C.c_void_p(caps.data_ptr()),
                     0 if caps is None else caps.shape[0])


class EdgeOut(C.Structure):
    _fields_ = [("j", C.c_void_p), ("status", C.c_void_p), ("margin", C.c_void_p),
                ("rho4", C.c_void_p), ("work", C.c_void_p), ("screened", C.c_void_p)]


class Refine(C.Structure):
    _fields_ = [("grid", C.c_void_p), ("n_t", C.c_int32), ("samples", C.c_int32),
                ("n_ary", C.c_int32), ("eps", C.c_float)]


class TrainCfg(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("cosine", C.c_int32), ("seed", C.c_uint64), ("grid", C.c_void_p),
                ("n_t", C.c_int32)]


class Risk(C.Structure):
    _fields_ = [("gz", C.c_double), ("sigma_mode", C.c_int32), ("sp", C.c_double),
                ("sv", C.c_double), ("sa", C.c_double), ("s0", C.c_double), ("s1", C.c_double),
                ("wv", C.c_double), ("vtarget", C.c_double), ("wp", C.c_double),
                ("wr", C.c_double), ("wx", C.c_double), ("r", C.c_double), ("nu0", C.c_double),
                ("lam", C.c_double)]


class Problem(C.Structure):
    _fields_ = [("tree", C.c_void_p), ("ld", C.c_int64), ("n_nodes", C.c_void_p),
                ("t_node", C.c_void_p), ("parent", C.c_void_p), ("nu", C.c_void_p),
                ("cand", C.c_void_p), ("kind", C.c_void_p), ("t_req", C.c_void_p),
                ("v_rel", C.c_void_p), ("vz0", C.c_void_p), ("t_fall", C.c_void_p),
                ("B", C.c_int32), ("obs", C.c_void_p), ("n_obs", C.c_int32), ("nbr", C.c_void_p),
                ("out_j", C.c_void_p), ("out_status", C.c_void_p), ("out_margin", C.c_void_p),
                ("out_rho4", C.c_void_p), ("out_T", C.c_void_p), ("out_node", C.c_void_p),
                ("out_J", C.c_void_p), ("out_best", C.c_void_p), ("caps", C.c_void_p),
                ("n_caps", C.c_int32), ("n_rounds", C.c_int32), ("incumbent", C.c_void_p),
                ("flight", C.c_void_p), ("out_reach", C.c_void_p)]


class Prune(C.Structure):
    _fields_ = [("v_tip", C.c_float), ("blade", C.c_float * 3)]


def make_prune(v_tip, blade):
    pr = Prune()
    pr.v_tip = float(v_tip)
    pr.blade[:] = [float(x) for x in blade]
    return pr


def flight_array(fl):
    """Device [11] flight of Eq. (1): x0, v0, g, t_enter, t_fall."""
    a = np.concatenate([np.asarray(fl["x0"], np.float32), np.asarray(fl["v0"], np.float32),
                        np.asarray(fl["g"], np.float32),
                        np.asarray([fl["t_enter"], fl["t_fall"]], np.float32)])
    return dev(a)


class ProblemSet(C.Structure):
    _fields_ = [("n_problems", C.c_int32), ("problems", C.POINTER(Problem)), ("k", C.c_int32),
                ("grid", C.c_void_p), ("n_t", C.c_int32), ("samples", C.c_int32),
                ("mode", C.c_int32), ("margin", C.c_float), ("risk", Risk)]


_lib = None
_lock = threading.Lock()


def lib():
    """Loads libfruitninja.so; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise FnError(f"{LIB_PATH} is missing: build it first "
                              "(python -m paper_2609_22608_amd.build)")
            L = C.CDLL(LIB_PATH)
            vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
            L.fn_last_error.restype = C.c_char_p
            L.fn_version.restype = C.c_char_p
            L.fn_create.argtypes = [C.POINTER(ArmDesc), C.POINTER(Caps), C.POINTER(vp)]
            L.fn_destroy.argtypes = [vp]
            L.plan_knn.argtypes = [vp, vp, i64, i32, vp, i32, i32, vp, vp, vp]
            L.edge_time_batch.argtypes = [vp, vp, i64, i32, vp, i32, vp, i32, C.POINTER(Search),
                                          C.POINTER(Obstacles), C.POINTER(EdgeOut), vp]
            L.edge_time_batch_noalloc.argtypes = L.edge_time_batch.argtypes
            L.fn_noalloc_scratch_bytes.restype = C.c_size_t
            L.edge_check.argtypes = [vp, vp, vp, vp, i64, i32, C.POINTER(Obstacles), vp, vp, vp, vp]
            L.fn_set_self_pairs.argtypes = [vp, vp, i32, C.c_float]
            L.fn_control.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, C.c_float,
                                     C.POINTER(C.c_double), vp, vp, vp, vp]
            L.edge_refine.argtypes = [vp, vp, i64, i32, vp, i32, vp, i32, vp, C.POINTER(Refine),
                                      C.POINTER(Obstacles), vp, vp, vp, vp, vp, vp]
            L.risk_score.argtypes = [vp, C.POINTER(Risk), vp, vp, vp, vp, vp, i32, vp, vp]
            L.fn_mlp_create.argtypes = [vp, C.c_uint64, C.POINTER(vp)]
            L.fn_mlp_destroy.argtypes = [vp]
            L.fn_mlp_param_count.restype = C.c_int
            L.fn_mlp_set_params.argtypes = [vp, vp, i64]
            L.fn_mlp_get_params.argtypes = [vp, vp, i64]
            L.fn_mlp_save.argtypes = [vp, C.c_char_p]
            L.fn_mlp_load.argtypes = [vp, C.c_char_p, C.POINTER(vp)]
            L.edge_features.argtypes = [vp, vp, i64, i32, vp, i32, vp, i32, vp, vp]
            L.surrogate_train.argtypes = [vp, vp, vp, vp, i64, C.POINTER(TrainCfg), vp, vp]
            L.surrogate_grad.argtypes = [vp, vp, vp, vp, i32, vp, i32, vp, vp, vp]
            L.surrogate_infer.argtypes = [vp, vp, vp, i64, vp, i32, i32, C.c_float, vp, vp, vp]
            L.surrogate_window.argtypes = [vp, vp, vp, i64, i32, vp, i32, vp, i32, vp, i32, i32,
                                           C.c_float, vp, vp, vp]
            L.fn_set_tuning.argtypes = [vp, C.POINTER(Tuning)]
            L.fn_batch_prepare.argtypes = [vp, C.POINTER(ProblemSet)]
            L.fn_batch_launch.argtypes = [vp, vp]
            L.fn_graph_capture.argtypes = [vp, vp]
            L.fn_graph_launch.argtypes = [vp, vp]
            L.fn_batch_round.argtypes = [vp, i32, vp]
            L.fn_batch_prune.argtypes = [vp, C.POINTER(Prune), vp]
            L.fn_cycle.argtypes = [vp, i32, i32, C.POINTER(Prune), vp]
            L.fn_graph_capture_cycle.argtypes = [vp, i32, i32, C.POINTER(Prune), vp]
            L.fn_reach_time.argtypes = [vp, vp, i64, i32, vp, vp, C.POINTER(Prune), vp, vp]
            L.fn_kernel_timing.argtypes = [vp, C.c_int]
            L.fn_kernel_times.argtypes = [vp, vp, i32, C.POINTER(i32)]
            _lib = L
    return _lib


def _check(rc, what):
    if rc != FN_OK:
        raise FnError(f"{what} failed ({rc}): {lib().fn_last_error().decode()}")


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def arm_desc(arm, terms: int = T_ALL) -> ArmDesc:
    """Packs a workload arm dict into the library's fn_arm_desc."""
    d = ArmDesc()
    d.n = int(arm["n"])
    d.terms = terms
    for i in range(7):
        d.alpha[i] = float(arm["alpha"][i])
        d.a[i] = float(arm["a"][i])
        d.d[i] = float(arm["d"][i])
        d.m[i] = float(arm["m"][i])
        for r in range(3):
            d.rc[i][r] = float(arm["rc"][i][r])
            d.inertia[i][r] = float(arm["I"][i][r])
        for key in ("Im", "psi1", "psi2", "psi3", "qmin", "qmax", "qdmax", "taumax", "acc"):
            getattr(d, key)[i] = float(arm[key][i])
    d.wmax = float(arm["wmax"])
    for r in range(3):
        d.g[r] = float(arm["g"][r])
    ns = len(arm["sph_link"])
    if ns > MAX_SPHERES:
        raise FnError(f"{ns} spheres (max {MAX_SPHERES})")
    d.n_spheres = ns
    for k in range(ns):
        d.sphere_link[k] = int(arm["sph_link"][k])
        for r in range(4):
            d.sphere[k][r] = float(arm["sph"][k][r])
    return d


def version() -> str:
    return lib().fn_version().decode()


def tree_soa(states, device="cuda", capacity=None):
    """Structure-of-arrays device copy of tree states [n][14] -> [14][ld]
    (ld a multiple of 4, padding zero).  Returns (tensor, ld, n)."""
    x = np.asarray(states, np.float32)
    n = x.shape[0]
    cap = max(n, capacity or 0)
    ld = max(4, (cap + 3) // 4 * 4)
    soa = np.zeros((14, ld), np.float32)
    soa[:, :n] = x.T
    return torch.from_numpy(soa).to(device), ld, n


def dev(x, dtype=torch.float32, device="cuda"):
    return torch.as_tensor(np.ascontiguousarray(x)).to(device=device, dtype=dtype).contiguous()


class Context:
    """An fn_ctx on the current device."""

    def __init__(self, arm, max_nodes, max_batch, max_k, max_edges=None, terms: int = T_ALL,
                 max_problems: int = 0):
        torch.cuda.init()
        self._desc = arm_desc(arm, terms)
        caps = Caps(int(max_nodes), int(max_batch), int(max_k),
                    int(max_edges if max_edges is not None else max_batch * max_k),
                    int(max_problems))
        self.caps = caps
        h = C.c_void_p()
        _check(lib().fn_create(C.byref(self._desc), C.byref(caps), C.byref(h)), "fn_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().fn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def kernel_timing(self, enable=True):
        """Event pairs around the search kernel of later edge_time_batch calls."""
        _check(lib().fn_kernel_timing(self.h, int(bool(enable))), "fn_kernel_timing")

    def kernel_times(self, max_n=256):
        """Elapsed ms of the timed search kernels since the last call (waits)."""
        buf = (C.c_float * max_n)()
        n = C.c_int32(0)
        _check(lib().fn_kernel_times(self.h, buf, max_n, C.byref(n)), "fn_kernel_times")
        return [buf[i] for i in range(n.value)]

    def set_tuning(self, knn_target_waves=None, knn_min_chunk=None, knn_form=None,
                   edge_form=None, mlp_rows=None):
        """Launch mappings (fn_set_tuning); a field left None keeps its current
        value (0, the library default, before the first call)."""
        cur = getattr(self, "_tuning", (0, 0, 0, 0, 0))
        new = tuple(c if v is None else int(v) for c, v in
                    zip(cur, (knn_target_waves, knn_min_chunk, knn_form, edge_form, mlp_rows)))
        t = Tuning(*new)
        _check(lib().fn_set_tuning(self.h, C.byref(t)), "fn_set_tuning")
        self._tuning = new
        self.tuned_knn_form = new[2]
        self.edge_form = new[3]
        self.mlp_rows = new[4]

    # -- plan_knn -----------------------------------------------------------
    def plan_knn(self, tree, ld, n_nodes, queries, k, out_idx=None, out_d2=None, want_d2=True):
        B = queries.shape[0]
        if out_idx is None:
            out_idx = torch.empty((B, k), dtype=torch.int32, device=queries.device)
        if out_d2 is None and want_d2:
            out_d2 = torch.empty((B, k), dtype=torch.float32, device=queries.device)
        _check(lib().plan_knn(self.h, _ptr(tree), ld, n_nodes, _ptr(queries), B, k,
                              _ptr(out_idx), _ptr(out_d2), _stream()), "plan_knn")
        return out_idx, out_d2

    # -- edge_time_batch ------------------------------------------------------
    def edge_time_batch(self, tree, ld, n_nodes, cand, nbr, grid, samples, obs=None,
                        margin=0.0, mode=SEARCH_PLAIN, j_max=None, win_lo=None, win_half=4,
                        out=None, want_rho=True, want_work=True, noalloc=False, caps=None):
        """edge_time_batch, or edge_time_batch_noalloc when noalloc is set."""
        B, k = nbr.shape
        E = B * k
        d = cand.device
        if out is None:
            out = dict(j=torch.empty(E, dtype=torch.int16, device=d),
                       status=torch.empty(E, dtype=torch.int16, device=d),
                       margin=torch.empty(E, dtype=torch.float32, device=d),
                       rho=torch.empty((E, 4), dtype=torch.float32, device=d) if want_rho else None,
                       work=torch.empty(E, dtype=torch.int32, device=d) if want_work else None,
                       screened=torch.empty(E, dtype=torch.int16, device=d) if want_work else None)
        s = Search(C.c_void_p(grid.data_ptr()), grid.shape[0], int(samples), int(mode),
                   int(win_half), None if j_max is None else C.c_void_p(j_max.data_ptr()),
                   None if win_lo is None else C.c_void_p(win_lo.data_ptr()))
        o = obstacles(obs, margin, caps)
        eo = EdgeOut(out["j"].data_ptr(), out["status"].data_ptr(), out["margin"].data_ptr(),
                     None if out["rho"] is None else out["rho"].data_ptr(),
                     None if out["work"] is None else out["work"].data_ptr(),
                     None if out.get("screened") is None else out["screened"].data_ptr())
        call = lib().edge_time_batch_noalloc if noalloc else lib().edge_time_batch
        _check(call(self.h, _ptr(tree), ld, n_nodes, _ptr(cand), B, _ptr(nbr), k, C.byref(s),
                    C.byref(o), C.byref(eo), _stream()),
               "edge_time_batch_noalloc" if noalloc else "edge_time_batch")
        return out

    def set_self_pairs(self, pairs, margin=0.0):
        """Self-collision sphere pairs [n][2] of the arm for edge_check."""
        a = np.ascontiguousarray(np.asarray(pairs, np.int32).reshape(-1, 2))
        _check(lib().fn_set_self_pairs(self.h, a.ctypes.data_as(C.c_void_p), len(a),
                                       C.c_float(margin)), "fn_set_self_pairs")

    # -- edge_refine ----------------------------------------------------------
    def edge_refine(self, tree, ld, n_nodes, cand, nbr, j_in, grid, samples, n_ary=3, eps=1e-4,
                    obs=None, margin=0.0, caps=None):
        B, k = nbr.shape
        E = B * k
        d = cand.device
        out = dict(T=torch.empty(E, dtype=torch.float32, device=d),
                   status=torch.empty(E, dtype=torch.int16, device=d),
                   rho=torch.empty((E, 4), dtype=torch.float32, device=d),
                   rounds=torch.empty(E, dtype=torch.int32, device=d),
                   work=torch.empty(E, dtype=torch.int32, device=d))
        r = Refine(C.c_void_p(grid.data_ptr()), grid.shape[0], int(samples), int(n_ary),
                   float(eps))
        o = obstacles(obs, margin, caps)
        _check(lib().edge_refine(self.h, _ptr(tree), ld, n_nodes, _ptr(cand), B, _ptr(nbr), k,
                                 _ptr(j_in), C.byref(r), C.byref(o), _ptr(out["T"]),
                                 _ptr(out["status"]), _ptr(out["rho"]), _ptr(out["rounds"]),
                                 _ptr(out["work"]), _stream()), "edge_refine")
        return out

    # -- edge_check -----------------------------------------------------------
    def reach_time(self, tree, ld, n, t_node, flight, v_tip, blade):
        """Eq. (8)'s earliest reach time of the first n nodes of an SoA tree;
        flight: dict (x0, v0, g, t_enter, t_fall) or a device [11] tensor."""
        fl = flight if isinstance(flight, torch.Tensor) else flight_array(flight)
        out = torch.empty(max(int(n), 1), dtype=torch.float32, device="cuda")
        pr = make_prune(v_tip, blade)
        _check(lib().fn_reach_time(self.h, _ptr(tree), int(ld), int(n), _ptr(t_node), _ptr(fl),
                                   C.byref(pr), _ptr(out), _stream()), "fn_reach_time")
        return out[:n]

    def edge_check(self, x0, x1, T, samples, obs=None, margin=0.0, want_tau=False, caps=None):
        E = x0.shape[0]
        d = x0.device
        st = torch.empty(E, dtype=torch.int16, device=d)
        rho = torch.empty((E, 5), dtype=torch.float32, device=d)
        tau = torch.empty((E, samples, 7), dtype=torch.float32, device=d) if want_tau else None
        o = obstacles(obs, margin, caps)
        _check(lib().edge_check(self.h, _ptr(x0), _ptr(x1), _ptr(T), E, int(samples), C.byref(o),
                                _ptr(st), _ptr(rho), _ptr(tau), _stream()), "edge_check")
        return dict(status=st, rho=rho, tau=tau)

    # -- risk_score -----------------------------------------------------------
    def risk_score(self, w: Risk, T, v_rel, nu, vz0, t_fall, out=None):
        n = T.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=T.device)
        _check(lib().risk_score(self.h, C.byref(w), _ptr(T), _ptr(v_rel), _ptr(nu), _ptr(vz0),
                                _ptr(t_fall), n, _ptr(out), _stream()), "risk_score")
        return out


class Surrogate:
    """An fn_mlp (the learned T-window network) bound to a Context."""

    def __init__(self, ctx: Context, seed: int = 0, handle=None):
        self.ctx = ctx
        if handle is None:
            handle = C.c_void_p()
            _check(lib().fn_mlp_create(ctx.h, C.c_uint64(seed), C.byref(handle)), "fn_mlp_create")
        self.h = handle

    @classmethod
    def load(cls, ctx: Context, path: str):
        h = C.c_void_p()
        _check(lib().fn_mlp_load(ctx.h, path.encode(), C.byref(h)), "fn_mlp_load")
        return cls(ctx, handle=h)

    def save(self, path: str):
        torch.cuda.synchronize()
        _check(lib().fn_mlp_save(self.h, path.encode()), "fn_mlp_save")

    def close(self):
        if getattr(self, "h", None):
            lib().fn_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def param_count() -> int:
        return lib().fn_mlp_param_count()

    def set_params(self, flat):
        a = np.ascontiguousarray(flat, np.float32)
        _check(lib().fn_mlp_set_params(self.h, a.ctypes.data_as(C.c_void_p), a.size),
               "fn_mlp_set_params")

    def get_params(self):
        torch.cuda.synchronize()
        a = np.zeros(self.param_count(), np.float32)
        _check(lib().fn_mlp_get_params(self.h, a.ctypes.data_as(C.c_void_p), a.size),
               "fn_mlp_get_params")
        return a

    def grad(self, X, y_j, grid):
        g = torch.empty(self.param_count(), dtype=torch.float32, device=X.device)
        l3 = torch.empty(3, dtype=torch.float32, device=X.device)
        _check(lib().surrogate_grad(self.ctx.h, self.h, _ptr(X), _ptr(y_j), X.shape[0],
                                    _ptr(grid), grid.shape[0], _ptr(g), _ptr(l3), _stream()),
               "surrogate_grad")
        return g, l3

    def train(self, X, y_j, grid, epochs=20, batch=4096, lr=1e-3, beta1=0.9, beta2=0.999,
              eps=1e-8, cosine=True, seed=0):
        cfg = TrainCfg(int(epochs), int(batch), float(lr), float(beta1), float(beta2), float(eps),
                       int(bool(cosine)), int(seed), grid.data_ptr(), grid.shape[0])
        losses = torch.zeros((epochs, 3), dtype=torch.float32, device=X.device)
        _check(lib().surrogate_train(self.ctx.h, self.h, _ptr(X), _ptr(y_j), X.shape[0],
                                     C.byref(cfg), _ptr(losses), _stream()), "surrogate_train")
        return losses

    def window(self, tree, ld, n_nodes, cand, nbr, grid, half=4, logit_min=0.0, want_out=False,
               win_lo=None, out=None):
        """surrogate_window: the windows of every (candidate, parent) edge,
        with the feature rows gathered inside the inference kernel."""
        B, k = nbr.shape
        N = B * k
        if out is None and want_out:
            out = torch.empty((N, 2), dtype=torch.float32, device=cand.device)
        if win_lo is None:
            win_lo = torch.empty(N, dtype=torch.int16, device=cand.device)
        _check(lib().surrogate_window(self.ctx.h, self.h, _ptr(tree), int(ld), int(n_nodes),
                                      _ptr(cand), B, _ptr(nbr), k, _ptr(grid), grid.shape[0],
                                      int(half), float(logit_min), _ptr(out), _ptr(win_lo),
                                      _stream()), "surrogate_window")
        return out, win_lo

    def infer(self, X, grid, half=4, logit_min=0.0, want_out=True, win_lo=None, out=None):
        N = X.shape[0]
        if out is None and want_out:
            out = torch.empty((N, 2), dtype=torch.float32, device=X.device)
        if win_lo is None:
            win_lo = torch.empty(N, dtype=torch.int16, device=X.device)
        _check(lib().surrogate_infer(self.ctx.h, self.h, _ptr(X), N, _ptr(grid), grid.shape[0],
                                     int(half), float(logit_min), _ptr(out), _ptr(win_lo),
                                     _stream()), "surrogate_infer")
        return out, win_lo


class Batch:
    """A batched planning iteration over several problems (fn_problem_set).

    Each problem is a dict of device tensors; ``add_problem`` allocates them
    from host arrays.  ``prepare`` uploads the tables; ``launch`` enqueues one
    round; ``capture`` / ``replay`` use a HIP graph."""

    def __init__(self, ctx: Context, grid, samples, k, mode=SEARCH_SCREEN, margin=0.0, risk=None):
        self.ctx, self.grid, self.samples, self.k = ctx, grid, int(samples), int(k)
        self.mode, self.margin = int(mode), float(margin)
        self.risk = risk if risk is not None else make_risk(sigma_mode=1, s0=0.01, s1=0.05)
        self.problems = []

    def add_problem(self, tree_x, tree_t, cand, obs, capacity, flight=None, parent=None):
        """tree_x [n][14], tree_t [n], cand dict (x, kind, t_req, flight) or a
        list of such dicts (one per round, equal sizes), obs [m][4].  With a
        flight dict (x0, v0, g, t_enter, t_fall) the problem carries the
        anytime loop's incumbent (initial t_best = t_fall) and can be pruned;
        parent [n]: initial parents (default -1)."""
        d = "cuda"
        n = len(tree_x)
        tree, ld, _ = tree_soa(tree_x, capacity=capacity)
        rounds = cand if isinstance(cand, (list, tuple)) else [cand]
        B = len(rounds[0]["x"])
        assert all(len(c["x"]) == B for c in rounds)
        k = self.k
        t_node = torch.zeros(ld, dtype=torch.float32, device=d)
        t_node[:n] = torch.as_tensor(np.asarray(tree_t, np.float32))
        par0 = torch.full((ld,), -1, dtype=torch.int32, device=d)
        if parent is not None:
            par0[:n] = torch.as_tensor(np.asarray(parent, np.int32))

        def cat(f):
            return np.concatenate([f(c) for c in rounds])

        P = dict(tree=tree, ld=ld, n0=n, n_nodes=torch.tensor([n], dtype=torch.int32, device=d),
                 t_node=t_node, t_node0=t_node.clone(), tree0=tree.clone(),
                 parent=par0.clone(), parent0=par0,
                 nu=torch.zeros(ld, dtype=torch.float32, device=d),
                 cand=dev(cat(lambda c: c["x"])), kind=dev(cat(lambda c: c["kind"]), torch.int32),
                 t_req=dev(cat(lambda c: c["t_req"])),
                 v_rel=dev(cat(lambda c: c["flight"]["v_rel"])),
                 vz0=dev(cat(lambda c: np.asarray(c["flight"]["v0"])[:, 2])),
                 t_fall=dev(cat(lambda c: c["flight"]["t_fall"])), n_rounds=len(rounds),
                 B=B, obs=dev(obs) if len(obs) else None, n_obs=len(obs),
                 nbr=torch.empty((B, k), dtype=torch.int32, device=d),
                 out_j=torch.empty(B * k, dtype=torch.int16, device=d),
                 out_status=torch.empty(B * k, dtype=torch.int16, device=d),
                 out_margin=torch.empty(B * k, dtype=torch.float32, device=d),
                 out_rho4=torch.empty((B * k, 4), dtype=torch.float32, device=d),
                 out_T=torch.empty(B * k, dtype=torch.float32, device=d),
                 out_node=torch.empty(B, dtype=torch.int32, device=d),
                 out_J=torch.empty(B, dtype=torch.float32, device=d),
                 out_best=torch.empty(2, dtype=torch.float32, device=d))
        if flight is not None:
            P["flight"] = flight_array(flight)
            P["inc0"] = torch.tensor([-np.inf, -1.0, np.float32(flight["t_fall"]), 0.0],
                                     dtype=torch.float32, device=d)
            P["incumbent"] = P["inc0"].clone()
            P["out_reach"] = torch.full((ld,), np.nan, dtype=torch.float32, device=d)
        self.problems.append(P)
        return P

    def reset_trees(self):
        """Back to the initial trees (node counts, times, parents, states,
        incumbents)."""
        for P in self.problems:
            P["n_nodes"].fill_(P["n0"])
            P["t_node"].copy_(P["t_node0"])
            P["tree"].copy_(P["tree0"])
            P["parent"].copy_(P["parent0"])
            P["nu"].zero_()
            if "incumbent" in P:
                P["incumbent"].copy_(P["inc0"])

    def prepare(self):
        arr = (Problem * len(self.problems))()
        for i, P in enumerate(self.problems):
            q = arr[i]
            for key in ("tree", "n_nodes", "t_node", "parent", "nu", "cand", "kind", "t_req",
                        "v_rel", "vz0", "t_fall", "nbr", "out_j", "out_status", "out_margin",
                        "out_rho4", "out_T", "out_node", "out_J", "out_best"):
                setattr(q, key, P[key].data_ptr())
            q.ld, q.B, q.n_obs = P["ld"], P["B"], P["n_obs"]
            q.obs = None if P["obs"] is None else P["obs"].data_ptr()
            q.n_rounds = P["n_rounds"]
            for key in ("incumbent", "flight", "out_reach"):
                setattr(q, key, P[key].data_ptr() if key in P else None)
        self._arr = arr
        ps = ProblemSet(len(self.problems), arr, self.k, self.grid.data_ptr(), self.grid.shape[0],
                        self.samples, self.mode, self.margin, self.risk)
        _check(lib().fn_batch_prepare(self.ctx.h, C.byref(ps)), "fn_batch_prepare")

    def launch(self):
        _check(lib().fn_batch_launch(self.ctx.h, _stream()), "fn_batch_launch")

    def round(self, r):
        _check(lib().fn_batch_round(self.ctx.h, int(r), _stream()), "fn_batch_round")

    def prune(self, v_tip, blade):
        pr = make_prune(v_tip, blade)
        _check(lib().fn_batch_prune(self.ctx.h, C.byref(pr), _stream()), "fn_batch_prune")

    def cycle(self, n_iter, n_round, v_tip, blade):
        pr = make_prune(v_tip, blade)
        _check(lib().fn_cycle(self.ctx.h, int(n_iter), int(n_round), C.byref(pr), _stream()),
               "fn_cycle")

    def capture_cycle(self, stream, n_iter, n_round, v_tip, blade):
        pr = make_prune(v_tip, blade)
        with torch.cuda.stream(stream):
            _check(lib().fn_graph_capture_cycle(self.ctx.h, int(n_iter), int(n_round), C.byref(pr),
                                                C.c_void_p(stream.cuda_stream)),
                   "fn_graph_capture_cycle")

    def capture(self, stream):
        with torch.cuda.stream(stream):
            _check(lib().fn_graph_capture(self.ctx.h, C.c_void_p(stream.cuda_stream)),
                   "fn_graph_capture")

    def replay(self):
        _check(lib().fn_graph_launch(self.ctx.h, _stream()), "fn_graph_launch")


def edge_features(ctx: Context, tree, ld, n_nodes, cand, nbr, out=None):
    B, k = nbr.shape
    if out is None:
        out = torch.empty((B * k, 28), dtype=torch.float32, device=cand.device)
    _check(lib().edge_features(ctx.h, _ptr(tree), ld, n_nodes, _ptr(cand), B, _ptr(nbr), k,
                               _ptr(out), _stream()), "edge_features")
    return out


PAPER_RISK = dict(wv=0.20, vtarget=9.0, wp=8.0, wr=8.0, wx=1.0, r=0.09, nu0=0.90, lam=1.2)


def make_risk(gz=-9.81, sigma_mode=0, sp=0.0048, sv=0.0186, sa=0.0, s0=0.01, s1=0.05, **w):
    r = Risk()
    r.gz, r.sigma_mode, r.sp, r.sv, r.sa, r.s0, r.s1 = gz, sigma_mode, sp, sv, sa, s0, s1
    ww = dict(PAPER_RISK)
    ww.update(w)
    for key, v in ww.items():
        setattr(r, key, v)
    return r


C_ACC, C_SLEW, C_TORQUE, C_POWER, C_BAD = 1, 2, 4, 8, 128


def control(ctx: Context, q, qd, tau_prev, qg, qdg, T, dt, slew):
    """One step of the tracking controller (fn_control) for n instances:
    device [n][7] float tensors and T [n]; slew: 7 limits (N m / s).
    Returns (tau, qdd, status) device tensors."""
    n = q.shape[0]
    d = q.device
    tau = torch.empty((n, 7), dtype=torch.float32, device=d)
    qdd = torch.empty((n, 7), dtype=torch.float32, device=d)
    st = torch.empty(n, dtype=torch.int16, device=d)
    sl = (C.c_double * 7)(*[float(x) for x in slew])
    _check(lib().fn_control(ctx.h, n, _ptr(q), _ptr(qd), _ptr(tau_prev), _ptr(qg), _ptr(qdg),
                            _ptr(T), C.c_float(dt), sl, _ptr(tau), _ptr(qdd), _ptr(st), _stream()),
           "fn_control")
    return tau, qdd, st
