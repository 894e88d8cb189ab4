"""Test-side kinematics written independently of the oracle: homogeneous
modified-DH transforms, geometric Jacobians, the joint-space mass matrix
from Jacobians and the gravity vector from the potential energy.  Used only
to pin the oracle's recursive Newton-Euler dynamics."""
import math

import numpy as np


def dh_T(alpha, a, d, q):
    ca, sa, cq, sq = math.cos(alpha), math.sin(alpha), math.cos(q), math.sin(q)
    Rx = np.array([[1, 0, 0, 0], [0, ca, -sa, 0], [0, sa, ca, 0], [0, 0, 0, 1.0]])
    Tx = np.eye(4)
    Tx[0, 3] = a
    Rz = np.array([[cq, -sq, 0, 0], [sq, cq, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1.0]])
    Tz = np.eye(4)
    Tz[2, 3] = d
    return Rx @ Tx @ Rz @ Tz


def frames(arm, q):
    """World poses of frames 1..n."""
    T = np.eye(4)
    out = []
    for i in range(arm["n"]):
        T = T @ dh_T(arm["alpha"][i], arm["a"][i], arm["d"][i], q[i])
        out.append(T.copy())
    return out


def com_jacobians(arm, q):
    """(J_v, J_w, R) of every link's COM: J_v[j][:, i] = z_i x (p_cj - o_i)."""
    n = arm["n"]
    Fr = frames(arm, q)
    res = []
    for j in range(n):
        R = Fr[j][:3, :3]
        pc = Fr[j][:3, 3] + R @ np.asarray(arm["rc"][j])
        Jv = np.zeros((3, n))
        Jw = np.zeros((3, n))
        for i in range(j + 1):
            z = Fr[i][:3, 2]
            o = Fr[i][:3, 3]
            Jv[:, i] = np.cross(z, pc - o)
            Jw[:, i] = z
        res.append((Jv, Jw, R, pc))
    return res


def mass_matrix(arm, q):
    n = arm["n"]
    M = np.zeros((n, n))
    for j, (Jv, Jw, R, _) in enumerate(com_jacobians(arm, q)):
        Ic = R @ np.diag(arm["I"][j]) @ R.T
        M += arm["m"][j] * Jv.T @ Jv + Jw.T @ Ic @ Jw
    return M


def gravity_vector(arm, q):
    """g(q) = dV/dq with V = -sum_j m_j g0 . p_cj, i.e. sum_j m_j J_vj^T (-g0)."""
    g0 = np.asarray(arm["g"], float)
    out = np.zeros(arm["n"])
    for j, (Jv, _, _, _) in enumerate(com_jacobians(arm, q)):
        out += arm["m"][j] * Jv.T @ (-g0)
    return out


def potential(arm, q):
    g0 = np.asarray(arm["g"], float)
    return sum(-arm["m"][j] * g0 @ pc for j, (_, _, _, pc) in enumerate(com_jacobians(arm, q)))


def coriolis_vector(arm, q, qd, h=1e-5):
    """c(q, qd) from Christoffel symbols of central-differenced M(q)."""
    n = arm["n"]
    dM = np.zeros((n, n, n))  # dM[:, :, k] = dM/dq_k
    for k in range(n):
        e = np.zeros(n)
        e[k] = h
        dM[:, :, k] = (mass_matrix(arm, q + e) - mass_matrix(arm, q - e)) / (2 * h)
    c = np.zeros(n)
    for i in range(n):
        for j in range(n):
            for k in range(n):
                gam = 0.5 * (dM[i, j, k] + dM[i, k, j] - dM[j, k, i])
                c[i] += gam * qd[j] * qd[k]
    return c


def random_arm(n, seed, alphas=None):
    rng = np.random.default_rng(seed)
    if alphas is None:
        alphas = rng.choice([0.0, math.pi / 2, -math.pi / 2], n)
    arm = dict(
        n=n, alpha=np.asarray(alphas, float), a=rng.uniform(0.05, 0.35, n),
        d=rng.uniform(0.05, 0.35, n), m=rng.uniform(0.5, 4, n),
        rc=rng.uniform(-0.1, 0.1, (n, 3)), I=rng.uniform(0.005, 0.05, (n, 3)),
        Im=rng.uniform(0.01, 0.1, n), psi1=rng.uniform(0.1, 0.6, n), psi2=rng.uniform(5, 50, n),
        psi3=rng.uniform(-0.05, 0.05, n), qmin=np.full(n, -2.8), qmax=np.full(n, 2.8),
        qdmax=np.full(n, 2.5), taumax=np.full(n, 50.0), acc=np.full(n, 10.0), wmax=300.0,
        g=np.array([0.0, 0.0, -9.81]), tool=np.array([0.0, 0.0, 0.1]),
        sph_link=np.zeros(0, np.int32), sph=np.zeros((0, 4)))
    return arm
