"""Brute-force dense F-form Newton (oracle part O4) for meshes of a few tets.

Builds the compatibility operator G (9m x 3n_f) densely and uses the exact
Hessian of the separated energy (eq. full-Hessian with per-element weights):

    d2E/dF2 = blockdiag(vol_i d2Psi_i) + B_w - B_w G (G^T B_w G)^{-1} G^T B_w,
    B_w = diag(beta_i) (x) I_9,

which is only tractable for tiny meshes (the paper notes the dense inverse is
what rules Newton out at scale).  Newton steps use the PSD-clamped full matrix
and a backtracking line search on E.
"""
from __future__ import annotations

import math

import numpy as np

from . import material as mat
from . import mesh as msh


def dense_G(M):
    nf = M.free.size
    G = np.zeros((M.m, 3, 3, nf, 3))
    for v in range(4):
        fp = M.fpos[M.tets[:, v]]
        ok = np.nonzero(fp >= 0)[0]
        for c in range(3):
            G[ok, c, :, fp[ok], c] += M.b[ok, v, :]
    return G.reshape(9 * M.m, 3 * nf)


def solve(M, a, tol=1e-11, max_iters=200):
    a_el = msh.activation_per_element(M, a)
    G = dense_G(M)
    Bw = np.repeat(M.beta, 9)
    K = G.T @ (Bw[:, None] * G)
    Kinv = np.linalg.inv(K)
    # constant pinned contribution to A: G_p q_p
    qp = np.zeros((M.n, 3))
    qp[M.pins] = M.pin_xyz
    Ap = msh.gather_A(M, qp).reshape(-1)
    Pq = Kinv @ (G.T * Bw[None, :])           # q_f = Pq (F - Ap)

    def energy(Fv):
        qf = Pq @ (Fv - Ap)
        Av = G @ qf + Ap
        F = Fv.reshape(M.m, 3, 3)
        D = (Av - Fv)
        e = M.vol * mat.psi(F, M.mu, M.lhat, a_el, M.kf, M.fiber)
        return math.fsum(e) + 0.5 * math.fsum(Bw * D * D), Av, qf

    # variables: one 3x3 per tet, or (affine bones, Sec. 3.3) one per non-bone
    # tet and one per bone: F = Pm F_red with Pm the 0/1 map of tets to variables
    nvar = M.m if M.red_of is None else M.m_red
    red = np.arange(M.m) if M.red_of is None else M.red_of
    Pm = np.zeros((9 * M.m, 9 * nvar))
    for i in range(M.m):
        Pm[9 * i:9 * i + 9, 9 * red[i]:9 * red[i] + 9] = np.eye(9)
    Fr = np.tile(np.eye(3), (nvar, 1, 1)).reshape(-1)
    Fv = Pm @ Fr
    E, Av, qf = energy(Fv)
    it = 0
    while True:
        F = Fv.reshape(M.m, 3, 3)
        g = Pm.T @ ((M.vol[:, None, None] * mat.pk1(F, M.mu, M.lhat, a_el, M.kf, M.fiber)).reshape(-1)
                    + Bw * (Fv - Av))
        gn = float(np.linalg.norm(g))
        if gn <= tol or it >= max_iters:
            break
        Hb = M.vol[:, None, None] * mat.hess(F, M.mu, M.lhat, a_el, M.kf, M.fiber)
        H = np.zeros((9 * M.m, 9 * M.m))
        for i in range(M.m):
            H[9 * i:9 * i + 9, 9 * i:9 * i + 9] = Hb[i]
        H += np.diag(Bw) - (Bw[:, None] * G) @ Kinv @ (G.T * Bw[None, :])
        H = Pm.T @ H @ Pm
        H = mat.clamp_psd(0.5 * (H + H.T)) + 1e-12 * np.abs(H).max() * np.eye(H.shape[0])
        step = -np.linalg.solve(H, g)
        gs = float(g @ step)
        t = 1.0
        for _ls in range(60):
            Et, Avt, qft = energy(Pm @ (Fr + t * step))
            if Et <= E + 1e-4 * t * gs or abs(Et - E) <= 1e-15 * abs(E):
                break
            t *= 0.5
        Fr = Fr + t * step
        Fv, E, Av, qf = Pm @ Fr, Et, Avt, qft
        it += 1
    q = qp.copy()
    q[M.free] = qf.reshape(-1, 3)
    return dict(q=q, F=Fv.reshape(M.m, 3, 3), iters=it, gnorm=gn, energy=E)
