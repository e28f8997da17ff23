"""Independent q-space Newton solvers (oracle parts O2 and O3), FP64.

O2 -- Moreau-envelope FEM.  Minimizing the separated energy (eq. separated)
over F and q jointly is the same as minimizing over q alone

    Ehat(q) = sum_i e_i(G_i q),  e_i(A) = min_X vol_i Psi_i(X) + 1/2 beta_i |A - X|^2,

because the ACAP term (eq. ACAPEnergy) is the only coupling and min_F min_q =
min_q min_F.  So a plain Newton solve of Ehat reaches EMU's minimizer without
sharing any of EMU's algorithm (no deformation-gradient iterates, no low-rank
Hessian, no Woodbury).  grad_A e = beta (A - X*), and by the implicit function
theorem on the prox condition vol P(X*) + beta (X* - A) = 0,
hess_A e = beta I - beta^2 (vol d2Psi(X*) + beta I)^{-1}.

O3 -- plain FEM on sum_i vol_i Psi_i(G_i q), the continuous problem of
eq. continuum discretized with linear tets; EMU approaches it as alpha grows.

External forces (Sec. 3.4).  EMU's energy subtracts the work f . q*(F) of
constant vertex forces through the nearest continuous mesh; since
f . q*(F) = sum_i nu_i . F_i + const with nu_i = w_i G_i L_ff^{-1} f, the joint
form above gains -nu_i . X in each element's prox (same minimizer, O2).  O3
subtracts f . q directly (the alpha -> infinity limit of the same term).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import material as mat
from . import mesh as msh


def _assemble(M, Hel):
    """K = sum_i G_i^T H_i G_i for 9x9 element blocks (F coordinates), free DOFs."""
    # K_i[(v,c),(v',c')] = sum_{d,d'} b[v,d] H[(c,d),(c',d')] b[v',d']
    H4 = Hel.reshape(-1, 3, 3, 3, 3)
    Ke = np.einsum("ivd,icdef,iwf->ivcwe", M.b, H4, M.b)       # [m,4,3,4,3]
    dof = (3 * M.tets[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 12)
    rows = np.repeat(dof, 12, axis=1).reshape(-1)
    cols = np.tile(dof, (1, 12)).reshape(-1)
    K = sp.coo_matrix((Ke.reshape(-1), (rows, cols)), shape=(3 * M.n, 3 * M.n)).tocsr()
    fdof = (3 * M.free[:, None] + np.arange(3)[None, :]).reshape(-1)
    return K[fdof][:, fdof].tocsc(), fdof


def _scatter_grad(M, GA):
    """sum_i G_i^T GA_i as [n,3]: out[v,c] = sum_i sum_d GA_i[c,d] b_{i,v}[d]."""
    contrib = np.einsum("icd,ivd->ivc", GA, M.b)
    out = np.zeros((M.n, 3))
    np.add.at(out, M.tets.reshape(-1), contrib.reshape(-1, 3))
    return out


def force_field(M):
    """nu_i = w_i G_i L_ff^{-1} f: the deformation-space form of the external
    work, f . q*(F) = sum_i nu_i . F_i + const (zero without forces)."""
    if M.vext is None:
        return np.zeros((M.m, 3, 3))
    return M.w[:, None, None] * msh.gather_A(M, M.vext)


def prox(M, A, a_el, tol=1e-13, max_iters=100, nu=None):
    """X* = argmin_X vol Psi(X) + 1/2 beta |A - X|^2 - nu . X per element
    (damped Newton from X = A; nu = 0 without external forces)."""
    X = A.copy()
    vol, beta = M.vol, M.beta
    nu = np.zeros_like(A) if nu is None else nu

    def obj(X):
        D = A - X
        # the work term relative to X = A: the same minimizer without a large
        # constant in the values the line search compares
        return (vol * mat.psi(X, M.mu, M.lhat, a_el, M.kf, M.fiber) + 0.5 * beta * np.einsum("icd,icd->i", D, D)
                + np.einsum("icd,icd->i", nu, D))

    # force scale of each element's stationarity condition: the ACAP term's
    # and the material's (a stiff element's gradient carries rounding of
    # vol (mu + lhat) |X|, far above beta |X| when it is not stiffness-weighted)
    scale = (beta + vol * (M.mu + M.lhat)) * (1.0 + np.sqrt(np.einsum("icd,icd->i", A, A)))
    for _ in range(max_iters):
        g = (vol[:, None, None] * mat.pk1(X, M.mu, M.lhat, a_el, M.kf, M.fiber) + beta[:, None, None] * (X - A)
             - nu)
        gn = np.sqrt(np.einsum("icd,icd->i", g, g))
        if np.all(gn <= tol * scale):
            break
        H = vol[:, None, None] * mat.hess(X, M.mu, M.lhat, a_el, M.kf, M.fiber) + beta[:, None, None] * np.eye(9)
        # damped Newton on a (possibly non-convex) element objective: each
        # eigenvalue of the Hessian replaced by its absolute value (a step
        # along negative curvature keeps the length a curvature of that size
        # gives), floored at 1e-12 of the largest so the step is defined
        w, V = np.linalg.eigh(H)
        w = np.abs(w)
        w = np.maximum(w, 1e-12 * w.max(axis=1, keepdims=True))
        step = -np.einsum("iab,ib,icb,ic->ia", V, 1.0 / w, V, g.reshape(-1, 9)).reshape(-1, 3, 3)
        f0 = obj(X)
        t = np.ones(M.m)
        for _ls in range(30):
            Xt = X + t[:, None, None] * step
            f1 = obj(Xt)
            bad = f1 > f0 + 1e-4 * t * np.einsum("icd,icd->i", g, step) + 1e-15 * np.abs(f0)
            if bad.any():
                # near the minimizer the decrease of the objective falls below
                # its rounding; a step that shrinks the gradient is then taken
                gt = (vol[:, None, None] * mat.pk1(Xt, M.mu, M.lhat, a_el, M.kf, M.fiber)
                      + beta[:, None, None] * (Xt - A) - nu)
                bad &= np.sqrt(np.einsum("icd,icd->i", gt, gt)) >= 0.5 * gn
            if not bad.any():
                break
            t = np.where(bad, 0.5 * t, t)
        X = X + t[:, None, None] * step
    H = vol[:, None, None] * mat.hess(X, M.mu, M.lhat, a_el, M.kf, M.fiber) + beta[:, None, None] * np.eye(9)
    return X, H


def moreau_solve(M, a, q0=None, tol=1e-10, max_iters=200, history=False, callback=None):
    """O2: Newton on Ehat(q), globalized by Levenberg-Marquardt; returns q, the
    prox F = X* and stats."""
    a_el = msh.activation_per_element(M, a)
    q = M.rest.copy() if q0 is None else q0.copy()
    q[M.pins] = M.pin_xyz
    hist = []

    nu = force_field(M)

    def Ehat(q):
        A = msh.gather_A(M, q)
        X, H = prox(M, A, a_el, nu=nu)
        D = A - X
        e = (M.vol * mat.psi(X, M.mu, M.lhat, a_el, M.kf, M.fiber) + 0.5 * M.beta * np.einsum("icd,icd->i", D, D)
             - np.einsum("icd,icd->i", nu, X))
        return math.fsum(e), A, X, H

    E, A, X, H = Ehat(q)
    it = 0
    lam = 0.0
    while True:
        GA = M.beta[:, None, None] * (A - X)
        grad = _scatter_grad(M, GA)[M.free].reshape(-1)
        gn = float(np.linalg.norm(grad))
        if history:
            hist.append((E, gn))
        if callback is not None:
            callback(it, E, gn, lam)
        if gn <= tol or it >= max_iters:
            break
        Hinv = np.linalg.inv(H)
        b2 = M.beta[:, None, None]
        He = b2 * np.eye(9) - b2 ** 2 * Hinv
        He = 0.5 * (He + np.transpose(He, (0, 2, 1)))
        # Newton step with the exact assembled Hessian K of Ehat, globalized by
        # Levenberg-Marquardt: (K + lam D) s = -grad with D the diagonal of the
        # assembly of the per-element PSD parts; lam shrinks after an accepted
        # step and grows after a rejected or non-descent one, so near the
        # minimizer the step is exact Newton (each element's envelope Hessian
        # is indefinite wherever Psi is; the sum is positive definite there)
        K, _ = _assemble(M, He)
        Dg = _assemble(M, mat.clamp_psd(He))[0].diagonal()
        Dg = sp.diags(np.maximum(Dg, 1e-12 * Dg.max()))
        accepted = False
        for _try in range(60):
            try:
                step = spla.spsolve((K + lam * Dg).tocsc(), -grad) if lam > 0 else spla.spsolve(K, -grad)
            except RuntimeError:
                step = None
            if step is None or not np.all(np.isfinite(step)) or not float(grad @ step) < 0.0:
                lam = max(4.0 * lam, 1e-6)
                continue
            gs = float(grad @ step)
            qt = q.copy()
            qt[M.free] += step.reshape(-1, 3)
            Et, At, Xt, Ht = Ehat(qt)
            if Et <= E + 1e-4 * gs or abs(Et - E) <= 1e-15 * abs(E):
                accepted = True
                lam = lam / 8.0 if lam > 1e-9 else 0.0
                break
            lam = max(4.0 * lam, 1e-6)
        if not accepted:
            break
        q, E, A, X, H = qt, Et, At, Xt, Ht
        it += 1
    out = dict(q=q, F=X, iters=it, gnorm=gn, energy=E)
    if history:
        out["history"] = hist
    return out


def fem_solve(M, a, q0=None, tol=1e-10, max_iters=200):
    """O3: plain FEM Newton on sum_i vol_i Psi_i(G_i q) with clamped element Hessians."""
    a_el = msh.activation_per_element(M, a)
    q = M.rest.copy() if q0 is None else q0.copy()
    q[M.pins] = M.pin_xyz

    def energy(q):
        A = msh.gather_A(M, q)
        return math.fsum(M.vol * mat.psi(A, M.mu, M.lhat, a_el, M.kf, M.fiber)) - msh.work(M, q), A

    E, A = energy(q)
    it = 0
    while True:
        P = M.vol[:, None, None] * mat.pk1(A, M.mu, M.lhat, a_el, M.kf, M.fiber)
        grad = _scatter_grad(M, P)[M.free]
        if M.fext is not None:
            grad = grad - M.fext[M.free]
        grad = grad.reshape(-1)
        gn = float(np.linalg.norm(grad))
        if gn <= tol or it >= max_iters:
            break
        He = mat.clamp_psd(M.vol[:, None, None] * mat.hess(A, M.mu, M.lhat, a_el, M.kf, M.fiber))
        K, _ = _assemble(M, He)
        step = -spla.spsolve(K, grad)
        gs = float(grad @ step)
        t = 1.0
        for _ls in range(60):
            qt = q.copy()
            qt[M.free] += t * step.reshape(-1, 3)
            Et, At = energy(qt)
            if Et <= E + 1e-4 * t * gs or abs(Et - E) <= 1e-15 * abs(E):
                break
            t *= 0.5
        q, E, A = qt, Et, At
        it += 1
    return dict(q=q, iters=it, gnorm=gn, energy=E)
