"""EMU quasi-Newton solver in deformation space (oracle part O1), FP64.

Variables: one free deformation gradient F_i per tet (Sec. 3.1).  Objective,
the separated energy (eq. separated):

    E(F) = sum_i vol_i Psi_i(F_i) + 1/2 sum_i beta_i |A_i(q*(F)) - F_i|^2 - W(q*(F)),
    beta_i = alpha w_i,  W(q) = f . q  (constant external forces, Sec. 3.4; 0 if unset),

with q*(F) the nearest continuous mesh (eq. acap) and A_i = G_i q.  One
iteration, in the order of Sec. 3.2.1 and Algorithm 1 (with the readings of its
inverted loop test, the sign of the step and the backtracking loop that the
design notes list):

1. q = q*(F), A = G q.  Exact gradient via the envelope theorem (eq. gradient,
   eq. gradient2): g_i = vol_i P(F_i) + beta_i (F_i - A_i).  Stop at |g|_2 <= tol.
2. Block Hessian H_i = clamp(vol_i d2Psi(F_i)) + beta_i I_9 (eq. not-yet with the
   definiteness fix), or -- with ``hessian="split"`` -- the block-diagonal part
   of it in the rotated frame dF = R_i dX (6x6 symmetric dX, 3x3 skew dX, each
   clamped), the GPU library's default block structure; or -- with
   ``hessian="coupled"`` -- the full 9x9 block with the fix applied to the
   isotropic term only (clamped per rotated-frame block) and the convex fiber
   term kept whole, the library's 9x9 option.
3. Low-rank correction (eq. low-rank, eq. Hessian-woodbury):
   B_i[(c,j),(c',e)] = w_i delta_cc' grad_i(phi_j)[e], y = sum B_i H_i^{-1} g_i,
   C = Lambda - alpha sum B_i H_i^{-1} B_i^T, z = C^{-1} y,
   d_i = H_i^{-1} g_i + alpha H_i^{-1} B_i^T z,  p = -d.
4. Backtracking Armijo line search from sigma = 10 (factor 0.5, c = 1e-4), each
   trial re-solving the ACAP problem for F + sigma p.
5. Accept F <- F + sigma p.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from . import contact as cnt
from . import material as mat
from . import mesh as msh

SQ2 = math.sqrt(2.0)
# basis of skew-symmetric 3x3 matrices, unit Frobenius norm, planes (0,1),(0,2),(1,2)
SKEW = np.zeros((3, 3, 3))
for _m, (_a, _b) in enumerate(((0, 1), (0, 2), (1, 2))):
    SKEW[_m, _a, _b] = 1.0 / SQ2
    SKEW[_m, _b, _a] = -1.0 / SQ2
# 9x9 orthonormal basis of 3x3 matrices: 6 symmetric then 3 skew (columns, row-major vec)
YBASIS = np.concatenate([mat.BASIS.reshape(6, 9), SKEW.reshape(3, 9)], axis=0).T


def rest_state(M):
    return np.tile(np.eye(3), (M.m, 1, 1))


def element_energy(M, F, A, a_el):
    D = A - F
    return (M.vol * mat.psi(F, M.mu, M.lhat, a_el, M.kf, M.fiber)
            + 0.5 * M.beta * np.einsum("icd,icd->i", D, D))


def grad_F(M, F, A, a_el):
    """Exact dE/dF per element (envelope theorem): vol P(F) + beta (F - A),
    minus w_i G_i L_ff^{-1} f (the derivative of the external work f . q*(F),
    Sec. 3.4) when forces are set."""
    g = (M.vol[:, None, None] * mat.pk1(F, M.mu, M.lhat, a_el, M.kf, M.fiber)
         + M.beta[:, None, None] * (F - A))
    if M.vext is not None:
        g = g - M.w[:, None, None] * msh.gather_A(M, M.vext)
    return g


def frame_basis(R):
    """T_i = (R_i (x) I) Y: maps coordinates in the rotated (sym, skew) basis to dF."""
    m = R.shape[0]
    T9 = np.einsum("ice,df->icdef", R, np.eye(3)).reshape(m, 9, 9)
    return T9 @ YBASIS


def block_hessian(M, F, a_el, hessian="full"):
    """Approximate element Hessian blocks (9x9, F coordinates)."""
    Hel = M.vol[:, None, None] * mat.hess(F, M.mu, M.lhat, a_el, M.kf, M.fiber)
    if hessian == "full":
        Hc = mat.clamp_psd(Hel)
    elif hessian == "split":
        T = frame_basis(mat.polar_rotation(F))
        HY = np.einsum("iab,ibc,icd->iad", np.transpose(T, (0, 2, 1)), Hel, T)
        Hb = np.zeros_like(HY)
        Hb[:, :6, :6] = mat.clamp_psd(HY[:, :6, :6])
        Hb[:, 6:, 6:] = mat.clamp_psd(HY[:, 6:, 6:])
        Hc = np.einsum("iab,ibc,idc->iad", T, Hb, T)
    elif hessian == "coupled":
        # the full 9x9 block with the definiteness fix on the term that needs
        # it: the isotropic Hessian (block diagonal in the rotated frame, each
        # block clamped) plus the fiber Hessian, a convex quadratic's (PSD)
        zero = np.zeros(M.m)
        Hiso = M.vol[:, None, None] * mat.hess(F, M.mu, M.lhat, zero, M.kf, M.fiber)
        Hfib = M.vol[:, None, None] * mat.hess(F, zero, zero, a_el, M.kf, M.fiber)
        T = frame_basis(mat.polar_rotation(F))
        HY = np.einsum("iab,ibc,icd->iad", np.transpose(T, (0, 2, 1)), Hiso, T)
        Hb = np.zeros_like(HY)
        Hb[:, :6, :6] = mat.clamp_psd(HY[:, :6, :6])
        Hb[:, 6:, 6:] = mat.clamp_psd(HY[:, 6:, 6:])
        Hc = np.einsum("iab,ibc,idc->iad", T, Hb, T) + Hfib
    else:
        raise ValueError(hessian)
    return Hc + M.beta[:, None, None] * np.eye(9)


def reduced_block_hessian(M, F, a_el, hessian="full"):
    """Blocks of the reduced variables: per-tet blocks for non-bone tets; for
    a bone, the definiteness fix of the summed element Hessians of its tets
    (they share F_b) plus the summed beta."""
    if M.red_of is None:
        return block_hessian(M, F, a_el, hessian)
    Hel = M.vol[:, None, None] * mat.hess(F, M.mu, M.lhat, a_el, M.kf, M.fiber)
    Hsum = reduce_sum(M, Hel)
    Fr = np.zeros((M.m_red, 3, 3))
    Fr[M.red_of] = F
    if hessian == "full":
        Hc = mat.clamp_psd(Hsum)
    elif hessian == "split":
        T = frame_basis(mat.polar_rotation(Fr))
        HY = np.einsum("iab,ibc,icd->iad", np.transpose(T, (0, 2, 1)), Hsum, T)
        Hb = np.zeros_like(HY)
        Hb[:, :6, :6] = mat.clamp_psd(HY[:, :6, :6])
        Hb[:, 6:, 6:] = mat.clamp_psd(HY[:, 6:, 6:])
        Hc = np.einsum("iab,ibc,idc->iad", T, Hb, T)
    else:
        raise ValueError(hessian)
    return Hc + reduce_sum(M, M.beta)[:, None, None] * np.eye(9)


def mode_gradients(M, idx=None):
    """grad_i phi_j = sum_v phi_j(v) b_{i,v} (pinned vertices carry zero), [m,k,3]."""
    k = M.phi.shape[0]
    phi_full = np.zeros((M.n, k))
    phi_full[M.free] = M.phi.T
    tets = M.tets if idx is None else M.tets[idx]
    b = M.b if idx is None else M.b[idx]
    return np.einsum("ivj,ivd->ijd", phi_full[tets], b)


def woodbury_blocks(M, idx):
    """B_i in R^{3k x 9}: B_i[(c,j),(c',e)] = w_i delta_cc' grad_i phi_j[e]."""
    gp = mode_gradients(M, idx)
    k = gp.shape[1]
    B = np.einsum("i,ce,ijd->icjed", M.w[idx], np.eye(3), gp)
    return B.reshape(len(idx), 3 * k, 9)


def reduce_sum(M, x):
    """Affine bones (Sec. 3.3): per-tet quantities summed onto the reduced
    variables (a bone's tets share its F_b); identity without bones."""
    if M.red_of is None:
        return x
    out = np.zeros((M.m_red,) + x.shape[1:])
    np.add.at(out, M.red_of, x)
    return out


def expand(M, x):
    """Reduced quantities back to the tets (a bone's value on each of its tets)."""
    return x if M.red_of is None else x[M.red_of]


def direction(M, H, g, chunk=4096, return_parts=False, B_all=None):
    """Woodbury direction d = Htilde^{-1} g for blocks H [m,9,9], gradient g [m,9]
    (one block per variable; ``B_all`` [m,k,9] gives the low-rank rows of the
    variables when they are not the tets', e.g. the summed rows of a bone)."""
    gbar = np.linalg.solve(H, g[..., None])[..., 0]
    if M.phi is None or M.phi.shape[0] == 0:
        return (gbar, None, None, None) if return_parts else gbar
    k3 = 3 * M.phi.shape[0]
    Lam = np.tile(M.nu, 3)
    y = np.zeros(k3)
    Gm = np.zeros((k3, k3))
    HiBt_all = []
    nvar = H.shape[0]
    for lo in range(0, nvar, chunk):
        idx = np.arange(lo, min(nvar, lo + chunk))
        B = woodbury_blocks(M, idx) if B_all is None else B_all[idx]
        HiBt = np.linalg.solve(H[idx], np.transpose(B, (0, 2, 1)))
        y += np.einsum("ikl,il->k", B, gbar[idx])
        Gm += np.tensordot(B, HiBt, axes=([0, 2], [0, 1]))
        HiBt_all.append(HiBt)
    C = np.diag(Lam) - M.alpha * Gm
    C = 0.5 * (C + C.T)
    cf = sla.cho_factor(C, lower=True)          # raises LinAlgError if C is not SPD
    z = sla.cho_solve(cf, y)
    HiBt = np.concatenate(HiBt_all, axis=0)
    d = gbar + M.alpha * np.einsum("ilk,k->il", HiBt, z)
    if return_parts:
        return d, y, C, z
    return d


def delta_energy(M, F, P, sigma, A, A_t, a_el, dwork=0.0):
    """E(F + sigma P) - E(F) as a compensated sum of per-element differences.
    Each element difference is expanded exactly in sigma (|F+tP|^2, det(F+tP),
    |(F+tP)u|^2 and the ACAP residual) so that no two total energies are
    subtracted; A_t is the trial's compatible gradient from its own ACAP solve
    and dwork = W(q_t) - W(q) the change of the external work."""
    t = sigma
    J = np.linalg.det(F)
    dJ = (t * np.einsum("iab,iab->i", mat.cof(F), P) + t * t * np.einsum("iab,iab->i", F, mat.cof(P))
          + t ** 3 * np.linalg.det(P))
    dI = 2 * t * np.einsum("iab,iab->i", F, P) + t * t * np.einsum("iab,iab->i", P, P)
    Fu = np.einsum("iab,ib->ia", F, M.fiber)
    Pu = np.einsum("iab,ib->ia", P, M.fiber)
    dfib = 2 * t * np.einsum("ia,ia->i", Fu, Pu) + t * t * np.einsum("ia,ia->i", Pu, Pu)
    dpsi = (0.5 * M.mu * dI - M.mu * dJ + 0.5 * M.lhat * dJ * (2 * (J - 1.0) + dJ)
            + a_el * M.kf * dfib)
    D = A - F
    dD = (A_t - A) - t * P
    dacap = 0.5 * M.beta * np.einsum("icd,icd->i", dD, 2 * D + dD)
    return math.fsum(np.append(M.vol * dpsi + dacap, -dwork))


def gradient_norm(M, F, a_el):
    q = msh.acap_solve(M, F)
    A = msh.gather_A(M, q)
    g = reduce_sum(M, grad_F(M, F, A, a_el))
    return math.sqrt(math.fsum((g * g).reshape(-1))), q


def solve(M, a, F0=None, tol=1e-8, max_iters=5000, sigma0=10.0, armijo_c=1e-4, rho=0.5,
          min_sigma_exp=40, hessian="full", trials="fresh", history=False, callback=None, contact=None):
    """Run the EMU quasi-Newton iteration from F0 (rest if None) to |g|_2 <= tol.

    ``trials="fresh"`` re-solves the ACAP problem for every line-search trial as
    Algorithm 1 does.  ``trials="affine"`` uses that q*(F) is affine in F: one
    homogeneous solve of the direction gives q(sigma) = q + sigma dq for every
    trial -- the same values without the rounding noise of differencing two
    independent solves, which sets a floor near 1e-10 on tiny meshes.

    ``contact`` (``oracle.contact.obstacles(...)``) runs Algorithm 1's contact
    loop after every accepted step with the iteration's Woodbury inverse."""
    a_el = msh.activation_per_element(M, a)
    F = rest_state(M) if F0 is None else np.array(F0, dtype=np.float64)
    hist = []
    stats = dict(iters=0, trials=0, solves=0, converged=False, status="ok", contact_rounds=0)
    if contact is not None and M.red_of is not None:
        raise ValueError("the contact loop runs on per-tet variables")
    q = msh.acap_solve(M, F)
    stats["solves"] += 1
    while True:
        A = msh.gather_A(M, q)
        G = grad_F(M, F, A, a_el)
        Gr = reduce_sum(M, G)
        gnorm = math.sqrt(math.fsum((Gr * Gr).reshape(-1)))
        E0 = math.fsum(element_energy(M, F, A, a_el)) - msh.work(M, q)
        if history:
            hist.append(dict(E=E0, gnorm=gnorm))
        if callback is not None:
            callback(stats["iters"], E0, gnorm)
        if gnorm <= tol:
            stats["converged"] = True
            break
        if stats["iters"] >= max_iters:
            stats["status"] = "not_converged"
            break
        if M.red_of is None:
            H = block_hessian(M, F, a_el, hessian)
            g = G.reshape(M.m, 9)
            d = direction(M, H, g)
            P = -d.reshape(M.m, 3, 3)
        else:
            H = reduced_block_hessian(M, F, a_el, hessian)
            g = reduce_sum(M, G.reshape(M.m, 9))
            Bred = reduce_sum(M, woodbury_blocks(M, np.arange(M.m)))
            d = direction(M, H, g, B_all=Bred)
            P = -expand(M, d).reshape(M.m, 3, 3)
        gp = -math.fsum((g * d).reshape(-1))
        if not gp < 0.0:
            stats["status"] = "not_descent"
            break
        sigma = sigma0
        accepted = False
        if trials == "affine":
            dq = msh.acap_solve(M, P, pinned=False)
            dA = msh.gather_A(M, dq)
            stats["solves"] += 1
        for _ in range(min_sigma_exp + 1):
            Ft = F + sigma * P
            if trials == "affine":
                qt = q + sigma * dq
                At = A + sigma * dA
            else:
                qt = msh.acap_solve(M, Ft)
                stats["solves"] += 1
                At = msh.gather_A(M, qt)
            stats["trials"] += 1
            dwork = 0.0
            if M.fext is not None:
                dwork = math.fsum((M.fext[M.free] * (qt - q)[M.free]).reshape(-1))
            if delta_energy(M, F, P, sigma, A, At, a_el, dwork) <= armijo_c * sigma * gp:
                accepted = True
                break
            sigma *= rho
        if not accepted:
            stats["status"] = "linesearch"
            break
        F, q = Ft, qt
        if contact is not None:
            F, q, rounds = cnt.contact_loop(M, F, q, lambda nu: direction(M, H, nu), contact)
            stats["contact_rounds"] += rounds
        stats["iters"] += 1
        if history:
            hist[-1]["sigma"] = sigma
    stats.update(gnorm=gnorm, energy=E0)
    out = dict(q=q, F=F, stats=stats)
    if history:
        out["history"] = hist
    return out
