"""Mesh setup of the oracle: geometry, ACAP weights, Laplacian, factor, modes.

* Deformation gradient of a linear tet (eq. defograd): F = D_s D_m^{-1}, so the
  compatible gradient is A_i(q) = sum_v q_v b_{i,v}^T with b_{i,1..3} the rows of
  D_m^{-1} and b_{i,4} = -(b_{i,1}+b_{i,2}+b_{i,3}).
* ACAP energy (eq. ACAPEnergy), weighted per element:
  1/2 sum_i w_i |A_i(q) - F_i|^2 with, by ``weight_mode``,
  0: w_i = vol_i mu_i / mu_ref (stiffness-proportional for every tet),
  1: w_i = vol_i (the printed unweighted energy as an integral),
  2: stiffness-proportional for muscle and tendon but w_i = vol_i for bone
     tets (the exception Sec. 3.3 states: a stiff spring on bones can lock).
  Its q-Hessian is L_w (x) I_3 with the scalar
  weighted Laplacian L_w = sum_i w_i sum_{v,v'} (b_{i,v}.b_{i,v'}) e_v e_v'^T.
* Nearest continuous mesh (eq. acap): q* solves L_ff q_f = r_f - L_fp qbar_p per
  coordinate, r_c[v] = sum_{i ∋ v} w_i b_{i,v} . F_i[c,:]; pins remove the
  rigid null space (Sec. 3.1).
* Low-rank modes (eq. low-rank): the 16 lowest eigenpairs of L_ff, used as the
  48 coordinate modes e_c (x) phi_j.
* External forces (Sec. 3.4): constant vertex forces f do the work
  W(q) = sum_{v free} f_v . q_v; forces at pinned vertices do no work.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import material as mat


@dataclasses.dataclass
class Mesh:
    rest: np.ndarray        # [n,3]
    tets: np.ndarray        # [m,4] oriented
    b: np.ndarray           # [m,4,3] hat gradients
    vol: np.ndarray         # [m]
    mu: np.ndarray
    lhat: np.ndarray
    fiber: np.ndarray       # [m,3] unit
    group: np.ndarray       # [m]
    bone: np.ndarray        # [m] bone id, -1 = not bone
    w: np.ndarray           # ACAP weights
    beta: np.ndarray        # alpha * w
    alpha: float
    mu_ref: float
    kf: float
    pins: np.ndarray
    pin_xyz: np.ndarray
    free: np.ndarray        # free vertex ids (ascending)
    fpos: np.ndarray        # [n] position in free list or -1
    L: sp.csr_matrix        # full weighted Laplacian (n x n)
    Lff: sp.csc_matrix
    Lfp: sp.csr_matrix
    lu: object              # factor of Lff
    nu: np.ndarray = None   # mode eigenvalues [k/3]
    phi: np.ndarray = None  # modes [k/3, n_f]
    fext: np.ndarray = None  # external vertex forces [n,3] (None: W = 0)
    vext: np.ndarray = None  # L_ff^{-1} f at free vertices, 0 at pins [n,3]
    red_of: np.ndarray = None  # affine bones: reduced variable of each tet (None: one per tet)
    m_red: int = 0

    @property
    def n(self):
        return self.rest.shape[0]

    @property
    def m(self):
        return self.tets.shape[0]


def orient(rest, tets):
    """Swap local vertices 1 and 2 of tets with negative rest volume."""
    t = np.array(tets, dtype=np.int64)
    x = rest[t]
    Dm = np.stack([x[:, 0] - x[:, 3], x[:, 1] - x[:, 3], x[:, 2] - x[:, 3]], axis=2)
    neg = np.linalg.det(Dm) < 0
    t[neg, 0], t[neg, 1] = t[neg, 1].copy(), t[neg, 0].copy()
    return t


def hat_gradients(rest, tets):
    x = rest[tets]
    Dm = np.stack([x[:, 0] - x[:, 3], x[:, 1] - x[:, 3], x[:, 2] - x[:, 3]], axis=2)
    Dinv = np.linalg.inv(Dm)
    b = np.empty((tets.shape[0], 4, 3))
    b[:, :3, :] = Dinv
    b[:, 3, :] = -Dinv.sum(axis=1)
    vol = np.linalg.det(Dm) / 6.0
    return b, vol


def build(problem, alpha_hat=None, n_modes=None, weight_mode=None, modes=True, factor=True,
          affine_bones=False, bone_slack=1e-3):
    """Set up the oracle mesh for a ``workloads.Problem``.  ``factor=False``
    skips the sparse factorization (and the modes): the element formulas,
    ``L``, ``scatter_GtWF`` and ``gather_A`` still work, which is what checks
    at sizes the factorization would take too long for need."""
    alpha_hat = problem.alpha_hat if alpha_hat is None else alpha_hat
    if weight_mode is None:
        weight_mode = getattr(problem, "weight_mode", 0)
    n_modes = problem.n_modes if n_modes is None else n_modes
    rest = np.asarray(problem.rest_xyz, np.float64)
    tets = orient(rest, problem.tets)
    b, vol = hat_gradients(rest, tets)
    mu, lhat = mat.lame(problem.youngs, problem.poisson)
    group = np.asarray(problem.group, np.int64)
    musc = group >= 0
    mu_ref = float(mu[musc].min()) if musc.any() else float(mu.min())
    kf = mu_ref
    alpha = alpha_hat * mu_ref
    m = tets.shape[0]
    bone = (np.full(m, -1, np.int64) if getattr(problem, "bone", None) is None
            else np.asarray(problem.bone, np.int64))
    if weight_mode == 0:
        w = vol * mu / mu_ref
    elif weight_mode == 1:
        w = vol.copy()
    elif weight_mode == 2:
        w = np.where(bone >= 0, vol, vol * mu / mu_ref)
    else:
        raise ValueError("weight_mode")
    if affine_bones:
        # Sec. 3.3: the tets of each bone share one deformation gradient F_b,
        # tied to the continuous mesh by B_q q = B_F F with the slack eps_2 of
        # eq. kkt-matrix; eliminating the slack's multiplier adds the penalty
        # |G_i q - F_b|^2 / (2 |eps_2|) per bone tet (read relative to the
        # tet's volume-weighted ACAP term), and bones are not stiffness-weighted
        w = np.where(bone >= 0, vol * (1.0 + 1.0 / bone_slack), w)
    beta = alpha * w
    fiber = problem.fiber / np.linalg.norm(problem.fiber, axis=1, keepdims=True)
    n = rest.shape[0]
    # weighted Laplacian
    bb = np.einsum("ivd,iud->ivu", b, b) * w[:, None, None]
    rows = np.repeat(tets, 4, axis=1).reshape(-1)
    cols = np.tile(tets, (1, 4)).reshape(-1)
    L = sp.coo_matrix((bb.reshape(-1), (rows, cols)), shape=(n, n)).tocsr()
    pins = np.asarray(problem.pins, np.int64)
    isfree = np.ones(n, bool)
    isfree[pins] = False
    free = np.nonzero(isfree)[0]
    fpos = -np.ones(n, np.int64)
    fpos[free] = np.arange(free.size)
    Lff = L[free][:, free].tocsc()
    Lfp = L[free][:, pins].tocsr()
    lu = spla.splu(Lff, permc_spec="MMD_AT_PLUS_A") if factor else None
    M = Mesh(rest=rest, tets=tets, b=b, vol=vol, mu=mu, lhat=lhat, fiber=fiber,
             group=group, bone=bone, w=w, beta=beta, alpha=alpha, mu_ref=mu_ref, kf=kf,
             pins=pins, pin_xyz=np.asarray(problem.pin_xyz, np.float64),
             free=free, fpos=fpos, L=L, Lff=Lff, Lfp=Lfp, lu=lu)
    # reduced variables: one per non-bone tet, one per bone (affine bones)
    if affine_bones and (bone >= 0).any():
        ids = np.unique(bone[bone >= 0])
        nonb = np.nonzero(bone < 0)[0]
        red_of = np.empty(m, np.int64)
        red_of[nonb] = np.arange(nonb.size)
        for k, b in enumerate(ids):
            red_of[bone == b] = nonb.size + k
        M.red_of, M.m_red = red_of, nonb.size + ids.size
    else:
        M.red_of, M.m_red = None, m
    if n_modes < 0:                       # default: 48 modes, capped by the mesh
        n_modes = min(48, 3 * (free.size - 1))
    if modes and factor and n_modes > 0:
        compute_modes(M, n_modes // 3)
    return M


def compute_modes(M, k):
    """Lowest k eigenpairs of L_ff (shift-invert about 0)."""
    nf = M.free.size
    if k >= nf - 1:
        w, V = np.linalg.eigh(M.Lff.toarray())
        w, V = w[:k], V[:, :k]
    else:
        # shift-invert about 0 with the factor already held (the same operator
        # L_ff^{-1} that eigsh would factor again itself)
        nf3 = M.free.size
        OPinv = spla.LinearOperator((nf3, nf3), matvec=lambda x: M.lu.solve(np.asarray(x, np.float64)),
                                    dtype=np.float64)
        w, V = spla.eigsh(M.Lff, k=k, sigma=0.0, which="LM", OPinv=OPinv)
    order = np.argsort(w)
    M.nu = w[order]
    M.phi = V[:, order].T.copy()
    return M


def activation_per_element(M, a):
    a = np.asarray(a, np.float64)
    out = np.zeros(M.m)
    musc = M.group >= 0
    out[musc] = a[M.group[musc]]
    return out


def gather_A(M, q):
    """A_i = sum_v q_v b_{i,v}^T, [m,3,3] with A[c,d] = sum_v q[v,c] b[v,d]."""
    return np.einsum("ivc,ivd->icd", q[M.tets], M.b)


def scatter_GtWF(M, F):
    """r[v,c] = sum_{i ∋ v} w_i b_{i,v} . F_i[c,:]  (= G^T W F), [n,3]."""
    contrib = np.einsum("i,ivd,icd->ivc", M.w, M.b, F)
    r = np.zeros((M.n, 3))
    np.add.at(r, M.tets.reshape(-1), contrib.reshape(-1, 3))
    return r


def acap_solve(M, F, pinned=True):
    """q*(F): nearest continuous mesh (eq. acap) with pins at their targets
    (``pinned=False`` gives the homogeneous solve with zero pin values)."""
    r = scatter_GtWF(M, F)
    q = np.zeros((M.n, 3))
    if pinned:
        q[M.pins] = M.pin_xyz
        rhs = r[M.free] - M.Lfp @ M.pin_xyz
    else:
        rhs = r[M.free]
    q[M.free] = M.lu.solve(np.asarray(rhs, order="F"))
    return q


def acap_energy(M, q, F):
    D = gather_A(M, q) - F
    return 0.5 * np.sum(M.w * np.einsum("icd,icd->i", D, D))


def set_external_forces(M, f):
    """Constant external vertex forces f [n,3] (None removes them).  Also keeps
    v = L_ff^{-1} f_f, the vertex field whose weighted gradient w_i G_i v is the
    derivative of f . q*(F) with respect to F_i."""
    if f is None:
        M.fext = M.vext = None
        return M
    f = np.array(f, dtype=np.float64).reshape(M.n, 3)
    M.fext = f
    v = np.zeros((M.n, 3))
    v[M.free] = M.lu.solve(np.asarray(f[M.free], order="F"))
    M.vext = v
    return M


def work(M, q):
    """External work W(q) = sum over free vertices of f . q (0 without forces)."""
    if M.fext is None:
        return 0.0
    return math.fsum((M.fext[M.free] * q[M.free]).reshape(-1))
