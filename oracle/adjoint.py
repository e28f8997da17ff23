"""q-space adjoint of the equilibrium w.r.t. muscle activations (oracle part O6).

At a minimizer q of Ehat(q) = sum_i e_i(G_i q; a) (the Moreau-envelope form of
the separated energy, see ``fem``), the implicit function theorem gives

    dq/da_g = -K^{-1} d(grad Ehat)/da_g,     K = sum_i G_i^T hess_A e_i G_i,

so for a loss L(q): dL/da_g = -lambda^T d(grad Ehat)/da_g with K lambda = dL/dq.
With the prox X* of each element (vol P(X*) + beta (X* - A) = 0) and the fiber
term a k_f |X u|^2 (Sec. 3.1):

    d(grad_A e_i)/da = beta (vol d2Psi(X*) + beta I)^{-1} vol 2 k_f X* u u^T.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import fem
from . import material as mat
from . import mesh as msh


def marker_loss(q, markers, target):
    d = q[markers] - target
    return float(np.sum(d * d)), 2.0 * d


def activation_gradient(M, a, q, markers, target):
    """dL/da (per group) at the equilibrium q for L = sum |q_m - target_m|^2."""
    a_el = msh.activation_per_element(M, a)
    A = msh.gather_A(M, q)
    X, H = fem.prox(M, A, a_el)
    Hinv = np.linalg.inv(H)
    b2 = M.beta[:, None, None]
    He = b2 * np.eye(9) - b2 ** 2 * Hinv
    He = 0.5 * (He + np.transpose(He, (0, 2, 1)))
    K, fdof = fem._assemble(M, He)
    L, dLdq_m = marker_loss(q, markers, target)
    dLdq = np.zeros((M.n, 3))
    np.add.at(dLdq, markers, dLdq_m)
    lam = spla.spsolve(K, dLdq[M.free].reshape(-1))
    lam_full = np.zeros((M.n, 3))
    lam_full[M.free] = lam.reshape(-1, 3)
    lamA = msh.gather_A(M, lam_full)                  # G_i lambda
    dP = 2.0 * M.kf * np.einsum("icd,id,ie->ice", X, M.fiber, M.fiber)
    dX = np.einsum("iab,ib->ia", Hinv, (M.vol[:, None, None] * dP).reshape(-1, 9)).reshape(-1, 3, 3)
    dgradA = M.beta[:, None, None] * dX               # d(grad_A e_i)/da_i
    per_el = np.einsum("icd,icd->i", lamA, dgradA)
    n_groups = int(np.max(M.group)) + 1 if np.any(M.group >= 0) else 0
    out = np.zeros(len(np.atleast_1d(a)))
    for g in range(n_groups):
        out[g] = -np.sum(per_el[M.group == g])
    return L, out
