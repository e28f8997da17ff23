"""Element energy of the oracle (FP64, vectorized over elements).

Isotropic part: stable Neo-Hookean (the paper uses it for Psi_iso, Sec. 3 and
Sec. 3.1, citing Smith et al. 2018 without printing it).  Reading used here:

    Psi_iso(F) = mu/2 (|F|^2 - 3) - mu (J - 1) + lhat/2 (J - 1)^2,
    J = det F,  lhat = lambda + mu,

which is zero with zero stress at F = I and reproduces the Lame constants
(mu, lambda) at small strain.

Fiber part: linear activation along a unit fiber u (Sec. 3.1):

    Psi_fiber(F) = a * k_f * u^T F^T F u,   a >= 0,

with the stress scale k_f carried separately because the activations are
dimensionless in [0, 1].

All second derivatives use row-major vectorization: index (c, d) -> 3c + d.
"""
from __future__ import annotations

import numpy as np

SQ2 = np.sqrt(2.0)

# Levi-Civita symbol
EPS = np.zeros((3, 3, 3))
EPS[0, 1, 2] = EPS[1, 2, 0] = EPS[2, 0, 1] = 1.0
EPS[0, 2, 1] = EPS[2, 1, 0] = EPS[1, 0, 2] = -1.0

# Orthonormal basis of symmetric 3x3 matrices:
#   v(X) = (X11, X22, X33, sqrt2 X12, sqrt2 X13, sqrt2 X23)
BASIS = np.zeros((6, 3, 3))
BASIS[0, 0, 0] = BASIS[1, 1, 1] = BASIS[2, 2, 2] = 1.0
for _l, (_a, _b) in zip((3, 4, 5), ((0, 1), (0, 2), (1, 2))):
    BASIS[_l, _a, _b] = BASIS[_l, _b, _a] = 1.0 / SQ2


def lame(youngs, poisson):
    """(mu, lhat = lambda + mu) from Young's modulus and Poisson ratio."""
    E = np.asarray(youngs, np.float64)
    nu = np.asarray(poisson, np.float64)
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam + mu


def sym_to_vec(X):
    """v(sym X) for [..., 3, 3]."""
    return np.einsum("lab,...ab->...l", BASIS, X)


def vec_to_sym(s):
    return np.einsum("...l,lab->...ab", s, BASIS)


def cof(F):
    """Cofactor matrix, cof(F)_cd = dJ/dF_cd, for [..., 3, 3]."""
    return 0.5 * np.einsum("ceg,dfh,...ef,...gh->...cd", EPS, EPS, F, F)


def psi(F, mu, lhat, a, kf, u):
    """Element energy density Psi(F) for arrays F [m,3,3], per-element
    mu, lhat, activation a, fiber scale kf and fibers u [m,3]."""
    J = np.linalg.det(F)
    I1 = np.einsum("...ab,...ab->...", F, F)
    Fu = np.einsum("...ab,...b->...a", F, u)
    return (0.5 * mu * (I1 - 3.0) - mu * (J - 1.0) + 0.5 * lhat * (J - 1.0) ** 2
            + a * kf * np.einsum("...a,...a->...", Fu, Fu))


def pk1(F, mu, lhat, a, kf, u):
    """First Piola-Kirchhoff stress P = dPsi/dF."""
    J = np.linalg.det(F)
    C = cof(F)
    Fu = np.einsum("...ab,...b->...a", F, u)
    return (mu[..., None, None] * F + (lhat * (J - 1.0) - mu)[..., None, None] * C
            + 2.0 * (a * kf)[..., None, None] * np.einsum("...a,...b->...ab", Fu, u))


def hess_J(F):
    """d^2 J / dF_cd dF_c'd' as [..., 9, 9]."""
    H = np.einsum("cpe,dqf,...ef->...cdpq", EPS, EPS, F)
    return H.reshape(F.shape[:-2] + (9, 9))


def hess(F, mu, lhat, a, kf, u):
    """d^2 Psi / dF^2 as [..., 9, 9] (row-major vectorization)."""
    J = np.linalg.det(F)
    c = cof(F).reshape(F.shape[:-2] + (9,))
    I9 = np.eye(9)
    fib = np.einsum("ab,...c,...d->...acbd", np.eye(3), u, u).reshape(F.shape[:-2] + (9, 9))
    return (mu[..., None, None] * I9
            + lhat[..., None, None] * np.einsum("...i,...j->...ij", c, c)
            + (lhat * (J - 1.0) - mu)[..., None, None] * hess_J(F)
            + 2.0 * (a * kf)[..., None, None] * fib)


def psi_s(s, mu, lhat, a, kf, u):
    """Psi at the symmetric stretch S = S(s) (rotation drops out: Psi(RS) = Psi(S))."""
    return psi(vec_to_sym(s), mu, lhat, a, kf, u)


def grad_s(s, mu, lhat, a, kf, u):
    """dPsi/ds_l = <P(S), E_l>: chain rule through the linear map s -> S."""
    P = pk1(vec_to_sym(s), mu, lhat, a, kf, u)
    return np.einsum("lab,...ab->...l", BASIS, P)


def hess_s(s, mu, lhat, a, kf, u):
    """d^2 Psi / ds_l ds_l' = E_l : d^2Psi(S) : E_l'."""
    H9 = hess(vec_to_sym(s), mu, lhat, a, kf, u)
    Bv = BASIS.reshape(6, 9)
    return np.einsum("li,...ij,kj->...lk", Bv, H9, Bv)


def polar_rotation(X):
    """Rotation factor of X: argmax_{R in SO(3)} tr(R^T X) via the SVD
    X = U Sigma V^T, R = U diag(1, 1, det(U V^T)) V^T."""
    U, _, Vt = np.linalg.svd(X)
    d = np.linalg.det(np.einsum("...ab,...bc->...ac", U, Vt))
    D = np.zeros(X.shape)
    D[..., 0, 0] = 1.0
    D[..., 1, 1] = 1.0
    D[..., 2, 2] = d
    return np.einsum("...ab,...bc,...cd->...ad", U, D, Vt)


def clamp_psd(H):
    """Projection onto the PSD cone: eigenvalues below zero set to zero."""
    w, V = np.linalg.eigh(H)
    return np.einsum("...ij,...j,...kj->...ik", V, np.maximum(w, 0.0), V)
