"""Pins of the oracle's element energy (Sec. 3.1 energy choices) against facts
fixed by the paper and by elasticity textbooks, not against its own formulas."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import material as mat
from oracle import emu
from paper_2006_08821_amd.workloads import random_rotation

RNG = np.random.default_rng(1)
E_MUS, NU = 6e4, 0.45


def _params(m, a=0.0):
    mu, lhat = mat.lame(np.full(m, E_MUS), np.full(m, NU))
    u = RNG.normal(size=(m, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    return mu, lhat, np.full(m, a), mu.copy(), u


def test_rest_is_stress_free():
    mu, lhat, a, kf, u = _params(4)
    F = np.tile(np.eye(3), (4, 1, 1))
    assert np.allclose(mat.psi(F, mu, lhat, a, kf, u), 0.0, atol=1e-12)
    assert np.allclose(mat.pk1(F, mu, lhat, a, kf, u), 0.0, atol=1e-9)


def test_small_strain_matches_linear_elasticity():
    # textbook Lame constants from (E, nu); second variation of Psi at I must be
    # mu tr(eps^2) + lambda/2 (tr eps)^2 for symmetric strains
    lam_tb = E_MUS * NU / ((1 + NU) * (1 - 2 * NU))
    mu_tb = E_MUS / (2 * (1 + NU))
    mu, lhat, a, kf, u = _params(1)
    for _ in range(5):
        e = RNG.normal(size=(3, 3))
        e = 0.5 * (e + e.T) * 1e-5
        lin = mu_tb * np.trace(e @ e) + 0.5 * lam_tb * np.trace(e) ** 2
        val = mat.psi((np.eye(3) + e)[None], mu, lhat, a, kf, u)[0]
        assert abs(val - lin) <= 1e-4 * lin


def test_frame_invariance_and_isotropy():
    mu, lhat, a, kf, u = _params(6, a=0.7)
    F = np.eye(3) + 0.3 * RNG.normal(size=(6, 3, 3))
    Q = np.stack([random_rotation(RNG) for _ in range(6)])
    base = mat.psi(F, mu, lhat, a, kf, u)
    assert np.allclose(mat.psi(Q @ F, mu, lhat, a, kf, u), base, rtol=1e-12)
    zero = np.zeros(6)
    iso = mat.psi(F, mu, lhat, zero, kf, u)
    assert np.allclose(mat.psi(F @ Q, mu, lhat, zero, kf, u), iso, rtol=1e-11)


def test_fiber_term_special_case():
    # uniaxial stretch along the fiber: a * kf * |F u|^2 = a * kf * stretch^2
    mu, lhat, _, kf, _ = _params(1)
    u = np.array([[0.0, 0.0, 1.0]])
    for lam in (0.7, 1.0, 1.3):
        F = np.diag([1.0, 1.0, lam])[None]
        d = (mat.psi(F, mu, lhat, np.array([0.4]), kf, u) - mat.psi(F, mu, lhat, np.zeros(1), kf, u))
        assert np.allclose(d, 0.4 * kf * lam ** 2, rtol=1e-13)


def test_cofactor_is_adjugate_transpose():
    F = np.eye(3) + 0.4 * RNG.normal(size=(5, 3, 3))
    ref = np.linalg.det(F)[:, None, None] * np.transpose(np.linalg.inv(F), (0, 2, 1))
    assert np.allclose(mat.cof(F), ref, rtol=1e-12, atol=1e-14)


def test_stress_and_hessian_finite_differences():
    mu, lhat, a, kf, u = _params(3, a=0.8)
    F = np.eye(3) + 0.25 * RNG.normal(size=(3, 3, 3))
    P = mat.pk1(F, mu, lhat, a, kf, u)
    H = mat.hess(F, mu, lhat, a, kf, u)
    h = 1e-6
    for k in range(9):
        E = np.zeros(9)
        E[k] = h
        E = E.reshape(3, 3)
        fd = (mat.psi(F + E, mu, lhat, a, kf, u) - mat.psi(F - E, mu, lhat, a, kf, u)) / (2 * h)
        assert np.allclose(fd, P.reshape(3, 9)[:, k], rtol=1e-7, atol=1e-3)
        fdP = (mat.pk1(F + E, mu, lhat, a, kf, u) - mat.pk1(F - E, mu, lhat, a, kf, u)) / (2 * h)
        assert np.allclose(fdP.reshape(3, 9), H[:, :, k], rtol=1e-6, atol=1e-2)


def test_s_basis_is_orthonormal():
    B = mat.BASIS.reshape(6, 9)
    assert np.allclose(B @ B.T, np.eye(6))
    Y = emu.YBASIS
    assert np.allclose(Y.T @ Y, np.eye(9))


def test_polar_rotation_properties():
    X = 1.2 * np.eye(3) + 0.5 * RNG.normal(size=(20, 3, 3))
    R = mat.polar_rotation(X)
    assert np.allclose(np.einsum("iab,iac->ibc", R, R), np.eye(3), atol=1e-13)
    assert np.allclose(np.linalg.det(R), 1.0, atol=1e-13)
    S = np.einsum("iba,ibc->iac", R, X)
    assert np.allclose(S, np.transpose(S, (0, 2, 1)), atol=1e-12)
    pos = np.linalg.det(X) > 0
    for i in np.nonzero(pos)[0]:
        Rp, _ = sla.polar(X[i])
        assert np.allclose(R[i], Rp, atol=1e-12)
    # maximizer of tr(R^T X) over SO(3), also for det X < 0
    for i in np.nonzero(~pos)[0][:3]:
        best = np.trace(R[i].T @ X[i])
        for _ in range(200):
            Q = random_rotation(RNG)
            assert np.trace(Q.T @ X[i]) <= best + 1e-12


def test_clamp_matches_eigendecomposition():
    A = RNG.normal(size=(10, 6, 6))
    A = A + np.transpose(A, (0, 2, 1))
    C = mat.clamp_psd(A)
    w = np.linalg.eigvalsh(C)
    assert w.min() > -1e-12
    assert np.allclose(np.linalg.eigvalsh(A).clip(0), w, atol=1e-12)
    P = A @ np.transpose(A, (0, 2, 1))
    assert np.allclose(mat.clamp_psd(P), P, rtol=1e-10, atol=1e-10)


def test_isotropic_hessian_splits_in_rotated_frame():
    # For an isotropic energy the Hessian in the frame dF = R dX (R the polar
    # rotation) has no coupling between symmetric and skew dX: the design's
    # 6x6 + 3x3 block structure loses nothing for the isotropic part.
    mu, lhat, _, kf, u = _params(8)
    F = np.eye(3) + 0.4 * RNG.normal(size=(8, 3, 3))
    H = mat.hess(F, mu, lhat, np.zeros(8), kf, u)
    T = emu.frame_basis(mat.polar_rotation(F))
    HY = np.einsum("iab,ibc,icd->iad", np.transpose(T, (0, 2, 1)), H, T)
    scale = np.abs(HY).max()
    assert np.abs(HY[:, :6, 6:]).max() < 1e-10 * scale
    # the fiber term does couple them (so the split is an approximation there)
    Hf = mat.hess(F, mu, lhat, np.ones(8), kf, u)
    HYf = np.einsum("iab,ibc,icd->iad", np.transpose(T, (0, 2, 1)), Hf, T)
    assert np.abs(HYf[:, :6, 6:]).max() > 1e-3 * scale
