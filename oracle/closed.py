"""Closed-form special cases (oracle part O5).

Homogeneous fiber contraction: a homogeneous muscle with a uniform fiber
u = e_z and uniform activation a.  The element energy (Sec. 3.1: stable
Neo-Hookean plus a * k_f * |F u|^2) restricted to F = diag(t, t, f) is

    psi(t, f) = mu/2 (2t^2 + f^2 - 3) - mu (t^2 f - 1) + lhat/2 (t^2 f - 1)^2 + a kf f^2.

Its stationary point F0 = diag(t, t, f) is found by a 2-D Newton iteration.  If
the pinned vertices sit at F0 Q, the uniform field F_i = F0, q = F0 Q has zero
ACAP energy and every element at an energy minimum, so it is a global minimizer
of the separated energy for every alpha.
"""
from __future__ import annotations

import numpy as np


def fiber_stretch(mu, lhat, a, kf, t0=1.0, f0=1.0, tol=1e-15, max_iters=100):
    """Return (t, f, psi) at the stationary point of psi(t, f)."""
    x = np.array([t0, f0], dtype=np.float64)

    def grad_hess(x):
        t, f = x
        J = t * t * f
        dJ = np.array([2 * t * f, t * t])
        d2J = np.array([[2 * f, 2 * t], [2 * t, 0.0]])
        g = np.array([2 * mu * t, mu * f + 2 * a * kf * f]) + (lhat * (J - 1) - mu) * dJ
        H = (np.diag([2 * mu, mu + 2 * a * kf]) + lhat * np.outer(dJ, dJ)
             + (lhat * (J - 1) - mu) * d2J)
        return g, H

    for _ in range(max_iters):
        g, H = grad_hess(x)
        dx = np.linalg.solve(H, g)
        x = x - dx
        if np.max(np.abs(dx)) < tol:
            break
    t, f = x
    J = t * t * f
    psi = (0.5 * mu * (2 * t * t + f * f - 3) - mu * (J - 1) + 0.5 * lhat * (J - 1) ** 2
           + a * kf * f * f)
    return float(t), float(f), float(psi)
