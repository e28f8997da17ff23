"""Contact loop (oracle part O7): the collision block of Algorithm 1 (Sec. 3.5).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline use this module.

After the line search of an iteration, Algorithm 1 resolves contacts of the
continuous vertices before the next gradient: contact forces are turned into a
step of the deformation gradients through the quasi-Newton Hessian (the
Woodbury inverse of the iteration) and the continuous mesh is re-solved, until
the contact forces stop changing.  The collision method the paper cites is
not described there, so analytic obstacles stand in for the colliding bodies:

* half-spaces, rows (n, b) with a unit normal n: a vertex x penetrates where
  n . x < b, by depth b - n . x, and is pushed along +n;
* spheres, rows (c, r): x penetrates where |x - c| < r, by r - |x - c|, and is
  pushed along (x - c) / |x - c| (a vertex exactly at c has no direction and
  gets no force).

Each penetrating free vertex receives the penalty force k * depth along the
push direction (the negative gradient of 1/2 k depth^2); pinned vertices get
none.  One round, with f the force increment of the current q:

    nu = w G L_ff^{-1} f            (the field of f . q*(F), eq. external-forces)
    z  = Htilde^{-1} nu             (the iteration's Woodbury inverse)
    F <- F + z,   q <- q*(F)        (an ACAP solve; q* is affine in F)

and rounds repeat until |f|_2 <= tol or max_rounds are done.
"""
from __future__ import annotations

import math

import numpy as np

from . import mesh as msh


def obstacles(planes=None, spheres=None, stiffness=1.0, tol=1e-8, max_rounds=8):
    """The contact description: planes [np,4], spheres [ns,4], penalty k,
    tolerance on |f|_2 per round and the round limit."""
    P = np.zeros((0, 4)) if planes is None else np.array(planes, dtype=np.float64).reshape(-1, 4)
    S = np.zeros((0, 4)) if spheres is None else np.array(spheres, dtype=np.float64).reshape(-1, 4)
    return dict(planes=P, spheres=S, k=float(stiffness), tol=float(tol), max_rounds=int(max_rounds))


def penetrations(x, contact):
    """Per vertex and obstacle: depth >= 0 and the unit push direction.
    Returns (depth [n, no], dirs [n, no, 3]) over planes then spheres."""
    n = x.shape[0]
    P, S = contact["planes"], contact["spheres"]
    depth = np.zeros((n, len(P) + len(S)))
    dirs = np.zeros((n, len(P) + len(S), 3))
    for k, (nx, ny, nz, b) in enumerate(P):
        nv = np.array([nx, ny, nz])
        d = b - x @ nv
        depth[:, k] = np.maximum(d, 0.0)
        dirs[:, k] = nv
    for k, (cx, cy, cz, r) in enumerate(S):
        rel = x - np.array([cx, cy, cz])
        dist = np.linalg.norm(rel, axis=1)
        inside = (dist < r) & (dist > 0.0)  # no push direction at the center
        j = len(P) + k
        depth[inside, j] = r - dist[inside]
        dirs[inside, j] = rel[inside] / dist[inside, None]
    return depth, dirs


def penalty_energy(M, q, contact):
    """1/2 k sum depth^2 over free vertices and obstacles."""
    depth, _ = penetrations(q, contact)
    return 0.5 * contact["k"] * math.fsum((depth[M.free] ** 2).reshape(-1))


def forces(M, q, contact):
    """Penalty forces [n,3] at the free vertices (zero at pins)."""
    depth, dirs = penetrations(q, contact)
    f = contact["k"] * np.einsum("no,noc->nc", depth, dirs)
    f[M.pins] = 0.0
    return f


def force_field(M, f):
    """nu_i = w_i G_i L_ff^{-1} f: dF-gradient of f . q*(F)."""
    v = np.zeros((M.n, 3))
    v[M.free] = M.lu.solve(np.asarray(f[M.free], order="F"))
    return M.w[:, None, None] * msh.gather_A(M, v)


def contact_loop(M, F, q, hinv, contact):
    """The rounds after one accepted step.  hinv(nu [m,9]) -> [m,9] applies the
    iteration's Htilde^{-1}.  Returns (F, q, rounds)."""
    Zc = np.zeros_like(F)
    rounds = 0
    for _ in range(contact["max_rounds"]):
        f = forces(M, q, contact)
        if math.sqrt(math.fsum((f * f).reshape(-1))) <= contact["tol"]:
            break
        nu = force_field(M, f)
        z = hinv(nu.reshape(M.m, 9)).reshape(M.m, 3, 3)
        Zc = Zc + z
        q = q + msh.acap_solve(M, z, pinned=False)
        rounds += 1
    return F + Zc, q, rounds
