"""Seeded synthetic workloads for the deformation-space quasi-static solve.

This module only builds inputs: rest meshes, materials, fiber fields, muscle
groups, pins and activation schedules.  It holds none of the method's
arithmetic (no orientation fix, no deformation gradients, no energies), so the
CPU oracle and the GPU library both consume the same arrays and share nothing
else.

Mesh construction (stand-ins for the paper's TetWild meshes of Sec. 3.6, which
are not available):

* Kuhn/Freudenthal split of an ``nx x ny x nz`` cube grid, 6 tets per cube: for
  every permutation ``pi`` of the three axes the tet is the path
  ``v000 -> +e_pi0 -> +e_pi1 -> +e_pi2``.  Vertex id of grid point (i, j, k) is
  ``(k*(ny+1) + j)*(nx+1) + i``.  Tets are emitted in raw path order, so half of
  them have a negative rest volume; the consumer fixes orientation.
* Material roles follow Sec. 3.6 (bone / tendon / muscle).  The limb layout is a
  radial bone core, tendon end caps and muscle elsewhere.
* Fibers: a helical field (30 deg pitch, 5 deg seeded jitter) standing in for
  the heat-equation field of Sec. 3.6.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import Dict, List, Optional

import numpy as np

H_EDGE = 0.01          # cube edge (m)
# ACAP weighting of the limb workloads (bone core, tendon caps): volume
# weights.  Stiffness-proportional weights on the 1.7e3x tendon and 1.7e5x bone
# contrast of these inputs stall the iteration (see the design notes).
LIMB_WEIGHT_MODE = 1
E_MUSCLE = 6.0e4       # Pa
E_TENDON = 1.0e8
E_BONE = 1.0e10
NU = 0.45


@dataclasses.dataclass
class Problem:
    """Inputs of one quasi-static solve (host arrays, user vertex order)."""
    name: str
    rest_xyz: np.ndarray          # [n,3] float64
    tets: np.ndarray              # [m,4] int32, raw (unoriented) vertex order
    youngs: np.ndarray            # [m] float64
    poisson: np.ndarray           # [m] float64
    fiber: np.ndarray             # [m,3] float64 (unit)
    group: np.ndarray             # [m] int32, -1 = passive
    pins: np.ndarray              # [p] int32
    pin_xyz: np.ndarray           # [p,3] float64
    activation: np.ndarray        # [n_groups] float64
    dims: tuple = ()
    alpha_hat: float = 10.0
    n_modes: int = -1               # -1: library default (48, capped by the mesh)
    extra: dict = dataclasses.field(default_factory=dict)
    bone: Optional[np.ndarray] = None  # [m] int32 bone id per tet, -1 = not bone (None: no bones)
    weight_mode: int = 0            # ACAP weights: 0 stiffness, 1 volume, 2 paper (bone by volume)

    @property
    def n_vertices(self) -> int:
        return int(self.rest_xyz.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])

    @property
    def n_groups(self) -> int:
        return int(self.activation.shape[0])

    def copy(self) -> "Problem":
        return dataclasses.replace(
            self, **{f.name: (getattr(self, f.name).copy()
                              if isinstance(getattr(self, f.name), np.ndarray)
                              else getattr(self, f.name))
                     for f in dataclasses.fields(self)})


def grid_vertices(nx: int, ny: int, nz: int, h: float = H_EDGE) -> np.ndarray:
    i, j, k = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1),
                          indexing="ij")
    # flatten in id order: id = (k*(ny+1)+j)*(nx+1)+i
    xyz = np.stack([i, j, k], axis=-1).transpose(2, 1, 0, 3).reshape(-1, 3)
    return xyz.astype(np.float64) * h


def kuhn_tets(nx: int, ny: int, nz: int) -> np.ndarray:
    def vid(i, j, k):
        return (k * (ny + 1) + j) * (nx + 1) + i
    perms = list(itertools.permutations(range(3)))
    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    # cube order: k slowest, then j, then i
    ci = ci.transpose(2, 1, 0).reshape(-1)
    cj = cj.transpose(2, 1, 0).reshape(-1)
    ck = ck.transpose(2, 1, 0).reshape(-1)
    out = np.empty((ci.size, 6, 4), dtype=np.int64)
    for p, perm in enumerate(perms):
        pos = np.stack([ci, cj, ck], axis=1).copy()
        out[:, p, 0] = vid(pos[:, 0], pos[:, 1], pos[:, 2])
        for s in range(3):
            pos[:, perm[s]] += 1
            out[:, p, s + 1] = vid(pos[:, 0], pos[:, 1], pos[:, 2])
    return out.reshape(-1, 4).astype(np.int32)


def _centroids(xyz: np.ndarray, tets: np.ndarray) -> np.ndarray:
    return xyz[tets].mean(axis=1)


def helical_fibers(cent: np.ndarray, axis_xy, rng: np.random.Generator,
                   pitch_deg: float = 30.0, jitter_deg: float = 5.0) -> np.ndarray:
    """Helix about the z axis through ``axis_xy``: u0 = cos(p) e_z + sin(p) e_theta,
    then a seeded tilt by delta ~ U(-jitter, jitter) about a random axis
    perpendicular to u0 (all azimuths drawn first, then all tilts)."""
    m = cent.shape[0]
    dx = cent[:, 0] - axis_xy[0]
    dy = cent[:, 1] - axis_xy[1]
    r = np.hypot(dx, dy)
    theta = np.arctan2(dy, dx)
    et = np.stack([-np.sin(theta), np.cos(theta), np.zeros(m)], axis=1)
    at_axis = r < 1e-12
    et[at_axis] = (1.0, 0.0, 0.0)
    ez = np.array([0.0, 0.0, 1.0])
    p = math.radians(pitch_deg)
    u0 = math.cos(p) * ez[None, :] + math.sin(p) * et
    er = np.cross(et, ez[None, :])                 # radial, perpendicular to u0
    e2 = np.cross(u0, er)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=m)
    delta = np.radians(rng.uniform(-jitter_deg, jitter_deg, size=m))
    k = np.cos(phi)[:, None] * er + np.sin(phi)[:, None] * e2
    u = u0 * np.cos(delta)[:, None] + np.cross(k, u0) * np.sin(delta)[:, None]
    return u / np.linalg.norm(u, axis=1, keepdims=True)


def _face_pins(xyz: np.ndarray, axis: int, value: float) -> np.ndarray:
    return np.nonzero(np.abs(xyz[:, axis] - value) < 1e-9)[0].astype(np.int32)


def box_beam(nx: int = 4, ny: int = 4, nz: int = 16, activation: float = 0.5,
             youngs: float = E_MUSCLE, name: str = "box_beam") -> Problem:
    """Homogeneous muscle box, fibers along z, one group, z=0 face pinned at rest."""
    xyz = grid_vertices(nx, ny, nz)
    tets = kuhn_tets(nx, ny, nz)
    m = tets.shape[0]
    pins = _face_pins(xyz, 2, 0.0)
    return Problem(
        name=name, rest_xyz=xyz, tets=tets,
        youngs=np.full(m, youngs), poisson=np.full(m, NU),
        fiber=np.tile([0.0, 0.0, 1.0], (m, 1)), group=np.zeros(m, np.int32),
        pins=pins, pin_xyz=xyz[pins].copy(), activation=np.array([activation]),
        dims=(nx, ny, nz))


def limb_materials(xyz: np.ndarray, tets: np.ndarray, nx: int, ny: int, nz: int):
    """Radial bands: bone core r<0.2 (of the half-width), tendon where the
    centroid lies in the outer 10% of the length at either end, muscle elsewhere.
    Returns (youngs, role) with role 0 muscle, 1 tendon, 2 bone."""
    cent = _centroids(xyz, tets)
    cx, cy = nx * H_EDGE / 2, ny * H_EDGE / 2
    L = nz * H_EDGE
    r = np.hypot(cent[:, 0] - cx, cent[:, 1] - cy) / (nx * H_EDGE / 2)
    role = np.zeros(tets.shape[0], np.int32)
    tendon = (cent[:, 2] < 0.1 * L) | (cent[:, 2] > 0.9 * L)
    role[tendon] = 1
    role[r < 0.2] = 2
    youngs = np.where(role == 2, E_BONE, np.where(role == 1, E_TENDON, E_MUSCLE))
    return youngs.astype(np.float64), role, cent


def quadrant_groups(cent: np.ndarray, role: np.ndarray, nx, ny, nz, split_z: bool) -> np.ndarray:
    cx, cy = nx * H_EDGE / 2, ny * H_EDGE / 2
    q = (cent[:, 0] >= cx).astype(np.int32) + 2 * (cent[:, 1] >= cy).astype(np.int32)
    if split_z:
        q = q + 4 * (cent[:, 2] >= nz * H_EDGE / 2).astype(np.int32)
    return np.where(role == 0, q, -1).astype(np.int32)


def limb(nx: int = 20, ny: int = 20, nz: int = 80, n_groups: int = 1, seed: int = 0,
         activation: Optional[np.ndarray] = None, name: str = "limb") -> Problem:
    """Heterogeneous limb: bone core, tendon caps, muscle with helical fibers,
    z=0 face pinned.  ``n_groups`` is 1, 4 (azimuth quadrants) or 8 (quadrants x
    lower/upper half)."""
    xyz = grid_vertices(nx, ny, nz)
    tets = kuhn_tets(nx, ny, nz)
    youngs, role, cent = limb_materials(xyz, tets, nx, ny, nz)
    rng = np.random.default_rng(seed)
    fiber = helical_fibers(cent, (nx * H_EDGE / 2, ny * H_EDGE / 2), rng)
    if n_groups == 1:
        group = np.where(role == 0, 0, -1).astype(np.int32)
    elif n_groups == 4:
        group = quadrant_groups(cent, role, nx, ny, nz, split_z=False)
    elif n_groups == 8:
        group = quadrant_groups(cent, role, nx, ny, nz, split_z=True)
    else:
        raise ValueError("n_groups must be 1, 4 or 8")
    pins = _face_pins(xyz, 2, 0.0)
    act = np.zeros(n_groups) if activation is None else np.asarray(activation, np.float64)
    bone = np.where(role == 2, 0, -1).astype(np.int32)
    return Problem(name=name, rest_xyz=xyz, tets=tets, youngs=youngs,
                   poisson=np.full(tets.shape[0], NU), fiber=fiber, group=group,
                   pins=pins, pin_xyz=xyz[pins].copy(), activation=act,
                   dims=(nx, ny, nz), extra={"role": role}, bone=bone,
                   weight_mode=LIMB_WEIGHT_MODE)


def heterogeneous_limb_ramp(steps: int = 20, nx=20, ny=20, nz=80) -> tuple:
    """Heterogeneous limb with one muscle group and the activation ramp
    a_t = t/steps, t = 1..steps (warm-started frames)."""
    p = limb(nx, ny, nz, n_groups=1, name=f"limb{nx}x{ny}x{nz}")
    ramp = [np.array([t / steps]) for t in range(1, steps + 1)]
    return p, ramp


def hinge_limb(nx: int = 40, ny: int = 40, nz: int = 160, frames: int = 60, seed: int = 0):
    """Two bones joined at mid-length by a revolute joint.  The bone core splits
    at z = L/2: mid-plane vertices used by upper-bone tets are duplicated, except
    those on the hinge line {y = centre, z = L/2}, which stay shared and are
    pinned.  Four azimuth-quadrant muscle groups; per-frame activations
    a ~ U[0,1]^4 drawn from ``seed``."""
    p = limb(nx, ny, nz, n_groups=4, seed=seed, name=f"hinge{nx}x{ny}x{nz}")
    xyz, tets = p.rest_xyz, p.tets.copy()
    role = p.extra["role"]
    L = nz * H_EDGE
    cent = _centroids(xyz, tets)
    upper_bone = (role == 2) & (cent[:, 2] > L / 2)
    mid = np.abs(xyz[:, 2] - L / 2) < 1e-9
    hinge = mid & (np.abs(xyz[:, 1] - ny * H_EDGE / 2) < 1e-9)
    used = np.unique(tets[upper_bone])
    dup_src = used[mid[used] & ~hinge[used]]
    new_id = np.full(xyz.shape[0], -1, np.int64)
    new_id[dup_src] = xyz.shape[0] + np.arange(dup_src.size)
    sub = tets[upper_bone]
    remap = np.where(new_id[sub] >= 0, new_id[sub], sub)
    tets[upper_bone] = remap.astype(np.int32)
    xyz2 = np.concatenate([xyz, xyz[dup_src]], axis=0)
    hinge_ids = np.nonzero(hinge)[0]
    # only hinge vertices that belong to bone tets are joint vertices
    bone_vs = np.unique(tets[role == 2])
    hinge_ids = np.intersect1d(hinge_ids, bone_vs).astype(np.int32)
    pins = np.unique(np.concatenate([_face_pins(xyz2, 2, 0.0), hinge_ids])).astype(np.int32)
    rng = np.random.default_rng(seed)
    acts = [rng.uniform(0.0, 1.0, size=4) for _ in range(frames)]
    bone = np.where(role == 2, np.where(upper_bone, 1, 0), -1).astype(np.int32)
    q = dataclasses.replace(p, rest_xyz=xyz2, tets=tets, pins=pins,
                            pin_xyz=xyz2[pins].copy(), activation=acts[0].copy(), bone=bone)
    q.extra = dict(p.extra, hinge=hinge_ids, duplicated=dup_src)
    return q, acts


def sub_problem(p: Problem, z_max: float) -> Problem:
    """The tets of ``p`` whose centroid lies below ``z_max`` with their
    materials, fibers, groups and bone labels, vertices renumbered in order;
    pins are the kept pinned vertices (targets as in ``p``)."""
    cz = p.rest_xyz[p.tets].mean(axis=1)[:, 2]
    keep = np.nonzero(cz < z_max)[0]
    used = np.unique(p.tets[keep])
    new = np.full(p.n_vertices, -1, np.int64)
    new[used] = np.arange(used.size)
    pin_keep = np.nonzero(new[p.pins] >= 0)[0]
    return dataclasses.replace(
        p, name=f"{p.name}_z<{z_max:g}", rest_xyz=p.rest_xyz[used].copy(),
        tets=new[p.tets[keep]].astype(np.int32), youngs=p.youngs[keep].copy(), poisson=p.poisson[keep].copy(),
        fiber=p.fiber[keep].copy(), group=p.group[keep].copy(),
        pins=new[p.pins[pin_keep]].astype(np.int32), pin_xyz=p.pin_xyz[pin_keep].copy(),
        activation=p.activation.copy(), bone=None if p.bone is None else p.bone[keep].copy(),
        extra={})


def adjoint_case(nx: int = 16, ny: int = 16, nz: int = 64, n_markers: int = 64, seed: int = 0):
    """8-group limb with marker vertices drawn without replacement from the free
    surface vertices, and seeded target activations a* ~ U[0,1]^8."""
    p = limb(nx, ny, nz, n_groups=8, seed=seed, name=f"adjoint{nx}x{ny}x{nz}")
    xyz = p.rest_xyz
    W, D, Hh = nx * H_EDGE, ny * H_EDGE, nz * H_EDGE
    surf = ((np.abs(xyz[:, 0]) < 1e-9) | (np.abs(xyz[:, 0] - W) < 1e-9) |
            (np.abs(xyz[:, 1]) < 1e-9) | (np.abs(xyz[:, 1] - D) < 1e-9) |
            (np.abs(xyz[:, 2] - Hh) < 1e-9))
    free = np.ones(xyz.shape[0], bool)
    free[p.pins] = False
    cand = np.nonzero(surf & free)[0]
    rng = np.random.default_rng(seed)
    markers = np.sort(rng.choice(cand, size=n_markers, replace=False)).astype(np.int32)
    a_star = rng.uniform(0.0, 1.0, size=8)
    p.activation = np.full(8, 0.5)
    p.extra.update(markers=markers, a_star=a_star)
    return p


def serving_trace(n_requests: int = 512, rate_hz: float = 200.0, seed: int = 0,
                  t_min: int = 2000, t_max: int = 300000, n_max: int = 23):
    """Poisson arrivals of box-grid limb requests N x N x 4N with log-uniform
    target tet counts, heterogeneous-limb materials, 4 quadrant groups with
    a ~ U[0,1]^4 and a pin pattern drawn from {z=0 face; both end faces;
    z=0 face plus the hinge line}.  Returns a list of dicts with keys
    ``arrival``, ``dims``, ``activation``, ``pin_mode``."""
    ss = np.random.SeedSequence(seed)
    children = ss.spawn(n_requests)
    t = 0.0
    arr_rng = np.random.default_rng(seed)
    out = []
    for c in children:
        r = np.random.default_rng(c)
        T = math.exp(r.uniform(math.log(t_min), math.log(t_max)))
        N = int(min(max(round((T / 24.0) ** (1.0 / 3.0)), 5), n_max))
        act = r.uniform(0.0, 1.0, size=4)
        pin_mode = int(r.integers(0, 3))
        t += arr_rng.exponential(1.0 / rate_hz)
        out.append(dict(arrival=t, dims=(N, N, 4 * N), activation=act, pin_mode=pin_mode))
    return out


def serving_problem(dims, activation, pin_mode: int) -> Problem:
    nx, ny, nz = dims
    p = limb(nx, ny, nz, n_groups=4, seed=0, activation=activation,
             name=f"serve{nx}x{ny}x{nz}")
    xyz = p.rest_xyz
    pins = _face_pins(xyz, 2, 0.0)
    if pin_mode == 1:
        pins = np.concatenate([pins, _face_pins(xyz, 2, nz * H_EDGE)])
    elif pin_mode == 2:
        hinge = np.nonzero((np.abs(xyz[:, 2] - nz * H_EDGE / 2) < 1e-9) &
                           (np.abs(xyz[:, 1] - ny * H_EDGE / 2) < 1e-9))[0]
        pins = np.concatenate([pins, hinge])
    pins = np.unique(pins).astype(np.int32)
    p.pins, p.pin_xyz = pins, xyz[pins].copy()
    return p


def tiny(kind: str, activation: float = 0.3, seed: int = 0) -> Problem:
    """Tiny meshes for brute-force checks: 'tet1', 'tet2', 'cube', 'cube2',
    'grid224', 'grid2216'.  Fibers are seeded random unit vectors; every vertex
    with z=0 is pinned, plus extra pins so that every case has >= 3
    non-collinear pinned vertices."""
    rng = np.random.default_rng(seed)
    if kind == "tet1":
        xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0.2, 0.3, 1.0]], float) * H_EDGE
        tets = np.array([[0, 1, 2, 3]], np.int32)
        pins = np.array([0, 1, 2], np.int32)
    elif kind == "tet2":
        xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0.2, 0.3, 1.0], [1.1, 1.0, 0.8]],
                       float) * H_EDGE
        tets = np.array([[0, 1, 2, 3], [1, 2, 3, 4]], np.int32)
        pins = np.array([0, 1, 2], np.int32)
    else:
        dims = {"cube": (1, 1, 1), "cube2": (2, 1, 1), "grid224": (2, 2, 4),
                "grid2216": (2, 2, 16)}[kind]
        xyz = grid_vertices(*dims)
        tets = kuhn_tets(*dims)
        pins = _face_pins(xyz, 2, 0.0)
    m = tets.shape[0]
    fib = rng.normal(size=(m, 3))
    fib /= np.linalg.norm(fib, axis=1, keepdims=True)
    return Problem(name=kind, rest_xyz=xyz, tets=tets, youngs=np.full(m, E_MUSCLE),
                   poisson=np.full(m, NU), fiber=fib, group=np.zeros(m, np.int32),
                   pins=pins, pin_xyz=xyz[pins].copy(),
                   activation=np.array([activation]))


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


CONFIGS: Dict[str, str] = {
    "box_beam": "4x4x16 homogeneous muscle box, fibers along z, a=0.5, z=0 pinned",
    "heterogeneous_limb": "20x20x80 limb (bone core, tendon caps, helical fibers), 20-step ramp",
    "hinge_limb": "40x40x160 limb, two bones with a pinned hinge, 4 groups, 60 frames",
    "serving_stream": "512 Poisson requests of N x N x 4N limbs, 2k-300k tets",
    "adjoint_limb": "16x16x64 limb, 8 groups, 64 markers",
}
