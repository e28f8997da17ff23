"""Pins of the oracle's contact loop (Algorithm 1's collision block, Sec. 3.5):
the penalty forces are the negative gradient of the penalty energy, the force
field is the F-gradient of the work f . q*(F), a round keeps q = q*(F), and
obstacles that nothing touches leave the iteration unchanged."""
import math

import numpy as np

from oracle import contact as cnt
from oracle import emu
from oracle import mesh as msh
from paper_2006_08821_amd import workloads as wl

H = wl.H_EDGE


def _beam():
    p = wl.box_beam(2, 2, 8, activation=0.2)
    M = msh.build(p)
    f = np.zeros((M.n, 3))
    f[:, 0] = -0.05
    msh.set_external_forces(M, f)
    return p, M


def test_contact_forces_are_the_penalty_gradient():
    p, M = _beam()
    c = cnt.obstacles(planes=[[0.6, 0.0, 0.8, 0.3 * H], [1, 0, 0, -0.1 * H]],
                      spheres=[[H, H, 4 * H, 1.3 * H]], stiffness=7.0)
    rng = np.random.default_rng(2)
    q = p.rest_xyz + 0.3 * H * rng.normal(size=p.rest_xyz.shape)
    f = cnt.forces(M, q, c)
    assert np.abs(f).max() > 0
    assert np.all(f[M.pins] == 0)
    h = 1e-7
    for v in M.free[:20]:
        for k in range(3):
            qp, qm = q.copy(), q.copy()
            qp[v, k] += h
            qm[v, k] -= h
            fd = -(cnt.penalty_energy(M, qp, c) - cnt.penalty_energy(M, qm, c)) / (2 * h)
            assert abs(fd - f[v, k]) <= 1e-6 * max(1.0, abs(f[v, k]))


def test_force_field_is_the_work_gradient():
    # nu = w G L_ff^-1 f is d(f . q*(F))/dF: central differences over F
    p, M = _beam()
    rng = np.random.default_rng(3)
    F = np.eye(3) + 0.1 * rng.normal(size=(M.m, 3, 3))
    f = rng.normal(size=(M.n, 3))
    f[M.pins] = 0
    nu = cnt.force_field(M, f)
    E = rng.normal(size=F.shape)
    h = 1e-6
    work = lambda FF: math.fsum((f * msh.acap_solve(M, FF)).reshape(-1))
    fd = (work(F + h * E) - work(F - h * E)) / (2 * h)
    assert abs(fd - float((nu * E).sum())) <= 1e-7 * abs(fd)


def test_contact_round_keeps_the_continuous_mesh_consistent():
    # after the rounds q equals a fresh ACAP solve of the new F
    p, M = _beam()
    c = cnt.obstacles(planes=[[1, 0, 0, 0.5 * H]], stiffness=5.0, max_rounds=3)
    F = emu.rest_state(M)
    q = msh.acap_solve(M, F)
    a_el = msh.activation_per_element(M, p.activation)
    Hb = emu.block_hessian(M, F, a_el, "split")
    F2, q2, rounds = cnt.contact_loop(M, F, q, lambda nu: emu.direction(M, Hb, nu), c)
    assert rounds == 3
    assert np.abs(q2 - msh.acap_solve(M, F2)).max() <= 1e-12 * np.abs(q2).max()
    # the push is along +x where the plane cuts the beam (free vertices)
    d0, _ = cnt.penetrations(q, c)
    d2, _ = cnt.penetrations(q2, c)
    assert d2[M.free].max() < d0[M.free].max()


def test_obstacles_out_of_reach_change_nothing():
    p, M = _beam()
    c = cnt.obstacles(planes=[[1, 0, 0, -1.0]], spheres=[[5.0, 5.0, 5.0, 0.5]], stiffness=10.0)
    a = emu.solve(M, p.activation, tol=0.0, max_iters=12, hessian="split", trials="affine")
    b = emu.solve(M, p.activation, tol=0.0, max_iters=12, hessian="split", trials="affine", contact=c)
    assert b["stats"]["contact_rounds"] == 0
    assert np.array_equal(a["q"], b["q"]) and np.array_equal(a["F"], b["F"])


def test_contact_keeps_the_loaded_beam_off_the_plane():
    # the side-loaded cantilever swings to x = -6 H without the plane; with
    # the plane at x = -H/2 the contact rounds hold it there, up to a small
    # overlap (each round shrinks a penetration by the factor 1 - k C, C the
    # vertex compliance, so a few rounds leave a remainder)
    p, M = _beam()
    free = emu.solve(M, p.activation, tol=0.0, max_iters=40, hessian="split", trials="affine")
    c = cnt.obstacles(planes=[[1, 0, 0, -0.5 * H]], stiffness=10.0, tol=1e-8, max_rounds=8)
    r = emu.solve(M, p.activation, tol=0.0, max_iters=40, hessian="split", trials="affine", contact=c)
    assert free["q"][:, 0].min() < -2 * H
    assert r["stats"]["contact_rounds"] > 0
    assert r["q"][:, 0].min() > -0.6 * H
