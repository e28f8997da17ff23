"""Affine bones (Sec. 3.3): the tets of each bone share one deformation gradient
F_b, tied to the continuous mesh with the slack eps_2 (a bone tet's ACAP weight
vol (1 + 1/eps_2)).  The GPU iteration on the reduced variables against the
oracle's EMU iteration over the same variables (O1, pinned against brute-force
Newton on a small mesh): evaluation, trajectories, converged minimizers, the
shared F of each bone, and the constraint residual's scaling with the slack.
"""
import ctypes as C
import json
import math
import os

import numpy as np
import pytest

from oracle import emu as oemu
from oracle import mesh as omesh
from paper_2006_08821_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _mesh(p, slack, **kw):
    from paper_2006_08821_amd.emu import Mesh
    return Mesh(p, affine_bones=True, bone_slack=slack, **kw)


def _share_modes(mesh, M):
    phi = np.zeros((M.phi.shape[0], M.n))
    phi[:, M.free] = M.phi
    mesh.set_modes(M.nu, phi)


def _disp_err(q, qref, rest):
    return float(np.abs(q - qref).max() / np.abs(qref - rest).max())


def _bone_spread(F, bone):
    """Largest difference between the F of two tets of one bone."""
    out = 0.0
    for b in sorted(set(int(x) for x in bone if x >= 0)):
        Fb = F[bone == b]
        out = max(out, float(np.abs(Fb - Fb[0]).max()))
    return out


CASES = [
    ("limb4x4x12", lambda: wl.limb(4, 4, 12, n_groups=4, activation=[0.3, 0.6, 0.1, 0.9]), 1e-3),
    ("hinge6x6x12", lambda: wl.hinge_limb(6, 6, 12, frames=1)[0], 1e-1),
]


@pytest.mark.parametrize("name,make,slack", CASES)
def test_affine_evaluate_matches_oracle(torch, name, make, slack):
    p = make()
    assert (p.bone >= 0).any()
    M = omesh.build(p, affine_bones=True, bone_slack=slack)
    mesh = _mesh(p, slack)
    _share_modes(mesh, M)
    rng = np.random.default_rng(17)
    F = oemu.expand(M, np.eye(3) + 0.05 * rng.normal(size=(M.m_red, 3, 3)))
    ev = mesh.evaluate(F)
    a_el = omesh.activation_per_element(M, p.activation)
    q = omesh.acap_solve(M, F)
    A = omesh.gather_A(M, q)
    E = math.fsum(oemu.element_energy(M, F, A, a_el)) - omesh.work(M, q)
    g = oemu.reduce_sum(M, oemu.grad_F(M, F, A, a_el).reshape(M.m, 9))
    gn = math.sqrt(math.fsum((g * g).reshape(-1)))
    H = oemu.reduced_block_hessian(M, F, a_el, "split")
    Bred = oemu.reduce_sum(M, oemu.woodbury_blocks(M, np.arange(M.m)))
    d = oemu.expand(M, oemu.direction(M, H, g, B_all=Bred)).reshape(M.m, 3, 3)
    assert np.abs(ev["q"].cpu().numpy() - q).max() <= 1e-12 * np.abs(q).max()
    assert math.isclose(ev["energy"], E, rel_tol=1e-11)
    assert math.isclose(ev["grad_norm"], gn, rel_tol=1e-10)
    dg = ev["direction"].cpu().numpy()
    assert np.abs(dg - d).max() <= 1e-9 * np.abs(d).max()
    # the per-tet gradient norm differs: the bone terms are summed first
    gt = oemu.grad_F(M, F, A, a_el)
    assert abs(math.sqrt(float((gt * gt).sum())) - gn) > 1e-6 * gn


@pytest.mark.parametrize("name,make,slack", CASES)
def test_affine_trajectory_matches_oracle(torch, name, make, slack):
    p = make()
    M = omesh.build(p, affine_bones=True, bone_slack=slack)
    mesh = _mesh(p, slack)
    _share_modes(mesh, M)
    q, st = mesh.solve(grad_tol=0.0, max_iters=30, iters_per_sync=32, raise_on_error=False)
    assert st["iters"] == 30, st
    o1 = oemu.solve(M, p.activation, tol=0.0, max_iters=30, hessian="split", trials="affine")
    assert o1["stats"]["iters"] == 30
    assert _disp_err(q.cpu().numpy(), o1["q"], M.rest) <= 1e-8
    F, _ = mesh.get_state()
    F = F.cpu().numpy()
    assert np.abs(F - o1["F"]).max() <= 1e-8
    assert _bone_spread(F, p.bone) == 0.0
    assert math.isclose(st["energy"], o1["stats"]["energy"], rel_tol=1e-10)


def _golden():
    with open(os.path.join(os.path.dirname(__file__), "golden", "affine_refs.json")) as f:
        return json.load(f)


GOLDEN = [
    ("limb5x5x20", lambda: wl.limb(5, 5, 20, n_groups=4, activation=np.array([0.5, 0.2, 0.8, 0.4]))),
    ("hinge6x6x24", lambda: wl.hinge_limb(6, 6, 24, frames=1)[0]),
]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-5), ("mixed", 1e-5)])
@pytest.mark.parametrize("name,make", GOLDEN)
def test_affine_converges_to_oracle_minimizer(torch, name, make, precision, tol):
    # both stop at |g| <= 1e-8 (the reduced gradient); the stiff bones
    # (weights 1 + 1/eps_2 times the tets') bound q's error by about 1e-5
    ref = _golden()[name]
    p = make()
    mesh = _mesh(p, ref["slack"], precision=precision)
    q, st = mesh.solve(grad_tol=ref["tol"], max_iters=20000)
    assert st["status"] == 0 and st["grad_norm"] <= ref["tol"], st
    assert _disp_err(q.cpu().numpy(), np.array(ref["q"]), p.rest_xyz) <= tol
    F, _ = mesh.get_state()
    F = F.cpu().numpy()
    assert _bone_spread(F, p.bone) == 0.0
    for b, Fb in enumerate(ref["bone_F"]):
        assert np.abs(F[p.bone == b][0] - np.array(Fb)).max() <= 10 * tol
    print(f"{name} {precision}: GPU {st['iters']} iterations, oracle {ref['iters']}", flush=True)


def test_affine_constraint_residual_scales_with_slack(torch):
    # the bone constraint G_i q = F_b is met to O(eps_2): on the 6x6x24 limb
    # (5184 tets) the residual on the bone tets shrinks tenfold per decade
    p = wl.limb(6, 6, 24, n_groups=4, activation=np.array([0.5, 0.2, 0.8, 0.4]))
    M = omesh.build(p, modes=False)
    sel = p.bone >= 0
    res = []
    for slack in (1e-2, 1e-3):
        mesh = _mesh(p, slack)
        q, st = mesh.solve(grad_tol=1e-8, max_iters=20000, raise_on_error=False)
        print(f"slack {slack}: {st}", flush=True)
        assert st["status"] == 0, st
        F, _ = mesh.get_state()
        F = F.cpu().numpy()
        assert _bone_spread(F, p.bone) == 0.0
        A = omesh.gather_A(M, q.cpu().numpy())
        res.append(float(np.abs(A[sel] - F[sel]).max()))
    assert 5 < res[0] / res[1] < 20, res


def test_affine_bones_rejected_where_unsupported(torch):
    from paper_2006_08821_amd import _lib
    from paper_2006_08821_amd.emu import Mesh, Server, _desc_arrays
    p = wl.limb(4, 4, 12, n_groups=4, activation=[0.3, 0.6, 0.1, 0.9])
    mesh = _mesh(p, 1e-2)
    mesh.solve(grad_tol=1e-8, max_iters=20000)
    w = torch.zeros((p.n_vertices, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.EmuError):
        mesh.solve_grad(w)
    with pytest.raises(_lib.EmuError):
        Mesh(p, affine_bones=True, hessian_blocks="coupled")
    s = Server()
    desc, keep = _desc_arrays(p, affine_bones=True)
    a = np.asarray(p.activation, float)
    t = C.c_uint64()
    code = s._lib.emu_server_submit(s._h, C.byref(desc), a.ctypes.data_as(_lib.DP), None, C.byref(t))
    s.close()
    assert code == 1
