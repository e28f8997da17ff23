"""The two forms of the forward triangular sweep on the same meshes.

Column form: one lane per row over the column-major copy of a supernode's
block.  It runs on forward levels of many narrow supernodes; automatically
only on meshes of about a million tets.  Row form: 8 lanes per row.
EMU_FWD_COLUMN=1, set before a mesh is created, forces the column form
wherever the supernode widths allow it; EMU_FWD_COLUMN=0 turns it off.

Checked on small meshes:
* both forms' ACAP solve q*(F) at a seeded deformation gradient against the
  oracle's (1e-12 relative, as the evaluation parity) and against each
  other;
* a served solve against emu_solve bit for bit with the column form forced
  (the batched launch takes the same items, one map entry per four)."""
import numpy as np
import pytest

from oracle import mesh as omesh
from paper_2006_08821_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


CASES = [
    ("limb8x8x32", lambda: wl.limb(8, 8, 32, n_groups=4, activation=[0.3, 0.6, 0.1, 0.9])),
    ("hinge10x10x40", lambda: wl.hinge_limb(10, 10, 40, frames=1)[0]),
]


@pytest.mark.parametrize("name,make", CASES)
def test_forward_sweep_forms_match_oracle(torch, monkeypatch, name, make):
    from paper_2006_08821_amd.emu import Mesh
    p = make()
    M = omesh.build(p, modes=False)
    rng = np.random.default_rng(19)
    F = np.eye(3) + 0.05 * rng.normal(size=(M.m, 3, 3))
    q_ref = omesh.acap_solve(M, F)
    qs, levels = {}, {}
    for mode in ("1", "0"):
        monkeypatch.setenv("EMU_FWD_COLUMN", mode)
        mesh = Mesh(p)
        levels[mode] = mesh.info()["fwd_column_levels"]
        qs[mode] = mesh.evaluate(F, direction=False)["q"].cpu().numpy()
        del mesh
    assert levels["1"] >= 2 and levels["0"] == 0, levels
    for mode, q in qs.items():
        assert np.abs(q - q_ref).max() <= 1e-12 * np.abs(q_ref).max(), mode
    assert np.abs(qs["1"] - qs["0"]).max() <= 1e-12 * np.abs(q_ref).max()
    print(f"{name}: {levels['1']} column-form levels forced", flush=True)


def test_served_solve_equals_single_mesh_with_column_form(torch, monkeypatch):
    from paper_2006_08821_amd.emu import Mesh, Server
    monkeypatch.setenv("EMU_FWD_COLUMN", "1")
    target = wl.serving_problem((8, 8, 32), np.array([0.2, 0.4, 0.6, 0.8]), 1)
    other = wl.serving_problem((6, 6, 24), np.array([0.7, 0.1, 0.5, 0.3]), 0)
    opts = dict(grad_tol=1e-8, max_iters=3000, warm_start=0)
    s = Server(iters_per_round=8)
    t0 = s.submit(other, **opts)
    t1 = s.submit(target, **opts)
    q_srv, st_srv, _ = s.wait(t1)
    s.wait(t0)
    s.close()
    mesh = Mesh(target)
    assert mesh.info()["fwd_column_levels"] >= 2
    q_one, st_one = mesh.solve(**opts)
    assert st_one["status"] == st_srv["status"] == 0, (st_one, st_srv)
    assert st_one["iters"] == st_srv["iters"]
    assert np.array_equal(q_one.cpu().numpy(), q_srv)
