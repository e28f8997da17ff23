"""GPU adjoint of the equilibrium w.r.t. per-group activations (emu_solve_grad),
against the oracle's independent q-space adjoint and central differences."""
import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import fem as ofem
from oracle import mesh as omesh
from paper_2006_08821_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _problem():
    # homogeneous muscle, two groups (lower / upper half), fibers along z
    p = wl.box_beam(2, 2, 8, activation=0.4)
    cz = p.rest_xyz[p.tets].mean(axis=1)[:, 2]
    p.group = (cz >= 0.04).astype(np.int32)
    p.activation = np.array([0.3, 0.6])
    top = np.nonzero(np.abs(p.rest_xyz[:, 2] - 0.08) < 1e-9)[0]
    markers = top[:6]
    target = p.rest_xyz[markers] + np.array([0.002, -0.001, -0.004])
    return p, markers, target


def _loss_and_grad(torch, q, markers, target):
    qn = q.cpu().numpy()
    dq = np.zeros_like(qn)
    diff = qn[markers] - target
    dq[markers] = 2.0 * diff
    return float(np.sum(diff * diff)), torch.as_tensor(dq, device="cuda")


def test_adjoint_matches_oracle_and_fd(torch):
    from paper_2006_08821_amd.emu import Mesh
    p, markers, target = _problem()
    mesh = Mesh(p)
    q, st = mesh.solve(grad_tol=1e-11)
    assert st["status"] == 0
    L, dq = _loss_and_grad(torch, q, markers, target)
    g, ast = mesh.solve_grad(dq, stats=True)
    assert ast["status"] == 0, ast
    # independent: q-space adjoint on the Moreau-envelope Newton solution
    M = omesh.build(p, modes=False)
    qo = ofem.moreau_solve(M, p.activation, tol=1e-13)["q"]
    Lo, go = oadj.activation_gradient(M, p.activation, qo, markers, target)
    assert abs(L - Lo) <= 1e-8 * abs(Lo)
    assert np.allclose(g, go, rtol=1e-6, atol=1e-9 * np.abs(go).max())
    # central differences of the GPU solve, h = 1e-4
    h = 1e-4
    F0, _ = mesh.get_state()
    for k in range(2):
        vals = []
        for sgn in (+1, -1):
            a = p.activation.copy()
            a[k] += sgn * h
            mesh.set_state(F0)
            mesh.set_activation(a)
            qk, sk = mesh.solve(grad_tol=1e-11)
            assert sk["status"] == 0
            vals.append(_loss_and_grad(torch, qk, markers, target)[0])
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-4 * abs(g[k]) + 1e-12


def test_autograd_function(torch):
    from paper_2006_08821_amd import emu
    p, markers, target = _problem()
    mesh = emu.Mesh(p)
    a = torch.tensor(p.activation, dtype=torch.float64, requires_grad=True)
    q = emu.solve(mesh, a, grad_tol=1e-11)
    tgt = torch.as_tensor(target, device="cuda")
    loss = ((q[torch.as_tensor(markers, device="cuda")] - tgt) ** 2).sum()
    loss.backward()
    g_direct = mesh.solve_grad(_loss_and_grad(torch, q.detach(), markers, target)[1])
    assert np.allclose(a.grad.numpy(), g_direct, rtol=1e-12, atol=0)


def test_solve_grad_requires_converged_state(torch):
    from paper_2006_08821_amd import _lib
    from paper_2006_08821_amd.emu import Mesh
    p, markers, target = _problem()
    mesh = Mesh(p)
    with pytest.raises(_lib.EmuError) as e:
        mesh.solve_grad(torch.zeros((p.n_vertices, 3), dtype=torch.float64, device="cuda"))
    assert e.value.code == 8


def test_adjoint_degenerate_right_hand_sides(torch):
    # the conjugate-gradient scalars and the stop test run on the device:
    # a zero dL/dq stops before the first step with dL/da = 0, a NaN in dL/dq
    # stops with EMU_E_NONFINITE (|b| not finite), and a repeated call gives
    # the same bits
    from paper_2006_08821_amd import _lib
    from paper_2006_08821_amd.emu import Mesh
    p, markers, target = _problem()
    mesh = Mesh(p)
    q, st = mesh.solve(grad_tol=1e-11)
    assert st["status"] == 0
    zero = torch.zeros((p.n_vertices, 3), dtype=torch.float64, device="cuda")
    g0, s0 = mesh.solve_grad(zero, stats=True)
    assert s0["status"] == 0 and s0["iters"] == 0, s0
    assert np.array_equal(g0, np.zeros_like(g0))
    _, dq = _loss_and_grad(torch, q, markers, target)
    g1, s1 = mesh.solve_grad(dq, stats=True)
    g2, s2 = mesh.solve_grad(dq, stats=True)
    assert s1["status"] == 0 and s1["iters"] > 0 and s1["iters"] == s2["iters"]
    assert np.array_equal(g1, g2)
    bad = dq.clone()
    bad[int(markers[0]), 0] = float("nan")
    with pytest.raises(_lib.EmuError) as e:
        mesh.solve_grad(bad)
    assert e.value.code == 5
    # the mesh state is unchanged: the next adjoint gives the same bits again
    g3 = mesh.solve_grad(dq)
    assert np.array_equal(g1, g3)


def test_adjoint_on_a_mixed_precision_mesh(torch):
    # form (1) with the adjoint: on a mixed-precision mesh the Hessian-vector
    # products stay FP64 and only the preconditioner (the stored FP32 block
    # inverses) changes, so dL/da matches the FP64 mesh's and the oracle's
    # q-space adjoint within the mixed path's state accuracy
    from paper_2006_08821_amd.emu import Mesh
    p, markers, target = _problem()
    g = {}
    for prec in ("fp64", "mixed"):
        mesh = Mesh(p, precision=prec)
        q, st = mesh.solve(grad_tol=1e-11, max_iters=5000)
        assert st["status"] == 0, (prec, st)
        _, dq = _loss_and_grad(torch, q, markers, target)
        g[prec], ast = mesh.solve_grad(dq, stats=True)
        assert ast["status"] == 0 and ast["iters"] > 0, (prec, ast)
        print(prec, "adjoint steps", ast["iters"], flush=True)
        mesh.close()
    M = omesh.build(p, modes=False)
    qo = ofem.moreau_solve(M, p.activation, tol=1e-13)["q"]
    _, go = oadj.activation_gradient(M, p.activation, qo, markers, target)
    scale = np.abs(go).max()
    assert np.abs(g["mixed"] - g["fp64"]).max() <= 1e-5 * scale, (g, go)
    assert np.abs(g["mixed"] - go).max() <= 1e-5 * scale, (g, go)


def test_solve_and_adjoint_without_modes(torch):
    # the degenerate case k = 0 (no low-rank correction: the quasi-Newton
    # Hessian is the block-diagonal part alone, and the adjoint's
    # preconditioner the block inverses): the solve still reaches the
    # oracle's minimizer and dL/da its q-space adjoint
    from paper_2006_08821_amd.emu import Mesh
    p, markers, target = _problem()
    mesh = Mesh(p, n_modes=0)
    assert mesh.info()["n_modes"] == 0
    q, st = mesh.solve(grad_tol=1e-11, max_iters=20000)
    assert st["status"] == 0, st
    _, dq = _loss_and_grad(torch, q, markers, target)
    g, ast = mesh.solve_grad(dq, stats=True)
    assert ast["status"] == 0 and ast["iters"] > 0, ast
    print("k = 0: iterations", st["iters"], "adjoint steps", ast["iters"], flush=True)
    mesh.close()
    M = omesh.build(p, modes=False)
    qo = ofem.moreau_solve(M, p.activation, tol=1e-13)["q"]
    qn = q.cpu().numpy()
    assert np.abs(qn - qo).max() <= 1e-6 * np.abs(qo - M.rest).max()
    _, go = oadj.activation_gradient(M, p.activation, qo, markers, target)
    assert np.abs(g - go).max() <= 1e-6 * np.abs(go).max(), (g, go)
