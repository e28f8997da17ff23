"""The allocation-free adjoint entry point (emu_solve_grad_noalloc) against
emu_solve_grad, through the C ABI: same dL/da on two calls in a row, the
second on a smaller mesh (the shared scratch keeps the first call's
contents), and a clear rejection of a mesh larger than the scratch."""
import numpy as np
import pytest

from paper_2006_08821_amd import _lib
from paper_2006_08821_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _grad_pair(torch, p, seed):
    from paper_2006_08821_amd.emu import Mesh
    mesh = Mesh(p)
    q, st = mesh.solve(grad_tol=1e-10, max_iters=20000)
    assert st["status"] == 0, st
    rng = np.random.default_rng(seed)
    dLdq = torch.as_tensor(rng.normal(size=(p.n_vertices, 3)), dtype=torch.float64, device="cuda")
    g_ref, st_ref = mesh.solve_grad(dLdq, stats=True)
    g_na, st_na = mesh.solve_grad(dLdq, stats=True, noalloc=True)
    return g_ref, g_na, st_ref, st_na


def test_noalloc_adjoint_matches_allocating_entry_point(torch):
    print("no-alloc adjoint: limb 4x4x12 (4 groups), then box 2x2x8 (1 group)", flush=True)
    big = wl.limb(4, 4, 12, n_groups=4, activation=[0.3, 0.6, 0.1, 0.9])
    small = wl.box_beam(2, 2, 8, activation=0.4)
    assert small.n_tets < big.n_tets
    for p, seed in ((big, 1), (small, 2)):
        g_ref, g_na, st_ref, st_na = _grad_pair(torch, p, seed)
        assert st_ref["status"] == st_na["status"] == 0
        # same kernels, same work sizes, fixed-order reductions: same result
        assert np.abs(g_na - g_ref).max() <= 1e-12 * np.abs(g_ref).max(), (g_na, g_ref)
        assert st_na["iters"] == st_ref["iters"]


def test_noalloc_rejects_a_mesh_larger_than_the_scratch(torch):
    print("no-alloc adjoint: size rejection on a 144k-tet box", flush=True)
    from paper_2006_08821_amd.emu import Mesh
    p = wl.box_beam(20, 20, 60, activation=0.3)
    mesh = Mesh(p)
    dLdq = torch.zeros((p.n_vertices, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.EmuError) as e:
        mesh.solve_grad(dLdq, noalloc=True)
    assert e.value.code == 1 and "scratch" in str(e.value)
