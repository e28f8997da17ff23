"""CPU tests of the C-ABI library: exported symbols and the host-side setup
(geometry, weighted Laplacian, nested-dissection supernodal factor, eigenpairs,
validation) against independent SciPy routines and the oracle's setup."""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import mesh as msh
from paper_2006_08821_amd import _lib
from paper_2006_08821_amd import workloads as wl
from paper_2006_08821_amd.emu import HostSetup

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in ("emu.h", "emu_host.h"):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for mt in re.finditer(r"\b(emu_\w+)\s*\(", src):
            names.add(mt.group(1))
    return names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    names = _declared_functions()
    assert "emu_solve" in names and "emu_create_mesh" in names and "emu_solve_grad" in names
    for nm in sorted(names):
        assert hasattr(lib, nm), nm
    # the binding covers every declared function
    assert names <= set(_lib.SIGNATURES), names - set(_lib.SIGNATURES)


CASES = [("box", lambda: wl.box_beam()), ("limb", lambda: wl.limb(6, 6, 24)),
         ("tet2", lambda: wl.tiny("tet2")), ("hinge", lambda: wl.hinge_limb(6, 6, 12, frames=1)[0])]


@pytest.mark.parametrize("name,make", CASES)
def test_factor_solve_matches_superlu(name, make):
    p = make()
    k = min(48, 3 * (p.n_vertices - len(p.pins) - 1))
    hs = HostSetup(p, n_modes=k)
    M = msh.build(p, n_modes=k)
    rng = np.random.default_rng(0)
    b = rng.normal(size=(p.n_vertices, 3))
    x = hs.solve(b)
    xr = np.zeros_like(b)
    xr[M.free] = M.lu.solve(b[M.free])
    assert np.abs(x - xr).max() <= 1e-11 * np.abs(xr).max()
    y = hs.apply(x)
    assert np.abs(M.L @ x - y).max() <= 1e-12 * np.abs(y).max()


def test_factor_solve_matches_superlu_with_wide_fronts():
    # a mesh whose top fronts run the factorization's multi-threaded dense
    # kernels (diagonal blocks over 128 wide, hundreds of off-diagonal rows,
    # row counts that are not multiples of the four- and eight-wide blocks)
    p = wl.limb(14, 14, 56)
    hs = HostSetup(p, n_modes=0)
    info = hs.info()
    assert info["n_supernodes"] > 100
    M = msh.build(p, modes=False)
    rng = np.random.default_rng(1)
    b = rng.normal(size=(p.n_vertices, 3))
    x = hs.solve(b)
    xr = np.zeros_like(b)
    xr[M.free] = M.lu.solve(b[M.free])
    assert np.abs(x - xr).max() <= 1e-11 * np.abs(xr).max()


@pytest.mark.parametrize("name,make", CASES)
def test_geometry_matches_oracle(name, make):
    p = make()
    hs = HostSetup(p, n_modes=0)
    M = msh.build(p, modes=False)
    t, vol, w = hs.geometry()
    assert (t == M.tets).all()
    assert np.allclose(vol, M.vol, rtol=1e-13)
    assert np.allclose(w, M.w, rtol=1e-13)


def test_eigenpairs_match_arpack():
    p = wl.limb(6, 6, 24)
    hs = HostSetup(p)
    nu, phi = hs.modes()
    free = np.setdiff1d(np.arange(p.n_vertices), p.pins)
    M = msh.build(p, modes=False)
    w = spla.eigsh(M.Lff, k=16, sigma=0.0, which="LM", return_eigenvectors=False)
    assert np.allclose(nu, np.sort(w), rtol=1e-10)
    # eigen-residual and orthonormality of the returned vectors
    P = phi[:, free]
    assert np.allclose(P @ P.T, np.eye(16), atol=1e-10)
    R = M.Lff @ P.T - P.T * nu
    assert np.abs(R).max() < 1e-6 * nu.max()
    assert np.all(phi[:, p.pins] == 0)


def test_nested_dissection_structure():
    p = wl.heterogeneous_limb_ramp(nx=8, ny=8, nz=32)[0]
    hs = HostSetup(p, n_modes=0)
    inf = hs.info()
    assert inf["n_free"] == p.n_vertices - len(p.pins)
    assert inf["n_levels"] >= 4 and inf["n_supernodes"] > 10
    # fill stays far below a dense factor
    assert inf["factor_nnz"] < 0.1 * inf["n_free"] ** 2


def _err(p, **kw):
    with pytest.raises(_lib.EmuError) as ei:
        HostSetup(p, **kw)
    return ei.value.code


def test_validation_errors():
    base = wl.tiny("cube")
    p = base.copy()
    p.rest_xyz[0, 0] = np.nan
    assert _err(p) == 1
    p = base.copy()
    p.tets[0, 1] = p.tets[0, 0]
    assert _err(p) == 1
    p = base.copy()
    p.pins = np.array([0, 0, 1], np.int32)
    p.pin_xyz = p.rest_xyz[p.pins]
    assert _err(p) == 1
    p = base.copy()
    p.poisson[0] = 0.5
    assert _err(p) == 1
    p = base.copy()
    p.youngs[0] = -1.0
    assert _err(p) == 1
    p = base.copy()
    p.tets[0, 0] = 99
    assert _err(p) == 1
    assert _err(base, n_modes=5) == 1
    # degenerate (flat) tet
    p = wl.tiny("tet1")
    p.rest_xyz[3, 2] = 0.0
    assert _err(p) == 1


def test_unpinned_component_is_singular():
    # two disjoint cubes, pins only on the first
    a = wl.tiny("cube")
    b = wl.tiny("cube")
    p = a.copy()
    p.rest_xyz = np.concatenate([a.rest_xyz, b.rest_xyz + [0.05, 0, 0]])
    p.tets = np.concatenate([a.tets, b.tets + a.n_vertices]).astype(np.int32)
    m = p.tets.shape[0]
    p.youngs = np.full(m, wl.E_MUSCLE)
    p.poisson = np.full(m, wl.NU)
    p.fiber = np.tile([0, 0, 1.0], (m, 1))
    p.group = np.zeros(m, np.int32)
    assert _err(p, n_modes=0) == 2


def test_server_entry_points_reject_null_without_touching_a_device():
    import ctypes as C
    lib = _lib.load()
    t = C.c_uint64()
    assert lib.emu_server_submit(None, None, None, None, C.byref(t)) == 1
    assert lib.emu_server_wait(None, C.c_uint64(1), None, None, None) == 1
    assert lib.emu_server_report_get(None, None) == 1
    assert lib.emu_server_destroy(None) == 0
    assert lib.emu_server_create(None, None) == 1


def test_server_create_reports_missing_device():
    import ctypes as C
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = _lib.load()
    h = C.c_void_p()
    assert lib.emu_server_create(None, C.byref(h)) == 7  # EMU_E_HIP
    assert not h.value
