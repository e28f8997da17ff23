"""The host C++ (mesh validation, geometry, ordering, factorization, modes and
the host-only API) built with AddressSanitizer and UndefinedBehaviorSanitizer
(g++, CPU only) and run on heterogeneous meshes and on invalid descriptions
(tests/host_sanitize_driver.cpp): no sanitizer report, every invalid input
rejected, and the same results as the regular build of the library."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2006_08821_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2006_08821_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("asan") / "host_sanitize")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           os.path.join(ROOT, "tests", "host_sanitize_driver.cpp"),
           os.path.join(CSRC, "host_setup.cpp"), os.path.join(CSRC, "api_host.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        if "asan" in (r.stderr + r.stdout).lower() and "cannot find" in (r.stderr + r.stdout).lower():
            pytest.skip("sanitizer runtime not installed")
        raise AssertionError(r.stderr[-4000:])
    return exe


def _write_mesh(path, p, b):
    bone = getattr(p, "bone", None)
    with open(path, "wb") as f:
        np.array([p.n_vertices, p.n_tets, int(p.group.max()) + 1, len(p.pins), p.n_modes,
                  int(getattr(p, "weight_mode", 0)), int(bone is not None)], np.int32).tofile(f)
        np.ascontiguousarray(p.rest_xyz, np.float64).tofile(f)
        np.ascontiguousarray(p.tets, np.int32).tofile(f)
        np.ascontiguousarray(p.youngs, np.float64).tofile(f)
        np.ascontiguousarray(p.poisson, np.float64).tofile(f)
        np.ascontiguousarray(p.fiber, np.float64).tofile(f)
        np.ascontiguousarray(p.group, np.int32).tofile(f)
        np.ascontiguousarray(p.pins, np.int32).tofile(f)
        if bone is not None:
            np.ascontiguousarray(bone, np.int32).tofile(f)
        np.ascontiguousarray(b, np.float64).tofile(f)


CASES = [
    ("limb4x4x12", lambda: wl.limb(4, 4, 12, n_groups=4, activation=[0.3, 0.6, 0.1, 0.9])),
    ("hinge6x6x12", lambda: wl.hinge_limb(6, 6, 12, frames=1)[0]),
]


@pytest.mark.parametrize("name,make", CASES)
def test_host_code_under_sanitizers(driver, tmp_path, name, make):
    from paper_2006_08821_amd.emu import HostSetup
    p = make()
    rng = np.random.default_rng(4)
    b = rng.normal(size=(p.n_vertices, 3))
    mesh_bin, out_bin = str(tmp_path / "mesh.bin"), str(tmp_path / "out.bin")
    _write_mesh(mesh_bin, p, b)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([driver, mesh_bin, out_bin], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    n, m = p.n_vertices, p.n_tets
    hs = HostSetup(p)
    k1 = hs.info()["n_modes"] // 3
    out = np.fromfile(out_bin, np.float64)
    x, y = out[:3 * n].reshape(n, 3), out[3 * n:6 * n].reshape(n, 3)
    nu = out[6 * n:6 * n + k1]
    vol = out[6 * n + k1 + k1 * n:6 * n + k1 + k1 * n + m]
    w = out[6 * n + k1 + k1 * n + m:]
    assert np.allclose(x, hs.solve(b), rtol=1e-10, atol=1e-14 * np.abs(x).max())
    assert np.allclose(y, hs.apply(b), rtol=1e-10, atol=1e-14 * np.abs(y).max())
    nu_ref, _ = hs.modes()
    assert np.allclose(nu, nu_ref, rtol=1e-8)
    _, vol_ref, w_ref = hs.geometry()
    assert np.allclose(vol, vol_ref, rtol=1e-12) and np.allclose(w, w_ref, rtol=1e-12)
