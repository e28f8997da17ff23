"""Device eigenpairs of L_ff (the modes of eq. low-rank) against the host
solver of the same library: equal eigenvalues, residuals checked with the
host's own L_ff product, orthonormal modes, the same subspace where the
spectrum has a gap after the k-th value, and the mesh setup time with each."""
import numpy as np
import pytest

from paper_2006_08821_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


CASES = [
    ("box_beam", lambda: wl.box_beam()),
    ("limb8x8x32", lambda: wl.limb(8, 8, 32, n_groups=4, activation=[0.3, 0.6, 0.1, 0.9])),
    ("hinge10x10x40", lambda: wl.hinge_limb(10, 10, 40, frames=1)[0]),
    ("serve16x16x64_pm2", lambda: wl.serving_problem((16, 16, 64), np.array([0.2, 0.4, 0.6, 0.8]), 2)),
]


@pytest.mark.parametrize("name,make", CASES)
def test_device_modes_match_host_modes(torch, name, make):
    from paper_2006_08821_amd.emu import HostSetup, Mesh
    p = make()
    hs = HostSetup(p)
    nu_h, phi_h = hs.modes()
    t_host = hs.info()["setup_ms"]
    mesh = Mesh(p)
    nu_d, phi_d = mesh.get_modes()
    t_dev = mesh.info()["setup_ms"]
    assert np.allclose(nu_d, nu_h, rtol=1e-9, atol=0), (nu_d, nu_h)
    free = np.ones(p.n_vertices, bool)
    free[p.pins] = False
    k1 = len(nu_d)
    for j in range(k1):
        x = np.zeros((p.n_vertices, 3))
        x[:, 0] = phi_d[j]
        y = hs.apply(x)[:, 0]
        r = np.linalg.norm(y[free] - nu_d[j] * phi_d[j][free]) / nu_d[j]
        assert r <= 1e-7, (j, r)
        assert np.all(phi_d[j][~free] == 0)
    Pd, Ph = phi_d[:, free], phi_h[:, free]
    assert np.abs(Pd @ Pd.T - np.eye(k1)).max() <= 1e-10
    # the span of the j lowest modes is the same where nu_j+1 is well above
    # nu_j (the largest such j < k): principal angles from the singular
    # values of Pd_j Ph_j^T
    j = max([i for i in range(1, k1) if (nu_h[i] - nu_h[i - 1]) / nu_h[i - 1] > 1e-2], default=0)
    if j > 0:
        sv = np.linalg.svd(Pd[:j] @ Ph[:j].T, compute_uv=False)
        assert 1.0 - sv.min() <= 1e-9, sv.min()
    print(f"{name}: setup {t_host:.0f} ms with host modes, {t_dev:.0f} ms with device modes; "
          f"subspace of the {j} lowest modes compared", flush=True)
