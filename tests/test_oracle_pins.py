"""Pins of the oracle parts that the solver-level tests alone would not catch:
the exact line-search energy change, the element block Hessian against the
exact Hessian of the separated energy, and the solver on heterogeneous meshes
(several materials, passive elements, several groups, each ACAP weighting)."""
import math

import numpy as np
import pytest

from oracle import dense, emu, fem
from oracle import material as mat
from oracle import mesh as msh
from paper_2006_08821_amd import workloads as wl

RNG = np.random.default_rng(11)


def _disp_err(q, qref, rest):
    return np.abs(q - qref).max() / max(np.abs(qref - rest).max(), 1e-300)


def _total_energy(M, F, a_el):
    """E(F) = sum_i e_i(F_i, A_i(q*(F))) - W(q*(F)) from scratch: a fresh ACAP
    solve and the element energy of the material module (eq. separated)."""
    q = msh.acap_solve(M, F)
    A = msh.gather_A(M, q)
    return math.fsum(emu.element_energy(M, F, A, a_el)) - msh.work(M, q), q, A


def _hetero(kind="grid224", seed=0):
    """Small mesh with three materials (muscle, a stiffer tissue 30x, a stiff one
    100x, labelled bone), passive tets (group -1) and two muscle groups."""
    p = wl.tiny(kind, activation=0.5, seed=seed)
    rng = np.random.default_rng(seed)
    m = p.n_tets
    cls = rng.integers(0, 4, size=m)
    p.youngs = np.where(cls == 2, 30 * wl.E_MUSCLE, np.where(cls == 3, 100 * wl.E_MUSCLE, wl.E_MUSCLE))
    p.group = np.where(cls == 0, 0, np.where(cls == 1, 1, -1)).astype(np.int32)
    p.bone = np.where(cls == 3, 0, -1).astype(np.int32)
    p.activation = np.array([0.6, 0.3])
    return p


# ------------------------------------------------------------ line search
@pytest.mark.parametrize("forces", [False, True])
def test_delta_energy_equals_direct_difference(forces):
    # The line search compares E(F + sigma P) - E(F) against the Armijo bound
    # (Algorithm 1).  delta_energy expands each element's change exactly in
    # sigma; the direct difference of two fresh total energies must agree to
    # the rounding of the totals, for steps where every power of sigma matters.
    p = _hetero("grid224", seed=3)
    M = msh.build(p)
    if forces:
        f = np.zeros((M.n, 3))
        f[:, 0] = -0.05
        f[:, 2] = 0.02 * RNG.normal(size=M.n)
        msh.set_external_forces(M, f)
    a_el = msh.activation_per_element(M, p.activation)
    for trial in range(3):
        F = np.eye(3) + 0.2 * RNG.normal(size=(M.m, 3, 3))
        P = 0.3 * RNG.normal(size=(M.m, 3, 3))
        E0, q0, A0 = _total_energy(M, F, a_el)
        for sigma in (2.0, 0.5, 0.05, 1e-3):
            E1, q1, A1 = _total_energy(M, F + sigma * P, a_el)
            dwork = msh.work(M, q1) - msh.work(M, q0)
            dE = emu.delta_energy(M, F, P, sigma, A0, A1, a_el, dwork)
            scale = max(abs(E0), abs(E1))
            assert abs(dE - (E1 - E0)) <= 1e-12 * scale + 1e-10 * abs(E1 - E0), (trial, sigma, dE, E1 - E0)


def test_delta_energy_is_a_degree_six_polynomial():
    # Each element change is a polynomial of degree <= 6 in sigma (det is cubic,
    # the volume term squares it) and the ACAP residual is affine in sigma: the
    # seventh finite difference over equispaced sigma vanishes, the sixth does not.
    p = _hetero("cube2", seed=5)
    M = msh.build(p)
    a_el = msh.activation_per_element(M, p.activation)
    F = np.eye(3) + 0.2 * RNG.normal(size=(M.m, 3, 3))
    P = RNG.normal(size=(M.m, 3, 3))
    q0 = msh.acap_solve(M, F)
    A0 = msh.gather_A(M, q0)
    dq = msh.acap_solve(M, P, pinned=False)
    dA = msh.gather_A(M, dq)
    s = np.arange(8) * 0.5
    vals = np.array([emu.delta_energy(M, F, P, t, A0, A0 + t * dA, a_el) for t in s])
    d7 = np.diff(vals, 7)[0]
    d6 = np.diff(vals, 6)
    assert abs(d7) <= 1e-9 * np.abs(vals).max()
    assert np.abs(d6).max() > 1e-3 * np.abs(vals).max()


# ------------------------------------------------------------ block Hessian
def _exact_hessian(M, F, a_el):
    """Exact d2E/dF2 of the separated energy (eq. full-Hessian, weighted):
    blockdiag(vol d2Psi) + B_w - B_w G (G^T B_w G)^{-1} G^T B_w, built densely
    from the compatibility operator alone (no modes, no Woodbury)."""
    G = dense.dense_G(M)
    Bw = np.repeat(M.beta, 9)
    K = G.T @ (Bw[:, None] * G)
    Hel = M.vol[:, None, None] * mat.hess(F, M.mu, M.lhat, a_el, M.kf, M.fiber)
    H = np.zeros((9 * M.m, 9 * M.m))
    for i in range(M.m):
        H[9 * i:9 * i + 9, 9 * i:9 * i + 9] = Hel[i]
    H += np.diag(Bw) - (Bw[:, None] * G) @ np.linalg.solve(K, G.T * Bw[None, :])
    return H, Hel


def _clamp_inactive_state(M, a_el, scale=0.01, tries=50):
    """A state whose element Hessians are positive definite (the definiteness
    fix of Sec. 3.2.1 is then the identity): rotated stretches under tension
    in every direction, where the twist curvature of the isotropic energy is
    positive."""
    for _ in range(tries):
        S = 1.05 * np.eye(3) + scale * RNG.normal(size=(M.m, 3, 3))
        S = 0.5 * (S + np.transpose(S, (0, 2, 1)))
        Rm = np.stack([wl.random_rotation(RNG) for _ in range(M.m)])
        F = Rm @ S
        Hel = M.vol[:, None, None] * mat.hess(F, M.mu, M.lhat, a_el, M.kf, M.fiber)
        lam = np.linalg.eigvalsh(Hel)
        if (lam[:, 0] > 1e-6 * lam[:, -1]).all():
            return F
    raise AssertionError("no clamp-inactive state found")


@pytest.mark.parametrize("hessian,act", [("full", 0.5), ("split", 0.0), ("coupled", 0.5)])
def test_all_modes_woodbury_is_exact_newton(hessian, act):
    # With every mode kept (k = 3 n_f) the low-rank term reproduces
    # alpha W G L_w^{-1} G^T W exactly (eq. low-rank with nothing dropped), so
    # where the clamp is inactive the quasi-Newton direction is the exact
    # Newton direction of the separated energy (eq. full-Hessian).  The split
    # block structure is exact for the isotropic energy (no fiber term, a = 0);
    # the coupled 9x9 structure keeps the fiber coupling and is exact with it.
    p = _hetero("cube2", seed=1)
    p.activation = np.array([act, act])
    M = msh.build(p, modes=False)
    msh.compute_modes(M, M.free.size)
    a_el = msh.activation_per_element(M, p.activation)
    F = _clamp_inactive_state(M, a_el)
    q = msh.acap_solve(M, F)
    g = emu.grad_F(M, F, msh.gather_A(M, q), a_el).reshape(-1)
    Hx, Hel = _exact_hessian(M, F, a_el)
    H = emu.block_hessian(M, F, a_el, hessian)
    d = emu.direction(M, H, g.reshape(M.m, 9)).reshape(-1)
    dx = np.linalg.solve(Hx, g)
    assert np.abs(d - dx).max() <= 1e-8 * np.abs(dx).max()


def test_block_hessian_is_clamped_element_hessian_plus_beta():
    # Definiteness fix (Sec. 3.2.1): each full block is the PSD projection of
    # vol d2Psi (eigenvalues below 0 set to 0) plus beta I; checked against an
    # eigendecomposition written out here, at indefinite states.
    p = _hetero("cube2", seed=2)
    M = msh.build(p, modes=False)
    a_el = msh.activation_per_element(M, p.activation)
    F = np.eye(3) + 0.5 * RNG.normal(size=(M.m, 3, 3))
    Hel = M.vol[:, None, None] * mat.hess(F, M.mu, M.lhat, a_el, M.kf, M.fiber)
    lam, V = np.linalg.eigh(Hel)
    assert (lam.min(axis=1) < 0).any()
    ref = np.einsum("iab,ib,icb->iac", V, np.maximum(lam, 0.0), V) + M.beta[:, None, None] * np.eye(9)
    H = emu.block_hessian(M, F, a_el, "full")
    assert np.abs(H - ref).max() <= 1e-12 * np.abs(ref).max()


# ------------------------------------------------------------ heterogeneous solves
@pytest.mark.parametrize("weight_mode", [0, 1, 2])
def test_heterogeneous_emu_equals_moreau_newton(weight_mode):
    # P8 on a mesh with three materials (contrast 100), passive elements and
    # two groups: the minimizer does not depend on the solver.  With equal
    # materials the weightings coincide, so these cases pin the per-element
    # mu, lhat, weights and passive elements at solver level.
    p = _hetero("grid224", seed=0)
    M = msh.build(p, weight_mode=weight_mode)
    o1 = emu.solve(M, p.activation, tol=1e-11, max_iters=3000, hessian="split", trials="affine")
    assert o1["stats"]["converged"], o1["stats"]
    o2 = fem.moreau_solve(M, p.activation, tol=1e-11, max_iters=40)
    assert _disp_err(o1["q"], o2["q"], M.rest) < 1e-7
    assert np.abs(o1["F"] - o2["F"]).max() < 1e-7


def test_heterogeneous_weightings_differ():
    # the three weightings give three different minimizers on this mesh
    p = _hetero("grid224", seed=0)
    qs = [fem.moreau_solve(msh.build(p, weight_mode=wm, modes=False), p.activation, tol=1e-9, max_iters=40)["q"]
          for wm in (0, 1, 2)]
    rest = p.rest_xyz
    for a in range(3):
        for b in range(a + 1, 3):
            assert _disp_err(qs[a], qs[b], rest) > 1e-3


@pytest.mark.parametrize("weight_mode", [0, 2])
def test_heterogeneous_emu_equals_dense_newton(weight_mode):
    # P10 with two materials and a passive tet: brute-force F-form Newton with
    # the exact Hessian (eq. full-Hessian)
    p = _hetero("cube2", seed=4)
    M = msh.build(p, weight_mode=weight_mode)
    o1 = emu.solve(M, p.activation, tol=1e-11, max_iters=4000, trials="affine")
    o4 = dense.solve(M, p.activation, tol=1e-12)
    assert o1["stats"]["converged"], o1["stats"]
    assert _disp_err(o1["q"], o4["q"], M.rest) < 1e-8
    assert np.abs(o1["F"] - o4["F"]).max() < 1e-8


def test_coupled_blocks_are_psd_and_equal_split_without_fibers():
    # the coupled 9x9 blocks are positive semi-definite (+ beta I) at indefinite
    # states; with no activation they reduce to the split blocks, and with
    # activation they differ from them only by the fiber's sym/skew coupling
    p = _hetero("cube2", seed=6)
    M = msh.build(p, modes=False)
    F = np.eye(3) + 0.5 * RNG.normal(size=(M.m, 3, 3))
    a0 = np.zeros(M.m)
    assert np.abs(emu.block_hessian(M, F, a0, "coupled") - emu.block_hessian(M, F, a0, "split")).max() \
        <= 1e-12 * np.abs(emu.block_hessian(M, F, a0, "split")).max()
    a_el = msh.activation_per_element(M, p.activation)
    Hc = emu.block_hessian(M, F, a_el, "coupled") - M.beta[:, None, None] * np.eye(9)
    assert np.linalg.eigvalsh(Hc).min() >= -1e-10 * np.abs(Hc).max()
    Hs = emu.block_hessian(M, F, a_el, "split")
    assert np.abs(Hc + M.beta[:, None, None] * np.eye(9) - Hs).max() > 1e-6 * np.abs(Hs).max()


# ------------------------------------------------------------ affine bones
def _two_bones(kind="grid224", seed=2):
    """Two rigid-ish layers (bone 0 and bone 1, 100x stiffer) in a muscle column:
    the cube layers 1 and 3 along z; layer 0 rests on the pinned face."""
    p = wl.tiny(kind, activation=0.6, seed=seed)
    cz = p.rest_xyz[p.tets].mean(axis=1)[:, 2] / wl.H_EDGE
    layer = np.floor(cz).astype(int)
    p.bone = np.where(layer == 1, 0, np.where(layer == 3, 1, -1)).astype(np.int32)
    p.youngs = np.where(p.bone >= 0, 100 * wl.E_MUSCLE, p.youngs)
    p.group = np.where(p.bone >= 0, -1, 0).astype(np.int32)
    p.weight_mode = 1
    return p


def test_affine_bones_emu_equals_dense_newton():
    # Sec. 3.3 with a soft constraint: each bone's tets share one F_b.  The EMU
    # iteration on the reduced variables (summed gradients and element blocks,
    # the clamp after the sum) against brute-force Newton with the exact
    # Hessian of E over the same reduced variables
    p = _two_bones()
    M = msh.build(p, affine_bones=True, bone_slack=1e-1)
    assert M.m_red == M.m - int((p.bone >= 0).sum()) + 2
    o1 = emu.solve(M, p.activation, tol=1e-11, max_iters=4000, trials="affine")
    o4 = dense.solve(M, p.activation, tol=1e-12)
    assert o1["stats"]["converged"], o1["stats"]
    assert _disp_err(o1["q"], o4["q"], M.rest) < 1e-8
    assert np.abs(o1["F"] - o4["F"]).max() < 1e-8
    for b in (0, 1):
        Fb = o1["F"][p.bone == b]
        assert np.abs(Fb - Fb[0]).max() == 0.0


def test_affine_bone_gradient_is_the_derivative_of_the_energy():
    # the reduced gradient of a bone is dE/dF_b: central differences of E over
    # a common perturbation of every tet of the bone (E from a fresh ACAP solve)
    p = _two_bones()
    M = msh.build(p, affine_bones=True, bone_slack=1e-2)
    a_el = msh.activation_per_element(M, p.activation)
    rng = np.random.default_rng(5)
    Fr = np.eye(3) + 0.2 * rng.normal(size=(M.m_red, 3, 3))
    F = emu.expand(M, Fr)
    _, q, A = _total_energy(M, F, a_el)
    g = emu.reduce_sum(M, emu.grad_F(M, F, A, a_el))
    for b in (0, 1):
        r = M.red_of[np.nonzero(p.bone == b)[0][0]]
        for c in range(9):
            h = 1e-6
            D = np.zeros((M.m_red, 9))
            D[r, c] = h
            Ep = _total_energy(M, emu.expand(M, Fr + D.reshape(-1, 3, 3)), a_el)[0]
            Em = _total_energy(M, emu.expand(M, Fr - D.reshape(-1, 3, 3)), a_el)[0]
            fd = (Ep - Em) / (2 * h)
            assert abs(fd - g[r].reshape(9)[c]) <= 1e-6 * max(1.0, np.abs(g[r]).max())


def test_affine_bone_constraint_residual_scales_with_the_slack():
    # the soft constraint G_i q = F_b: its residual on the bone tets at the
    # minimizer shrinks in proportion to |eps_2|
    p = _two_bones()
    res = []
    for slack in (1e-1, 1e-3):
        M = msh.build(p, affine_bones=True, bone_slack=slack)
        o = dense.solve(M, p.activation, tol=1e-12)
        A = msh.gather_A(M, o["q"])
        sel = p.bone >= 0
        res.append(np.abs(A[sel] - o["F"][sel]).max())
    assert 50 < res[0] / res[1] < 200, res
