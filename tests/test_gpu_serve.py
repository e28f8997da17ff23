"""GPU tests of the serving loop (continuous batching), through the C ABI.

* A cold-started request gives the same bits alone, in a mix of other
  requests (different sizes, pin patterns and precisions) and through the
  plain single-mesh solve, and matches the oracle.
* Admission respects the HBM budget; a mesh that alone exceeds it fails with
  EMU_E_OOM; repeated meshes reuse the cached setup and resident state.
"""
import numpy as np
import pytest

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


def _server(**kw):
    from paper_2006_08821_amd.emu import Server
    return Server(**kw)


def _disp_err(q, qref, rest):
    return float(np.abs(q - qref).max() / np.abs(qref - rest).max())


def _mix():
    rng = np.random.default_rng(5)
    out = []
    for dims, pm in [((5, 5, 20), 0), ((6, 6, 24), 1), ((5, 5, 20), 2), ((7, 7, 28), 0), ((4, 4, 16), 1)]:
        out.append(wl.serving_problem(dims, rng.uniform(0, 1, 4), pm))
    return out


OPTS = dict(grad_tol=0.0, grad_rtol=1e-6, max_iters=200, warm_start=0)


def test_alone_equals_in_mix(torch):
    target = wl.box_beam()                      # 1536 tets, a = 0.5
    others = _mix()
    s = _server(iters_per_round=8)
    t = s.submit(target, grad_tol=1e-8, max_iters=2000, warm_start=0)
    q_alone, st_alone, _ = s.wait(t)
    s.close()
    assert st_alone["status"] == 0, st_alone

    s = _server(iters_per_round=8)
    tickets = [s.submit(p, **OPTS) for p in others[:3]]
    tickets.append(s.submit(others[3], precision="mixed", **OPTS))
    tt = s.submit(target, grad_tol=1e-8, max_iters=2000, warm_start=0)
    tickets.append(s.submit(others[4], **OPTS))
    q_mix, st_mix, tm = s.wait(tt)
    res = [s.wait(k) for k in tickets]
    rep = s.report()
    s.close()
    assert rep["peak_active"] >= 2, rep
    assert np.array_equal(q_alone, q_mix)
    assert st_alone["iters"] == st_mix["iters"]
    assert st_alone["energy"] == st_mix["energy"]
    for q, st, _ in res:
        assert st["status"] in (0, 3), st
        assert np.isfinite(q).all()

    # the same solve through the single-mesh path, and the oracle
    from paper_2006_08821_amd.emu import Mesh
    M = omesh.build(target, modes=False)
    mesh = Mesh(target)
    q_plain, st_plain = mesh.solve(grad_tol=1e-8, max_iters=2000, warm_start=0)
    q_plain = q_plain.cpu().numpy()
    assert st_plain["iters"] == st_mix["iters"]
    assert st_plain["energy"] == st_mix["energy"]
    assert np.array_equal(q_plain, q_mix)
    ref = ofem.moreau_solve(M, target.activation, tol=1e-11)["q"]
    assert _disp_err(q_mix, ref, M.rest) <= 1e-6


def test_each_mix_member_matches_alone(torch):
    probs = _mix()
    s = _server(iters_per_round=16)
    tk = [s.submit(p, precision=("mixed" if i == 3 else "fp64"), **OPTS) for i, p in enumerate(probs)]
    mixed = [s.wait(k) for k in tk]
    s.close()
    for i, p in enumerate(probs):
        s = _server(iters_per_round=4)
        q, st, _ = s.wait(s.submit(p, precision=("mixed" if i == 3 else "fp64"), **OPTS))
        s.close()
        assert np.array_equal(q, mixed[i][0]), i
        assert st["iters"] == mixed[i][1]["iters"]


def test_budget_and_oom(torch):
    probs = _mix()
    s = _server()
    sizes = []
    for p in probs:
        _, st, tm = s.wait(s.submit(p, **OPTS))
        sizes.append(tm["device_bytes"])
    s.close()
    budget = int(1.2 * max(sizes))
    s = _server(hbm_budget_bytes=budget, max_slots=8)
    tk = [s.submit(p, **OPTS) for p in probs + probs]
    out = [s.wait(k) for k in tk]
    rep = s.report()
    assert rep["peak_resident_bytes"] <= budget, (rep, budget)
    assert rep["completed"] + rep["failed"] == len(tk)
    assert all(st["status"] in (0, 3) for _, st, _ in out)
    # second pass over the same meshes: cached setups
    assert all(tm["setup_cached"] == 1 for _, _, tm in out[len(probs):])
    big = wl.serving_problem((9, 9, 36), [0.5] * 4, 0)
    q, st, tm = s.wait(s.submit(big, **OPTS))
    assert st["status"] == 6  # EMU_E_OOM: the mesh alone exceeds the budget
    s.close()


def test_warm_reuse_of_resident_mesh(torch):
    p = wl.box_beam(2, 2, 8, activation=0.5)
    s = _server()
    q0, st0, tm0 = s.wait(s.submit(p, grad_tol=1e-9, max_iters=3000, warm_start=0))
    q1, st1, tm1 = s.wait(s.submit(p, grad_tol=1e-9, max_iters=3000, warm_start=1))
    s.close()
    assert st0["status"] == 0 and st1["status"] == 0
    assert tm1["setup_cached"] == 1
    # restarting at the converged state: one check, no further iterations
    assert st1["iters"] <= 1
    assert _disp_err(q1, q0, p.rest_xyz) <= 1e-8


def test_failed_request_releases_slot_and_memory(torch, monkeypatch):
    # the fault hook EMU_FAULT=linesearch:T fails the request with ticket T in
    # its first round; it releases its slot and its mesh's device memory, and
    # every other request of the mix ends with the same bits as without it
    probs = _mix()[:4]
    s = _server(iters_per_round=8)
    tk = [s.submit(p, **OPTS) for p in probs]
    ref = [s.wait(k) for k in tk]
    s.close()
    monkeypatch.setenv("EMU_FAULT", f"linesearch:{tk[1]}")
    s = _server(iters_per_round=8)
    tk2 = [s.submit(p, **OPTS) for p in probs]
    assert tk2 == tk
    out = [s.wait(k) for k in tk2]
    rep = s.report()
    s.close()
    assert out[1][1]["status"] == 4  # EMU_E_LINESEARCH
    for i in (0, 2, 3):
        assert out[i][1]["status"] == ref[i][1]["status"] and out[i][1]["status"] in (0, 3)
        assert np.array_equal(out[i][0], ref[i][0]), i
    n_ok = sum(ref[i][1]["status"] == 0 for i in (0, 2, 3))
    assert rep["completed"] == n_ok and rep["failed"] == 4 - n_ok, rep
    kept = sum(out[i][2]["device_bytes"] for i in (0, 2, 3))
    assert rep["resident_bytes"] == kept, (rep, kept, out[1][2]["device_bytes"])
