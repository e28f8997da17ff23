"""Write tests/golden/hinge40x40x160_state.json: the oracle's ACAP solve,
energy, exact gradient and quasi-Newton direction of the hinge limb
40x40x160 (1.536M tets) at a seeded state F, on sampled elements and
vertices.  Calls only the oracle and the input generator.

    python tests/golden/make_hinge_golden.py   # about 15 minutes, ~12 GB RAM
"""
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import emu as oemu  # noqa: E402
from oracle import mesh as omesh  # noqa: E402
from paper_2006_08821_amd import workloads as wl  # noqa: E402

SEED = 5
AMP = 0.05
N_SAMPLE = 96


def seeded_state(m, seed=SEED, amp=AMP):
    """F_i = I + amp N(0, 1)^{3x3}, i in user tet order (shared with the test)."""
    rng = np.random.default_rng(seed)
    return np.eye(3) + amp * rng.normal(size=(m, 3, 3))


def sample_ids(count, n, seed):
    return np.sort(np.random.default_rng(seed).choice(n, size=count, replace=False))


def main():
    t0 = time.time()
    p = wl.hinge_limb(40, 40, 160, frames=1)[0]
    M = omesh.build(p)
    print(f"setup {time.time() - t0:.0f}s", flush=True)
    F = seeded_state(M.m)
    a_el = omesh.activation_per_element(M, p.activation)
    q = omesh.acap_solve(M, F)
    A = omesh.gather_A(M, q)
    E = math.fsum(oemu.element_energy(M, F, A, a_el))
    g = oemu.grad_F(M, F, A, a_el)
    gn = math.sqrt(math.fsum((g * g).reshape(-1)))
    H = oemu.block_hessian(M, F, a_el, "split")
    d = oemu.direction(M, H, g.reshape(M.m, 9)).reshape(M.m, 3, 3)
    print(f"evaluated {time.time() - t0:.0f}s", flush=True)
    el = sample_ids(N_SAMPLE, M.m, 1)
    vx = sample_ids(N_SAMPLE, M.n, 2)
    out = dict(
        workload="hinge_limb 40x40x160 (1,536,000 tets), activation of frame 0, weight_mode %d" % p.weight_mode,
        state=dict(seed=SEED, amp=AMP, rule="F_i = I + amp * default_rng(seed).normal(size=(m,3,3))"),
        n_modes=int(3 * M.nu.size), nu=M.nu.tolist(),
        energy=E, grad_norm=gn, grad_max=float(np.abs(g).max()), dir_max=float(np.abs(d).max()),
        elements=el.tolist(), grad=g[el].reshape(-1, 9).tolist(), direction=d[el].reshape(-1, 9).tolist(),
        vertices=vx.tolist(), q=q[vx].tolist(), q_max=float(np.abs(q).max()),
    )
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "hinge40x40x160_state.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path} in {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
