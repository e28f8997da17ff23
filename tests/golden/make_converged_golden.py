"""Write tests/golden/converged_refs.json: the oracle's converged Moreau-
envelope Newton minimizers (O2) of small heterogeneous workloads (bone core,
tendon caps, helical fibers, volume ACAP weights, several groups and pin
patterns), and the q-space adjoint (O6) of the eight-group marker loss.  Calls
only the oracle and the input generator.

    python tests/golden/make_converged_golden.py    # about 6 minutes
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import adjoint as oadj  # noqa: E402
from oracle import fem as ofem  # noqa: E402
from oracle import mesh as omesh  # noqa: E402
from paper_2006_08821_amd import workloads as wl  # noqa: E402

LIMB_ACT = [0.5, 0.2, 0.8, 0.4]


def cases():
    """name -> Problem; the tests rebuild the same inputs by these calls."""
    rng = np.random.default_rng(3)
    serve = [wl.serving_problem(d, rng.uniform(0, 1, 4), pm) for d, pm in [((5, 5, 20), 0), ((5, 5, 20), 1),
                                                                          ((6, 6, 24), 2)]]
    return {
        "limb5x5x20": wl.limb(5, 5, 20, n_groups=4, activation=np.array(LIMB_ACT)),
        "hinge6x6x24": wl.hinge_limb(6, 6, 24, frames=1)[0],
        "serve5x5x20_pm0": serve[0],
        "serve5x5x20_pm1": serve[1],
        "serve6x6x24_pm2": serve[2],
    }


def adjoint_problem():
    return wl.adjoint_case(6, 6, 24)


def _solve(p, a):
    M = omesh.build(p, modes=False)
    r = ofem.moreau_solve(M, a, tol=1e-10, max_iters=60)
    assert r["gnorm"] <= 1e-10, r["gnorm"]
    return M, r


def main():
    out = {}
    for name, p in cases().items():
        t0 = time.time()
        _, r = _solve(p, p.activation)
        out[name] = dict(activation=p.activation.tolist(), q=r["q"].tolist(), energy=r["energy"],
                         gnorm=r["gnorm"], iters=r["iters"])
        print(f"{name}: {r['iters']} Newton steps, |grad| {r['gnorm']:.1e}, {time.time() - t0:.0f}s", flush=True)
    p = adjoint_problem()
    markers = p.extra["markers"]
    t0 = time.time()
    _, rt = _solve(p, p.extra["a_star"])
    target = rt["q"][markers]
    M, r = _solve(p, p.activation)
    L, g = oadj.activation_gradient(M, p.activation, r["q"], markers, target)
    out["adjoint6x6x24"] = dict(markers=markers.tolist(), a_star=p.extra["a_star"].tolist(),
                                activation=p.activation.tolist(), target=target.tolist(), q=r["q"].tolist(),
                                loss=L, dL_da=g.tolist())
    print(f"adjoint6x6x24: {time.time() - t0:.0f}s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "converged_refs.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
