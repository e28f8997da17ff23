"""Write tests/golden/affine_refs.json: converged minimizers with affine bones
(Sec. 3.3: the tets of each bone share one deformation gradient, tied to the
continuous mesh with the slack eps_2), from the oracle's EMU iteration on the
reduced variables (O1; pinned against brute-force Newton on a small mesh).
Calls only the oracle and the input generator.

    python tests/golden/make_affine_golden.py    # about 6 minutes
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import emu as oemu  # noqa: E402
from oracle import mesh as omesh  # noqa: E402
from paper_2006_08821_amd import workloads as wl  # noqa: E402

TOL = 1e-8


def cases():
    """name -> (Problem, bone slack); the tests rebuild the same inputs."""
    return {
        "limb5x5x20": (wl.limb(5, 5, 20, n_groups=4, activation=np.array([0.5, 0.2, 0.8, 0.4])), 1e-3),
        "hinge6x6x24": (wl.hinge_limb(6, 6, 24, frames=1)[0], 1e-1),
    }


def main():
    out = {}
    for name, (p, slack) in cases().items():
        t0 = time.time()
        M = omesh.build(p, affine_bones=True, bone_slack=slack)
        r = oemu.solve(M, p.activation, tol=TOL, max_iters=20000, hessian="split", trials="affine")
        assert r["stats"]["converged"], r["stats"]
        bones = sorted(set(int(b) for b in p.bone if b >= 0))
        Fb = [r["F"][np.nonzero(p.bone == b)[0][0]].tolist() for b in bones]
        out[name] = dict(slack=slack, tol=TOL, q=r["q"].tolist(), energy=r["stats"]["energy"],
                         gnorm=r["stats"]["gnorm"], iters=r["stats"]["iters"], bone_F=Fb)
        print(f"{name}: {r['stats']['iters']} iterations, |grad| {r['stats']['gnorm']:.1e}, "
              f"{time.time() - t0:.0f}s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "affine_refs.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
