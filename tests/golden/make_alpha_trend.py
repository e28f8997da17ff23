"""Writes alpha_trend_box2x2x8.json: iteration counts of the oracle's EMU
iteration (split blocks, affine trials) on the 2x2x8 box beam at a = 0.5 for
alpha_hat = 1, 10, 100, 1000, to |g| <= 1e-6 |g_0| with at most 3000
iterations (Sec. 3.7: the count rises with alpha, sharply past a threshold).

    python tests/golden/make_alpha_trend.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import emu, mesh  # noqa: E402
from paper_2006_08821_amd import workloads as wl  # noqa: E402


def main():
    p = wl.box_beam(2, 2, 8, activation=0.5)
    out = {"problem": "box_beam(2, 2, 8, activation=0.5)", "grad_rtol": 1e-6, "max_iters": 3000,
           "alpha_hats": [], "iters": [], "converged": []}
    for ah in (1.0, 10.0, 100.0, 1000.0):
        M = mesh.build(p, alpha_hat=ah)
        a_el = mesh.activation_per_element(M, p.activation)
        g0 = emu.gradient_norm(M, emu.rest_state(M), a_el)[0]
        o = emu.solve(M, p.activation, tol=1e-6 * g0, max_iters=3000, hessian="split", trials="affine")
        out["alpha_hats"].append(ah)
        out["iters"].append(o["stats"]["iters"])
        out["converged"].append(bool(o["stats"]["converged"]))
    with open(os.path.join(HERE, "alpha_trend_box2x2x8.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
