#!/usr/bin/env python3
"""Benchmark of the EMU quasi-Newton iteration on one MI355X.

A step is one full iteration of the method (Sec. 3.2.1 / Algorithm 1): element
pass, Woodbury Gram and solve, direction, ACAP triangular solve, exact
line-search polynomial, Armijo test and accept.  The workload is the
heterogeneous limb: a 20x20x80 Kuhn grid (192,000 tets), bone core / tendon
caps / muscle, helical fibers, z=0 face pinned, one muscle group on a 20-step
activation ramp (frame 1, a = 0.05, warm-started from rest).

Prints ONE JSON line: element-iterations/s (whole job, inputs resident in HBM),
the roofline of the dominant kernel (HIP-event timing inside this process),
frame solves/s with p50/p99 latency, the mixed-precision line and the CPU
oracle baseline.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6

# Algorithmic bytes per element of each HBM-bound kernel (FP64 path; unique
# bytes: static element data, state and intermediates, vertex gathers counted
# once per vertex with n/m from the mesh).  See the design notes.
STATIC_B = 148          # 4 ids, D_m^-1, vol, mu, lhat, w, fiber, group


def algorithmic_bytes(kernel, m, n, nnz, mixed=False):
    t = 4 if mixed else 8
    vq = 24.0 * n / m                      # one 3-vector per vertex
    if kernel == "element":
        return m * (STATIC_B + 120 + 72 + 120 + vq + 9 * t + 27 * t)
    if kernel == "direction":
        return m * (16 + 72 + 8 + 72 + 27 * t + 9 * t + vq + 72 + 96)
    if kernel == "lscoef":
        return m * (STATIC_B + 120 + 72 + 2 * vq)
    if kernel == "rhs":
        return m * 96 + n * 24 * 2
    if kernel in ("fwd_sweep", "bwd_sweep"):
        return nnz * 8.0
    return None


GRAM_FLOPS_PER_ELEMENT = 9.6e3   # Z g (9x48x3 MAC) + 1176 x 3 MAC, x2 flops


def run(args):
    import torch
    from paper_2006_08821_amd import workloads as wl
    from paper_2006_08821_amd.emu import Mesh

    p, ramp = wl.heterogeneous_limb_ramp()
    p.activation = ramp[0].copy()
    res = {}
    lines = {}
    for prec in (["fp64", "mixed"] if args.precision == "both" else [args.precision]):
        t0 = time.time()
        mesh = Mesh(p, precision=prec)
        setup_s = time.time() - t0
        info = mesh.info()
        # warmup
        mesh.solve(grad_tol=0.0, max_iters=args.warmup, raise_on_error=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = mesh.solve(grad_tol=0.0, max_iters=args.steps, iters_per_sync=32, raise_on_error=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        iters = max(1, st["iters"])
        prof = mesh.profile_kernels(reps=args.profile_reps)
        lines[prec] = dict(mesh=mesh, info=info, st=st, dt=dt, iters=iters, prof=prof, setup_s=setup_s)
        print(f"[bench] {prec}: {iters} iterations in {dt*1e3:.1f} ms ({dt/iters*1e3:.3f} ms/iter), "
              f"|g| {st['grad_norm']:.3e}, setup {setup_s:.1f} s", file=sys.stderr, flush=True)
    main = lines.get("fp64") or lines[args.precision]
    m, n = p.n_tets, p.n_vertices
    nnz = main["info"]["factor_nnz"]
    # roofline of the dominant kernel by time
    prof = main["prof"]
    dom = max((k for k in prof if algorithmic_bytes(k, m, n, nnz) is not None or k == "gram"),
              key=lambda k: prof[k])
    if dom == "gram":
        flops = GRAM_FLOPS_PER_ELEMENT * m
        ach = flops / (prof[dom] * 1e-3) / 1e12
        roof = dict(bound="alu", kernel=dom, achieved=ach, peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                    frac=ach / FP64_PEAK_TFLOPS, traffic=None, ms=prof[dom])
    else:
        b = algorithmic_bytes(dom, m, n, nnz)
        ach = b / (prof[dom] * 1e-3) / 1e9
        roof = dict(bound="hbm", kernel=dom, achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=ach / HBM_PEAK_GBS, traffic=None, ms=prof[dom])
    value = m * main["iters"] / main["dt"]
    out = {
        "metric": "element-iterations/s",
        "value": value,
        "unit": "element-iterations/s",
        "n_gpus": 1,
        "steps": main["iters"],
        "warmup": args.warmup,
        "ms_per_step": main["dt"] / main["iters"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "heterogeneous_limb_20x20x80", "tets": m, "vertices": n,
                   "free_vertices": main["info"]["n_free"], "modes": main["info"]["n_modes"],
                   "alpha_hat": 10.0, "factor_nnz": nnz, "supernodes": main["info"]["n_supernodes"],
                   "levels": main["info"]["n_levels"], "activation": float(p.activation[0])},
        "roofline": roof,
        "kernel_ms": prof,
    }
    if "mixed" in lines and "fp64" in lines:
        mx = lines["mixed"]
        out["mixed"] = {"value": m * mx["iters"] / mx["dt"], "ms_per_step": mx["dt"] / mx["iters"] * 1e3,
                        "dtype": "f32 element / f64 operator", "kernel_ms": mx["prof"]}
    # frame solves of the activation ramp (warm-started), latency percentiles
    if args.frames > 0:
        mesh = main["mesh"]
        lat = []
        conv = 0
        tot_it = 0
        mesh.solve(grad_tol=0.0, max_iters=0, warm_start=0, raise_on_error=False)
        t_all = time.perf_counter()
        for f in range(args.frames):
            mesh.set_activation(ramp[f])
            t0 = time.perf_counter()
            _, st = mesh.solve(grad_tol=args.frame_tol, max_iters=args.frame_max_iters, raise_on_error=False)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - t0) * 1e3)
            conv += st["status"] == 0
            tot_it += st["iters"]
        t_all = time.perf_counter() - t_all
        out["frames"] = {"count": args.frames, "converged": conv, "grad_tol": args.frame_tol,
                         "max_iters_per_frame": args.frame_max_iters, "iterations": tot_it,
                         "solves_per_s": args.frames / t_all,
                         "latency_ms_p50": float(np.percentile(lat, 50)),
                         "latency_ms_p99": float(np.percentile(lat, 99))}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, args)
    return out


def cpu_baseline(p, args):
    """The FP64 oracle (NumPy/SciPy) timed on this host on a bounded sample: one
    quasi-Newton iteration of the same workload (setup excluded)."""
    from oracle import emu as oemu
    from oracle import mesh as omesh
    M = omesh.build(p)
    t0 = time.perf_counter()
    o = oemu.solve(M, p.activation, max_iters=args.cpu_iters, hessian="split")
    dt = time.perf_counter() - t0
    it = max(1, o["stats"]["iters"])
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": p.n_tets * it / dt, "unit": "element-iterations/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{it} oracle iteration(s) of the same 192k-tet workload from rest "
                      f"(fresh ACAP solve per Armijo trial), mesh setup excluded; {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--precision", default="both", choices=["fp64", "mixed", "both"])
    ap.add_argument("--frames", type=int, default=20)
    ap.add_argument("--frame-tol", type=float, default=1e-6)
    ap.add_argument("--frame-max-iters", type=int, default=400)
    ap.add_argument("--profile-reps", type=int, default=20)
    ap.add_argument("--cpu-iters", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU only; multi-GPU runs are not supported "
              "(the sharded design is described in the design notes).", file=sys.stderr)
        sys.exit(2)
    out = run(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
