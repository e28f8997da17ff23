#!/usr/bin/env python3
"""Benchmark of the EMU quasi-Newton iteration on one MI355X.

A step is one full iteration of the method (Sec. 3.2.1 / Algorithm 1): element
pass, Woodbury Gram and solve, direction, ACAP triangular solve, exact
line-search polynomial, Armijo test and accept.  The headline workload is the
largest single-GPU configuration: the hinge limb, a 40x40x160 Kuhn grid
(1,536,000 tets), two bones joined by a pinned hinge line at mid-length, bone
core / tendon caps / muscle, helical fibers, four quadrant muscle groups at
the seeded activations of frame 0, FP64, warm state.

Prints ONE JSON line: element-iterations/s (whole job, inputs resident in HBM),
the roofline of the dominant kernel (HIP-event timing inside this process),
converged frame solves/s with p50/p99 latency, the mixed-precision line, the
192k-tet heterogeneous limb (its 20-frame activation ramp), the serving leg,
the alpha search and the CPU oracle baseline.
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
# once per vertex with n/m from the mesh).
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


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/*.md: FETCH_SIZE and WRITE_SIZE passes scaled by a plain copy
    kernel), or None when the summary was taken on a different kernel source
    or build (the hash covers kernels.hip and the build flags in build.py)."""
    import glob
    import hashlib
    pkg = os.path.join(ROOT, "paper_2006_08821_amd")
    h = hashlib.sha256()
    for src in (os.path.join(pkg, "csrc", "kernels.hip"), os.path.join(pkg, "build.py")):
        h.update(open(src, "rb").read())
    sha = h.hexdigest()
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        lines = open(f).read().splitlines()
        if f"kernels.hip + build.py sha256: {sha}" not in lines:
            continue
        for ln in lines:
            if ln.startswith(f"traffic: kernel={kernel} "):
                return float(ln.split("bytes=")[1].split()[0])
    return None


def timed_line(p, prec, args, label):
    """Host setup, warmup, then exactly ``steps`` iterations (a multiple of
    the graph length, so every replayed iteration is a timed one) from the
    warm state with the stop test off; per-kernel HIP-event times and
    per-phase times of a short extra run."""
    import torch
    from paper_2006_08821_amd.emu import Mesh
    t0 = time.time()
    mesh = Mesh(p, precision=prec, leaf_size=args.leaf_size)
    setup_s = time.time() - t0
    info = mesh.info()
    sync = args.iters_per_sync
    steps = max(sync, (args.steps + sync - 1) // sync * sync)
    mesh.solve(grad_tol=0.0, max_iters=args.warmup, iters_per_sync=sync, raise_on_error=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    q, st = mesh.solve(grad_tol=0.0, max_iters=steps, iters_per_sync=sync, raise_on_error=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    iters = max(1, st["iters"])
    prof = mesh.profile_kernels(reps=args.profile_reps)
    _, sp = mesh.solve(grad_tol=0.0, max_iters=2 * sync, iters_per_sync=sync, phase_timing=1,
                       raise_on_error=False)
    ni = max(1, sp["iters"])
    phases = {k: sp["ms_" + k] / ni for k in ("elem", "woodbury", "solve", "linesearch")}
    print(f"[bench] {label} {prec}: {iters} iterations in {dt*1e3:.1f} ms ({dt/iters*1e3:.3f} ms/iter), "
          f"setup {setup_s:.1f} s", file=sys.stderr, flush=True)
    return dict(mesh=mesh, info=info, st=st, dt=dt, iters=iters, prof=prof, setup_s=setup_s,
                q=q.cpu().numpy(), phases=phases)


def roofline(prof, m, n, nnz, mixed=False):
    """Roofline of the dominant kernel class by time (HIP events, on the
    mesh's stream): algorithmic bytes (or Gram flops) per launch over the
    average launch time."""
    dom = max((k for k in prof if algorithmic_bytes(k, m, n, nnz, mixed) is not None or k == "gram"),
              key=lambda k: prof[k])
    if dom == "gram":
        ach = GRAM_FLOPS_PER_ELEMENT * m / (prof[dom] * 1e-3) / 1e12
        peak = FP64_PEAK_TFLOPS
        return dict(bound="mfma", kernel=dom, achieved=ach, peak=peak, unit="TFLOP/s", frac=ach / peak,
                    traffic=measured_traffic(dom), ms=prof[dom])
    ach = algorithmic_bytes(dom, m, n, nnz, mixed) / (prof[dom] * 1e-3) / 1e9
    return dict(bound="hbm", kernel=dom, achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                traffic=measured_traffic(dom), ms=prof[dom])


def frame_solves(mesh, acts, tol, max_iters, keep_q=None):
    """Warm-started frame solves (each from the previous frame's equilibrium)
    to |g| <= tol; solves/s and latency over the frames, counting converged
    ones.  ``keep_q`` (a list) receives the last frame's positions."""
    import torch
    lat, conv, its = [], 0, 0
    q = None
    t_all = time.perf_counter()
    for a in acts:
        mesh.set_activation(a)
        t0 = time.perf_counter()
        q, st = mesh.solve(grad_tol=tol, max_iters=max_iters, raise_on_error=False)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t0) * 1e3)
        conv += st["status"] == 0
        its += st["iters"]
    t_all = time.perf_counter() - t_all
    if keep_q is not None and q is not None:
        keep_q.append(q.cpu().numpy())
    ok = conv == len(acts)
    return {"count": len(acts), "converged": conv, "grad_tol": tol, "iterations": its,
            "solves_per_s": len(acts) / t_all if ok else None,
            "latency_ms_p50": float(np.percentile(lat, 50)) if ok else None,
            "latency_ms_p99": float(np.percentile(lat, 99)) if ok else None,
            "wall_s": t_all}


def run(args):
    import torch
    from paper_2006_08821_amd import workloads as wl

    p, acts = wl.hinge_limb(40, 40, 160, frames=max(1, args.frames + 1))
    lines = {}
    for prec in (["fp64", "mixed"] if args.precision == "both" else [args.precision]):
        lines[prec] = timed_line(p, prec, args, "hinge_limb_40x40x160")
    main = lines.get("fp64") or lines[args.precision]
    m, n = p.n_tets, p.n_vertices
    nnz = main["info"]["factor_nnz"]
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
        "config": {"workload": "hinge_limb_40x40x160", "tets": m, "vertices": n,
                   "free_vertices": main["info"]["n_free"], "modes": main["info"]["n_modes"],
                   "alpha_hat": 10.0, "acap_weights": "volume", "factor_nnz": nnz,
                   "supernodes": main["info"]["n_supernodes"], "levels": main["info"]["n_levels"],
                   "groups": 4, "activation": [float(x) for x in p.activation],
                   "iters_per_sync": args.iters_per_sync, "setup_s": main["setup_s"]},
        "roofline": roofline(main["prof"], m, n, nnz),
        "kernel_ms": main["prof"],
        "phase_ms_per_iter": main["phases"],
    }
    if "mixed" in lines and "fp64" in lines:
        mx = lines["mixed"]
        q64, qmx = lines["fp64"]["q"], mx["q"]
        disp = np.abs(q64 - p.rest_xyz).max()
        out["mixed"] = {"value": m * mx["iters"] / mx["dt"], "ms_per_step": mx["dt"] / mx["iters"] * 1e3,
                        "dtype": "f32 element / f64 operator", "kernel_ms": mx["prof"],
                        "phase_ms_per_iter": mx["phases"],
                        "roofline": roofline(mx["prof"], m, n, nnz, mixed=True),
                        "position_diff_vs_fp64_after_same_iterations":
                            float(np.abs(qmx - q64).max() / disp) if disp > 0 else None}
    # converged frame solves of the hinge limb (seeded activations per frame,
    # each warm-started from the previous frame's equilibrium)
    last_q = {}
    if args.frames > 0:
        for prec, ln in lines.items():
            mesh = ln["mesh"]
            mesh.set_activation(acts[0])
            _, st0 = mesh.solve(grad_tol=args.frame_tol, max_iters=args.frame_max_iters, warm_start=0,
                                raise_on_error=False)
            kq = []
            fr = frame_solves(mesh, acts[1:args.frames + 1], args.frame_tol, args.frame_max_iters, keep_q=kq)
            if fr["converged"] == fr["count"] and kq:
                last_q[prec] = kq[0]
            fr["first_frame_from_rest"] = {"status": st0["status"], "iters": st0["iters"],
                                           "ms": st0["ms_total"]}
            key = "frames" if prec == "fp64" else "frames_mixed"
            out[key] = fr
            print(f"[bench] hinge frames {prec}: {fr['converged']}/{fr['count']} converged, "
                  f"{fr['iterations']} iterations, {fr['wall_s']:.1f} s", file=sys.stderr, flush=True)
    if "fp64" in last_q and "mixed" in last_q:
        # form (1): position error of the converged mixed frames against the
        # converged FP64 frames (same activations), relative to the displacement
        d = np.abs(last_q["fp64"] - p.rest_xyz).max()
        out["mixed"]["converged_position_err_vs_fp64"] = float(np.abs(last_q["mixed"] - last_q["fp64"]).max() / d)
    for ln in lines.values():
        ln["mesh"].close()
    if args.limb:
        out["heterogeneous_limb_20x20x80"] = limb_leg(args)
    if args.serve > 0:
        out["serving"] = serving(args)
    if args.alpha_search:
        out["alpha_search"] = alpha_search_leg()
    if args.adjoint:
        out["adjoint"] = adjoint_leg()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, args)
    return out


def limb_leg(args):
    """The 192k-tet heterogeneous limb: timed iterations (FP64 and mixed) and
    its 20-frame activation ramp a = t/20, each frame warm-started from the
    previous equilibrium, to |g| <= frame_tol."""
    from paper_2006_08821_amd import workloads as wl
    p, ramp = wl.heterogeneous_limb_ramp()
    p.activation = ramp[0].copy()
    out = {"workload": "heterogeneous limb 20x20x80 (192,000 tets), one group, 20-step ramp"}
    for prec in ("fp64", "mixed"):
        ln = timed_line(p, prec, args, "heterogeneous_limb_20x20x80")
        ln["mesh"].solve(grad_tol=0.0, max_iters=0, warm_start=0, raise_on_error=False)
        fr = frame_solves(ln["mesh"], ramp, args.frame_tol, args.frame_max_iters)
        out[prec] = {"element_iterations_per_s": p.n_tets * ln["iters"] / ln["dt"],
                     "ms_per_step": ln["dt"] / ln["iters"] * 1e3, "kernel_ms": ln["prof"],
                     "phase_ms_per_iter": ln["phases"], "ramp": fr}
        print(f"[bench] limb ramp {prec}: {fr['converged']}/{fr['count']} converged, {fr['iterations']} iterations, "
              f"{fr['wall_s']:.1f} s", file=sys.stderr, flush=True)
        ln["mesh"].close()
    return out


def adjoint_leg():
    """The adjoint of the 8-group marker limb (16x16x64, 98,304 tets): a
    forward solve from rest to |g| <= 1e-8, then dL/da for the marker loss
    L = 1/2 sum_markers |q_v - X_v|^2 (X: rest positions), and the adjoint's
    wall time against the forward solve's."""
    import torch
    from paper_2006_08821_amd import workloads as wl
    from paper_2006_08821_amd.emu import Mesh
    p = wl.adjoint_case()
    mesh = Mesh(p)
    mesh.solve(grad_tol=1e-8, max_iters=20000, warm_start=0)  # first call: graph capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    q, st = mesh.solve(grad_tol=1e-8, max_iters=20000, warm_start=0)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    mk = p.extra["markers"]
    dLdq = torch.zeros_like(q)
    dLdq[mk] = q[mk] - torch.as_tensor(p.rest_xyz[mk], dtype=q.dtype, device=q.device)
    mesh.solve_grad(dLdq)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g, sta = mesh.solve_grad(dLdq, stats=True)
    torch.cuda.synchronize()
    t_adj = time.perf_counter() - t0
    mesh.close()
    out = {"workload": "adjoint limb 16x16x64 (98,304 tets), 8 groups, 64 markers",
           "forward": {"status": st["status"], "iters": st["iters"], "s": t_fwd},
           "adjoint": {"status": sta["status"], "cg_steps": sta["iters"], "s": t_adj,
                       "ms_per_cg_step": t_adj / max(1, sta["iters"]) * 1e3},
           "adjoint_over_forward": t_adj / t_fwd}
    print(f"[bench] adjoint: forward {st['iters']} iterations {t_fwd:.3f} s, adjoint {sta['iters']} CG steps "
          f"{t_adj:.3f} s", file=sys.stderr, flush=True)
    return out


def alpha_search_leg():
    """Sec. 3.7 alpha search on the 4x4x16 box beam (a = 0.5): four candidates
    alpha_hat = 1, 10, 100, 1000 to |g| <= 1e-6 |g_0| (at most 3000
    iterations), as one batch on the serving loop and one after the other
    through the single-mesh solve."""
    import torch
    from paper_2006_08821_amd import workloads as wl
    from paper_2006_08821_amd.emu import Mesh, alpha_search
    p = wl.box_beam(4, 4, 16, activation=0.5)
    cands = (1.0, 10.0, 100.0, 1000.0)
    r = alpha_search(p, alpha_hats=cands, grad_rtol=1e-6, max_iters=3000)
    t0 = time.perf_counter()
    seq = []
    for a in cands:
        pa = p.copy()
        pa.alpha_hat = a
        _, st = Mesh(pa).solve(grad_tol=0.0, grad_rtol=1e-6, max_iters=3000, warm_start=0, raise_on_error=False)
        seq.append(st["iters"])
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    return {"workload": "box beam 4x4x16, a = 0.5", "alpha_hats": list(cands), "iters": r["iters"],
            "chosen_alpha_hat": r["alpha_hat"], "batched_s": r["wall_s"], "one_at_a_time_s": t_seq,
            "same_iters": seq == r["iters"]}


def serving(args):
    """The serving stream: the first ``args.serve`` requests of the seeded
    Poisson trace (200 req/s, 2k-300k tets log-uniform, 4 groups, random pin
    pattern) submitted in real time to the continuous-batching server, then the
    same requests solved one mesh at a time (create, solve, destroy) in arrival
    order.  Both to the same accuracy: |g| <= serve_tol from rest."""
    import threading
    import torch
    from paper_2006_08821_amd import workloads as wl
    from paper_2006_08821_amd.emu import Mesh, Server

    trace = wl.serving_trace(n_requests=args.serve)
    probs = [wl.serving_problem(r["dims"], r["activation"], r["pin_mode"]) for r in trace]
    opts = dict(grad_tol=args.serve_tol, max_iters=args.serve_max_iters, warm_start=0)

    srv = Server(max_slots=args.serve_slots, setup_threads=args.serve_setup_threads,
                 iters_per_round=args.serve_iters_per_round)
    tickets = [None] * len(probs)
    t_start = time.perf_counter()

    def feeder():
        for k, (r, p) in enumerate(zip(trace, probs)):
            dt = r["arrival"] - (time.perf_counter() - t_start)
            if dt > 0:
                time.sleep(dt)
            tickets[k] = srv.submit(p, **opts)

    th = threading.Thread(target=feeder)
    th.start()
    th.join()
    res = [srv.wait(t) for t in tickets]
    rep = srv.report()
    srv.close()
    lat = np.array([tm["t_finish"] - tm["t_submit"] for _, _, tm in res]) * 1e3
    setup = np.array([tm["t_setup_done"] - tm["t_submit"] for _, _, tm in res]) * 1e3
    queue = np.array([tm["t_admit"] - tm["t_setup_done"] for _, _, tm in res]) * 1e3
    span = max(tm["t_finish"] for _, _, tm in res) - min(tm["t_submit"] for _, _, tm in res)
    el_it = sum(p.n_tets * st["iters"] for p, (_, st, _) in zip(probs, res))
    n_conv = int(sum(st["status"] == 0 for _, st, _ in res))
    served = {"requests": len(res), "converged": n_conv,
              "requests_per_s": len(res) / span, "element_iterations_per_s": el_it / span,
              "latency_ms_p50": float(np.percentile(lat, 50)), "latency_ms_p99": float(np.percentile(lat, 99)),
              "setup_ms_p50": float(np.percentile(setup, 50)), "setup_ms_p99": float(np.percentile(setup, 99)),
              "queue_ms_p50": float(np.percentile(queue, 50)),
              "peak_active": rep["peak_active"], "peak_resident_mb": rep["peak_resident_bytes"] / 1e6,
              "rounds": rep["rounds"]}
    print(f"[bench] served {len(res)} requests in {span:.2f} s", file=sys.stderr, flush=True)

    # plain: one mesh at a time, in arrival order, same options
    lat1 = []
    el_it1 = 0
    conv1 = 0
    t_start = time.perf_counter()
    for r, p in zip(trace, probs):
        now = time.perf_counter() - t_start
        if now < r["arrival"]:
            time.sleep(r["arrival"] - now)
        mesh = Mesh(p)
        _, st = mesh.solve(raise_on_error=False, **opts)
        torch.cuda.synchronize()
        mesh.close()
        lat1.append((time.perf_counter() - t_start - r["arrival"]) * 1e3)
        el_it1 += p.n_tets * st["iters"]
        conv1 += st["status"] == 0
    span1 = time.perf_counter() - t_start - trace[0]["arrival"]
    plain = {"requests": len(trace), "converged": int(conv1), "requests_per_s": len(trace) / span1,
             "element_iterations_per_s": el_it1 / span1,
             "latency_ms_p50": float(np.percentile(lat1, 50)), "latency_ms_p99": float(np.percentile(lat1, 99))}
    print(f"[bench] plain {len(trace)} requests in {span1:.2f} s", file=sys.stderr, flush=True)
    return {"workload": f"serving trace, first {len(trace)} requests (Poisson 200/s, 2k-300k tets)",
            "grad_tol": args.serve_tol, "max_iters": args.serve_max_iters,
            "served": served, "plain_one_at_a_time": plain}


def cpu_baseline(p, args):
    """The FP64 oracle (NumPy/SciPy, as it stands) timed on this host on a
    bounded sample of the headline workload: one quasi-Newton iteration (fresh
    ACAP solve per Armijo trial, as Algorithm 1 does) on the bottom slab of the
    hinge limb, its tets with centroid below z = 20 cube edges (a 40x40x20
    sub-mesh of the same generator: 192,000 tets, bone core, tendon cap,
    helical fibers, the z = 0 face pinned), oracle setup (factor, modes)
    excluded.  Run once on one core and once with every BLAS thread the host
    offers (NumPy's element-wise work is single-threaded either way)."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import emu as oemu
    from oracle import mesh as omesh
    from paper_2006_08821_amd import workloads as wl
    sub = wl.sub_problem(p, z_max=20 * wl.H_EDGE)
    t0 = time.perf_counter()
    M = omesh.build(sub)
    setup_s = time.perf_counter() - t0
    blas = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    runs = {}
    for label, limit in (("one_core", 1), ("all_cores", blas)):
        with threadpool_limits(limits=limit):
            t0 = time.perf_counter()
            o = oemu.solve(M, sub.activation, max_iters=args.cpu_iters, hessian="split")
            dt = time.perf_counter() - t0
        it = max(1, o["stats"]["iters"])
        runs[label] = dict(value=sub.n_tets * it / dt, seconds=dt, iterations=it, threads=limit)
        print(f"[bench] oracle {label}: {it} iteration(s) in {dt:.1f} s", file=sys.stderr, flush=True)
    r1 = runs["one_core"]
    return {"value": r1["value"], "unit": "element-iterations/s", "cores": 1, "kind": "oracle",
            "sample": f"{r1['iterations']} oracle iteration(s) on the 40x40x20 bottom slab of the hinge limb "
                      f"({sub.n_tets} tets), setup ({setup_s:.0f} s) excluded, one core: {r1['seconds']:.1f} s",
            "all_cores": {"value": runs["all_cores"]["value"], "cores": blas,
                          "seconds": runs["all_cores"]["seconds"],
                          "note": "BLAS threads; element-wise NumPy work and SuperLU stay single-threaded"},
            "host_cpus": os.cpu_count()}


def calibrate_copy(mib):
    """A plain elementwise copy (y = 1.0 * x, FP64) of known size: under a
    counter run its FETCH_SIZE / WRITE_SIZE give the factor between the
    counters and bytes actually moved."""
    import torch
    n = mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(f"[bench] copy calibration: 3 x ({n * 8} B read + {n * 8} B written)", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=384)
    ap.add_argument("--warmup", type=int, default=32)
    ap.add_argument("--iters-per-sync", type=int, default=32)
    ap.add_argument("--precision", default="both", choices=["fp64", "mixed", "both"])
    ap.add_argument("--frames", type=int, default=4, help="converged hinge-limb frames after frame 0")
    ap.add_argument("--frame-tol", type=float, default=1e-8)
    ap.add_argument("--frame-max-iters", type=int, default=20000)
    ap.add_argument("--limb", type=int, default=1, help="run the 192k-tet limb leg (0: skip)")
    ap.add_argument("--profile-reps", type=int, default=20)
    ap.add_argument("--leaf-size", type=int, default=0, help="nested-dissection leaf size (0: library default)")
    ap.add_argument("--cpu-iters", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve", type=int, default=24, help="requests of the serving trace (0: skip)")
    ap.add_argument("--serve-tol", type=float, default=1e-8)
    ap.add_argument("--serve-max-iters", type=int, default=20000)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-setup-threads", type=int, default=0,
                    help="host threads for mesh setups (0: the library default)")
    ap.add_argument("--serve-iters-per-round", type=int, default=0,
                    help="iterations per scheduler round (0: the library default)")
    ap.add_argument("--alpha-search", type=int, default=1, help="run the alpha-search leg (0: skip)")
    ap.add_argument("--adjoint", type=int, default=1, help="run the adjoint leg (0: skip)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (for scaling HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: measures one GPU only; runs on more than one GPU are not supported "
              "(the path would split each mesh's elements over the GPUs and all-reduce the Woodbury "
              "Gram and the line-search sums; not implemented here).",
              file=sys.stderr)
        sys.exit(2)
    out = run(args)
    if args.calibrate_copy_mib > 0:
        calibrate_copy(args.calibrate_copy_mib)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
