"""Python front end of the EMU library: meshes, solves, evaluation, serving.

PyTorch is used only for device memory and the current HIP stream; all
computation runs in libemu.so.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from . import _lib
from ._lib import check, dptr, iptr

PRECISION = {"fp64": 0, "mixed": 1}


WEIGHT_MODES = {"stiffness": 0, "volume": 1, "paper": 2}


BLOCKS = {"split": 0, "coupled": 1}


def _desc_arrays(problem, alpha_hat=None, n_modes=None, precision="fp64", weight_mode=None,
                 leaf_size=0, mu_ref=0.0, fiber_k=0.0, hessian_blocks="split", affine_bones=False,
                 bone_slack=0.0):
    """Contiguous host arrays + the emu_mesh_desc struct that points at them.
    ``weight_mode`` None takes the problem's (``Problem.weight_mode``)."""
    if weight_mode is None:
        weight_mode = getattr(problem, "weight_mode", 0)
    if isinstance(weight_mode, str):
        weight_mode = WEIGHT_MODES[weight_mode]
    keep = dict(
        rest=np.ascontiguousarray(problem.rest_xyz, np.float64),
        tets=np.ascontiguousarray(problem.tets, np.int32),
        youngs=np.ascontiguousarray(problem.youngs, np.float64),
        poisson=np.ascontiguousarray(problem.poisson, np.float64),
        fiber=np.ascontiguousarray(problem.fiber, np.float64),
        group=np.ascontiguousarray(problem.group, np.int32),
        pins=np.ascontiguousarray(problem.pins, np.int32),
        pin_xyz=np.ascontiguousarray(problem.pin_xyz, np.float64),
    )
    if getattr(problem, "bone", None) is not None:
        keep["bone"] = np.ascontiguousarray(problem.bone, np.int32)
    d = _lib.MeshDesc()
    d.n_vertices = keep["rest"].shape[0]
    d.n_tets = keep["tets"].shape[0]
    d.n_groups = int(len(problem.activation))
    d.n_pins = keep["pins"].shape[0]
    d.rest_xyz = dptr(keep["rest"])
    d.tets = iptr(keep["tets"])
    d.youngs = dptr(keep["youngs"])
    d.poisson = dptr(keep["poisson"])
    d.fiber = dptr(keep["fiber"])
    d.group = iptr(keep["group"])
    d.pins = iptr(keep["pins"])
    d.pin_xyz = dptr(keep["pin_xyz"])
    d.alpha_hat = float(problem.alpha_hat if alpha_hat is None else alpha_hat)
    d.mu_ref = float(mu_ref)
    d.fiber_k = float(fiber_k)
    d.weight_mode = int(weight_mode)
    d.n_modes = int(problem.n_modes if n_modes is None else n_modes)
    d.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    d.leaf_size = int(leaf_size)
    d.bone = iptr(keep["bone"]) if "bone" in keep else None
    d.hessian_blocks = BLOCKS[hessian_blocks] if isinstance(hessian_blocks, str) else int(hessian_blocks)
    d.affine_bones = int(bool(affine_bones))
    d.bone_slack = float(bone_slack)
    return d, keep


class HostSetup:
    """Host-only mesh setup (no GPU): factor and modes of the ACAP operator."""

    def __init__(self, problem, **kw):
        self._lib = _lib.load()
        desc, self._keep = _desc_arrays(problem, **kw)
        h = C.c_void_p()
        check(self._lib.emu_host_setup_create(C.byref(desc), C.byref(h)), "emu_host_setup_create")
        self._h = h
        self.n = problem.n_vertices
        self.m = problem.n_tets

    def close(self):
        if getattr(self, "_h", None):
            self._lib.emu_host_setup_destroy(self._h)
            self._h = None

    __del__ = close

    def info(self):
        inf = _lib.MeshInfo()
        check(self._lib.emu_host_setup_info(self._h, C.byref(inf)))
        return inf.as_dict()

    def solve(self, b):
        b = np.ascontiguousarray(b, np.float64)
        x = np.zeros((self.n, 3))
        check(self._lib.emu_host_setup_solve(self._h, dptr(b), dptr(x)))
        return x

    def apply(self, x):
        x = np.ascontiguousarray(x, np.float64)
        y = np.zeros((self.n, 3))
        check(self._lib.emu_host_setup_apply(self._h, dptr(x), dptr(y)))
        return y

    def modes(self):
        k1 = self.info()["n_modes"] // 3
        nu = np.zeros(k1)
        phi = np.zeros((k1, self.n))
        check(self._lib.emu_host_setup_modes(self._h, dptr(nu), dptr(phi)))
        return nu, phi

    def geometry(self):
        t = np.zeros((self.m, 4), np.int32)
        vol = np.zeros(self.m)
        w = np.zeros(self.m)
        check(self._lib.emu_host_setup_geometry(self._h, iptr(t), dptr(vol), dptr(w)))
        return t, vol, w


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("EMU device meshes need a HIP GPU (torch.cuda.is_available() is False)")
    return torch


def _stream(torch):
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def default_opts(**kw):
    o = _lib.load().emu_solve_opts_default()
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _torch_allocator(torch):
    """emu_dev_alloc_fn / emu_dev_free_fn drawing from torch's caching
    allocator on the current device and stream (a failed allocation returns
    NULL, which the library reports as EMU_E_OOM)."""
    dev = torch.cuda.current_device()
    stream = torch.cuda.current_stream(dev)

    def alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream)
        except Exception:
            return None

    def free(ptr, ctx):
        try:
            torch.cuda.caching_allocator_delete(ptr)
        except Exception:
            pass

    return _lib.ALLOC_FN(alloc), _lib.FREE_FN(free)


class Mesh:
    """A mesh resident on the current HIP device (factor, modes and state).

    Its device memory comes from torch's caching allocator (``torch_alloc``),
    so it shows in ``torch.cuda.memory_allocated()``; with ``torch_alloc=False``
    the library allocates with hipMalloc itself."""

    def __init__(self, problem, torch_alloc=True, **kw):
        self.torch = _torch()
        self._lib = _lib.load()
        desc, keep = _desc_arrays(problem, **kw)
        if torch_alloc:
            # kept alive as long as the mesh: the library frees through them
            self._alloc_fns = _torch_allocator(self.torch)
            desc.dev_alloc, desc.dev_free = self._alloc_fns
        h = C.c_void_p()
        check(self._lib.emu_create_mesh(C.byref(desc), C.byref(h)), "emu_create_mesh")
        self._h = h
        self.n = problem.n_vertices
        self.m = problem.n_tets
        self.n_groups = problem.n_groups
        self.set_activation(problem.activation)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.emu_destroy_mesh(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def info(self):
        inf = _lib.MeshInfo()
        check(self._lib.emu_mesh_get_info(self._h, C.byref(inf)))
        return inf.as_dict()

    def set_activation(self, a):
        a = np.ascontiguousarray(np.atleast_1d(a), np.float64)
        check(self._lib.emu_set_activation(self._h, dptr(a)), "emu_set_activation")

    def set_pin_targets(self, pin_xyz):
        p = np.ascontiguousarray(pin_xyz, np.float64)
        check(self._lib.emu_set_pin_targets(self._h, dptr(p)), "emu_set_pin_targets")

    def set_external_forces(self, f):
        """Constant vertex forces [n,3] (N), or None to remove them."""
        if f is None:
            check(self._lib.emu_set_external_forces(self._h, None), "emu_set_external_forces")
            return
        f = np.ascontiguousarray(f, np.float64).reshape(self.n, 3)
        check(self._lib.emu_set_external_forces(self._h, dptr(f)), "emu_set_external_forces")

    def set_contact(self, planes=None, spheres=None, stiffness=1.0, tol=1e-8, max_rounds=8):
        """Obstacles for the contact loop after every accepted step: planes
        [np,4] rows (unit normal, b), spheres [ns,4] rows (center, radius),
        penalty stiffness (N/m), stop tolerance on |f|_2 (N) and the round
        limit; no obstacles removes contact."""
        P = np.zeros((0, 4)) if planes is None else np.ascontiguousarray(planes, np.float64).reshape(-1, 4)
        S = np.zeros((0, 4)) if spheres is None else np.ascontiguousarray(spheres, np.float64).reshape(-1, 4)
        desc = _lib.ContactDesc(len(P), dptr(P) if len(P) else None, len(S), dptr(S) if len(S) else None,
                                float(stiffness), float(tol), int(max_rounds))
        check(self._lib.emu_set_contact(self._h, C.byref(desc)), "emu_set_contact")

    def set_modes(self, nu, phi):
        nu = np.ascontiguousarray(nu, np.float64)
        phi = np.ascontiguousarray(phi, np.float64)
        check(self._lib.emu_set_modes(self._h, int(nu.shape[0]), dptr(nu), dptr(phi)), "emu_set_modes")

    def get_modes(self):
        k1 = self.info()["n_modes"] // 3
        nu = np.zeros(k1)
        phi = np.zeros((k1, self.n))
        check(self._lib.emu_get_modes(self._h, dptr(nu), dptr(phi)))
        return nu, phi

    def solve(self, opts=None, raise_on_error=True, **kw):
        """Run the solver; returns (q [n,3] float64 device tensor, stats dict)."""
        t = self.torch
        o = opts if opts is not None else default_opts(**kw)
        q = t.empty((self.n, 3), dtype=t.float64, device="cuda")
        st = _lib.SolveStats()
        code = self._lib.emu_solve(self._h, C.byref(o), C.c_void_p(q.data_ptr()), C.byref(st), _stream(t))
        stats = st.as_dict()
        stats["status_name"] = _lib.STATUS_NAMES.get(code, str(code))
        if raise_on_error and code not in (0, 3):
            check(code, "emu_solve")
        return q, stats

    def get_state(self):
        t = self.torch
        F = t.empty((self.m, 3, 3), dtype=t.float64, device="cuda")
        q = t.empty((self.n, 3), dtype=t.float64, device="cuda")
        check(self._lib.emu_get_state(self._h, C.c_void_p(F.data_ptr()), C.c_void_p(q.data_ptr()), _stream(t)))
        return F, q

    def set_state(self, F):
        t = self.torch
        F = t.as_tensor(F, dtype=t.float64, device="cuda").contiguous()
        check(self._lib.emu_set_state(self._h, C.c_void_p(F.data_ptr()), _stream(t)), "emu_set_state")

    def restore_equilibrium(self, F, a, grad_tol=1e-8, max_iters=10000):
        """Put the mesh back at a converged state F (from get_state) for the
        activations a: set_state re-splits F and re-solves q*(F); the warm
        solve that follows confirms convergence at once (it stops on the
        first gradient test) and re-arms emu_solve_grad."""
        self.set_activation(a)
        self.set_state(F)
        _, st = self.solve(grad_tol=grad_tol, max_iters=max_iters, warm_start=1)
        if st["status"] != 0:
            raise _lib.EmuError(st["status"], "could not restore the converged state")
        return st

    def solve_grad(self, dL_dq, stats=False, noalloc=False):
        """dL/da (numpy [n_groups]) at the converged state for dL/dq ([n,3] GPU
        tensor); ``noalloc`` uses the allocation-free entry point."""
        t = self.torch
        g = t.as_tensor(dL_dq, dtype=t.float64, device="cuda").contiguous()
        out = np.zeros(max(1, self.n_groups))
        st = _lib.SolveStats()
        fn = self._lib.emu_solve_grad_noalloc if noalloc else self._lib.emu_solve_grad
        check(fn(self._h, C.c_void_p(g.data_ptr()), dptr(out), C.byref(st), _stream(t)),
              "emu_solve_grad_noalloc" if noalloc else "emu_solve_grad")
        return (out[:self.n_groups], st.as_dict()) if stats else out[:self.n_groups]

    def profile_kernels(self, reps=20):
        """Average device ms per kernel class (HIP events), {name: ms}."""
        t = self.torch
        names = []
        while self._lib.emu_kernel_name(len(names)) is not None:
            names.append(self._lib.emu_kernel_name(len(names)).decode())
        out = np.zeros(len(names))
        check(self._lib.emu_profile_kernels(self._h, int(reps), dptr(out), _stream(t)), "emu_profile_kernels")
        return {nm: float(out[k]) for k, nm in enumerate(names)}

    def evaluate(self, F, direction=True):
        """q*(F), E(F), |dE/dF| and the quasi-Newton direction at F (state unchanged)."""
        t = self.torch
        F = t.as_tensor(F, dtype=t.float64, device="cuda").contiguous()
        q = t.empty((self.n, 3), dtype=t.float64, device="cuda")
        dvec = t.empty((self.m, 3, 3), dtype=t.float64, device="cuda") if direction else None
        e = C.c_double()
        g = C.c_double()
        check(self._lib.emu_evaluate(self._h, C.c_void_p(F.data_ptr()), C.c_void_p(q.data_ptr()),
                                     C.byref(e), C.byref(g),
                                     C.c_void_p(dvec.data_ptr()) if dvec is not None else None,
                                     _stream(t)), "emu_evaluate")
        return dict(q=q, energy=e.value, grad_norm=g.value, direction=dvec)


class _SolveFn:
    """torch.autograd.Function: activations -> equilibrium positions.

    forward: emu_set_activation + emu_solve (to the given tolerance);
    backward: emu_solve_grad (adjoint of the equilibrium w.r.t. activations)."""

    _cls = None

    @classmethod
    def get(cls):
        if cls._cls is None:
            import torch

            class SolveFunction(torch.autograd.Function):
                @staticmethod
                def forward(ctx, a, mesh, grad_tol, max_iters):
                    a_host = a.detach().cpu().numpy().astype(np.float64)
                    mesh.set_activation(a_host)
                    q, st = mesh.solve(grad_tol=grad_tol, max_iters=max_iters)
                    if st["status"] != 0:
                        raise _lib.EmuError(st["status"], "forward solve did not converge")
                    # the equilibrium this graph node stands for: the mesh may be
                    # solved again (another forward, a probe) before backward
                    F, _ = mesh.get_state()
                    ctx.mesh, ctx.a_host, ctx.F = mesh, a_host, F
                    ctx.opts = (grad_tol, max_iters)
                    ctx.a_device = a.device
                    return q

                @staticmethod
                def backward(ctx, grad_q):
                    mesh = ctx.mesh
                    mesh.restore_equilibrium(ctx.F, ctx.a_host, *ctx.opts)
                    g = mesh.solve_grad(grad_q.contiguous())
                    return torch.as_tensor(g, dtype=torch.float64, device=ctx.a_device), None, None, None

            cls._cls = SolveFunction
        return cls._cls


def solve(mesh: "Mesh", a, grad_tol: float = 1e-8, max_iters: int = 10000):
    """Differentiable equilibrium q(a) (float64 [n,3] on the GPU)."""
    import torch
    a = torch.as_tensor(a, dtype=torch.float64)
    return _SolveFn.get().apply(a, mesh, grad_tol, max_iters)


class Server:
    """Continuous-batching solve server on the current HIP device.

    ``submit`` queues one solve (a ``workloads.Problem`` with its activations)
    and returns a ticket; ``wait`` blocks for its result.  Host setup, HBM
    admission and the batched iteration all run inside the library."""

    def __init__(self, hbm_budget_bytes=0, max_slots=0, setup_threads=0, iters_per_round=0):
        _torch()
        self._lib = _lib.load()
        o = _lib.ServerOpts(int(hbm_budget_bytes), int(max_slots), int(setup_threads), int(iters_per_round))
        h = C.c_void_p()
        check(self._lib.emu_server_create(C.byref(o), C.byref(h)), "emu_server_create")
        self._h = h
        self._n = {}

    def submit(self, problem, activation=None, precision="fp64", opts=None, **kw):
        desc, keep = _desc_arrays(problem, precision=precision)
        a = np.ascontiguousarray(problem.activation if activation is None else activation, np.float64)
        if opts is None:
            opts = default_opts(**kw)
        t = C.c_uint64()
        check(self._lib.emu_server_submit(self._h, C.byref(desc), dptr(a), C.byref(opts), C.byref(t)),
              "emu_server_submit")
        del keep  # the library copied every array
        self._n[t.value] = problem.n_vertices
        return t.value

    def wait(self, ticket, raise_on_error=False):
        """(q [n,3] numpy, stats dict, times dict); stats['status'] is the
        request's emu_status (a failed request raises only with
        ``raise_on_error``)."""
        n = self._n.pop(ticket, 0)
        q = np.zeros((n, 3))
        st = _lib.SolveStats()
        tm = _lib.RequestTimes()
        code = self._lib.emu_server_wait(self._h, C.c_uint64(ticket), dptr(q), C.byref(st), C.byref(tm))
        if code == 1 or (raise_on_error and code != 0):  # EMU_E_INVALID: unknown ticket
            check(code, "emu_server_wait")
        stats = st.as_dict()
        stats["status"] = code
        return q, stats, tm.as_dict()

    def report(self):
        r = _lib.ServerReport()
        check(self._lib.emu_server_report_get(self._h, C.byref(r)))
        return r.as_dict()

    def close(self):
        if getattr(self, "_h", None):
            code = self._lib.emu_server_destroy(self._h)
            self._h = None
            check(code, "emu_server_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def choose_alpha(alphas, iters, converged, spike=3.0):
    """The weighting-parameter rule of Sec. 3.7: walk the candidates upward and
    stop at the first one whose iteration count jumps by more than ``spike``
    times the previous count (or that does not converge); return the
    candidate just before the jump (the last candidate if none jumps).
    ``alphas`` ascending; returns (alpha, index)."""
    if len(alphas) == 0:
        raise ValueError("no candidates")
    for k in range(1, len(alphas)):
        if not converged[k] or iters[k] > spike * max(1, iters[k - 1]):
            return alphas[k - 1], k - 1
    return alphas[-1], len(alphas) - 1


def alpha_search(problem, alpha_hats=(1.0, 10.0, 100.0, 1e3, 1e4, 1e5), grad_rtol=1e-6, max_iters=5000,
                 spike=3.0, precision="fp64", server=None):
    """Sec. 3.7: solve the problem at its activations once per candidate
    alpha_hat (cold start, |g| <= grad_rtol |g_0|), all candidates as one
    batch on the serving loop, and pick alpha_hat by ``choose_alpha``.
    Returns a dict with the choice, the per-candidate iteration counts and
    statuses and the wall time of the batch."""
    import time
    alphas = sorted(float(a) for a in alpha_hats)
    own = server is None
    srv = Server() if own else server
    t0 = time.perf_counter()
    tickets = []
    for a in alphas:
        p = problem.copy()
        p.alpha_hat = a
        tickets.append(srv.submit(p, precision=precision, grad_tol=0.0, grad_rtol=grad_rtol,
                                  max_iters=max_iters, warm_start=0))
    res = [srv.wait(t) for t in tickets]
    wall = time.perf_counter() - t0
    if own:
        srv.close()
    iters = [st["iters"] for _, st, _ in res]
    conv = [st["status"] == 0 for _, st, _ in res]
    best, k = choose_alpha(alphas, iters, conv, spike)
    return {"alpha_hat": best, "index": k, "alpha_hats": alphas, "iters": iters, "converged": conv,
            "q": res[k][0], "wall_s": wall}
