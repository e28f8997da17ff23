"""ctypes binding of the C ABI in include/emu.h and include/emu_host.h.

Argument marshalling only: every step of the solve runs in the shared library
(libemu.so, built by ``paper_2006_08821_amd.build``).  Loading fails loudly if
the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libemu.so")

EMU_OK = 0
STATUS_NAMES = {0: "EMU_OK", 1: "EMU_E_INVALID", 2: "EMU_E_SINGULAR", 3: "EMU_E_NOT_CONVERGED",
                4: "EMU_E_LINESEARCH", 5: "EMU_E_NONFINITE", 6: "EMU_E_OOM", 7: "EMU_E_HIP",
                8: "EMU_E_STATE", 9: "EMU_E_BUSY"}

P = C.c_void_p
I32P = C.POINTER(C.c_int32)
DP = C.POINTER(C.c_double)
# emu_dev_alloc_fn / emu_dev_free_fn
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class MeshDesc(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("n_tets", C.c_int32), ("n_groups", C.c_int32),
                ("n_pins", C.c_int32), ("rest_xyz", DP), ("tets", I32P), ("youngs", DP),
                ("poisson", DP), ("fiber", DP), ("group", I32P), ("pins", I32P), ("pin_xyz", DP),
                ("alpha_hat", C.c_double), ("mu_ref", C.c_double), ("fiber_k", C.c_double),
                ("weight_mode", C.c_int32), ("n_modes", C.c_int32), ("precision", C.c_int32),
                ("leaf_size", C.c_int32), ("bone", I32P), ("affine_bones", C.c_int32),
                ("bone_slack", C.c_double), ("hessian_blocks", C.c_int32),
                ("dev_alloc", ALLOC_FN), ("dev_free", FREE_FN), ("alloc_ctx", P)]


class SolveOpts(C.Structure):
    _fields_ = [("grad_tol", C.c_double), ("max_iters", C.c_int32), ("sigma0", C.c_double),
                ("armijo_c", C.c_double), ("rho", C.c_double), ("warm_start", C.c_int32),
                ("iters_per_sync", C.c_int32), ("stall_rel", C.c_double), ("grad_rtol", C.c_double),
                ("phase_timing", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("ls_trials", C.c_int32),
                ("acap_solves", C.c_int32), ("inverted", C.c_int32), ("clamped", C.c_int32),
                ("energy", C.c_double), ("grad_norm", C.c_double), ("grad_norm0", C.c_double),
                ("ms_total", C.c_double), ("ms_elem", C.c_double), ("ms_woodbury", C.c_double),
                ("ms_solve", C.c_double), ("ms_linesearch", C.c_double), ("contact_rounds", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class MeshInfo(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("n_tets", C.c_int32), ("n_free", C.c_int32),
                ("n_modes", C.c_int32), ("n_supernodes", C.c_int32), ("n_levels", C.c_int32),
                ("factor_nnz", C.c_int64), ("device_bytes", C.c_int64), ("mu_ref", C.c_double),
                ("alpha", C.c_double), ("fiber_k", C.c_double), ("setup_ms", C.c_double),
                ("mode_captured", C.c_double), ("fwd_column_levels", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerOpts(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("max_slots", C.c_int32),
                ("setup_threads", C.c_int32), ("iters_per_round", C.c_int32)]


class ContactDesc(C.Structure):
    _fields_ = [("n_planes", C.c_int32), ("planes", DP), ("n_spheres", C.c_int32), ("spheres", DP),
                ("stiffness", C.c_double), ("tol", C.c_double), ("max_rounds", C.c_int32)]


class RequestTimes(C.Structure):
    _fields_ = [("t_submit", C.c_double), ("t_setup_done", C.c_double), ("t_admit", C.c_double),
                ("t_finish", C.c_double), ("device_bytes", C.c_int64), ("setup_cached", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerReport(C.Structure):
    _fields_ = [("peak_resident_bytes", C.c_int64), ("peak_active", C.c_int32),
                ("submitted", C.c_int32), ("completed", C.c_int32), ("failed", C.c_int32),
                ("rounds", C.c_int32), ("resident_bytes", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# name -> (restype, argtypes); mirrors the declarations of the two headers
SIGNATURES = {
    "emu_solve_opts_default": (SolveOpts, []),
    "emu_last_error": (C.c_char_p, []),
    "emu_create_mesh": (C.c_int, [C.POINTER(MeshDesc), C.POINTER(P)]),
    "emu_destroy_mesh": (C.c_int, [P]),
    "emu_mesh_get_info": (C.c_int, [P, C.POINTER(MeshInfo)]),
    "emu_set_activation": (C.c_int, [P, DP]),
    "emu_set_pin_targets": (C.c_int, [P, DP]),
    "emu_set_external_forces": (C.c_int, [P, DP]),
    "emu_set_contact": (C.c_int, [P, C.POINTER(ContactDesc)]),
    "emu_set_modes": (C.c_int, [P, C.c_int32, DP, DP]),
    "emu_get_modes": (C.c_int, [P, DP, DP]),
    "emu_solve": (C.c_int, [P, C.POINTER(SolveOpts), P, C.POINTER(SolveStats), P]),
    "emu_solve_grad": (C.c_int, [P, P, DP, C.POINTER(SolveStats), P]),
    "emu_solve_grad_noalloc": (C.c_int, [P, P, DP, C.POINTER(SolveStats), P]),
    "emu_get_state": (C.c_int, [P, P, P, P]),
    "emu_set_state": (C.c_int, [P, P, P]),
    "emu_evaluate": (C.c_int, [P, P, P, DP, DP, P, P]),
    "emu_profile_kernels": (C.c_int, [P, C.c_int32, DP, P]),
    "emu_kernel_name": (C.c_char_p, [C.c_int32]),
    "emu_server_create": (C.c_int, [C.POINTER(ServerOpts), C.POINTER(P)]),
    "emu_server_submit": (C.c_int, [P, C.POINTER(MeshDesc), DP, C.POINTER(SolveOpts),
                                    C.POINTER(C.c_uint64)]),
    "emu_server_wait": (C.c_int, [P, C.c_uint64, DP, C.POINTER(SolveStats), C.POINTER(RequestTimes)]),
    "emu_server_report_get": (C.c_int, [P, C.POINTER(ServerReport)]),
    "emu_server_destroy": (C.c_int, [P]),
    "emu_host_setup_create": (C.c_int, [C.POINTER(MeshDesc), C.POINTER(P)]),
    "emu_host_setup_destroy": (C.c_int, [P]),
    "emu_host_setup_info": (C.c_int, [P, C.POINTER(MeshInfo)]),
    "emu_host_setup_solve": (C.c_int, [P, DP, DP]),
    "emu_host_setup_apply": (C.c_int, [P, DP, DP]),
    "emu_host_setup_modes": (C.c_int, [P, DP, DP]),
    "emu_host_setup_geometry": (C.c_int, [P, I32P, DP, DP]),
}

_LIB = None


class EmuError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def load():
    """Load libemu.so (raises if it is missing)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2006_08821_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _LIB = lib
    return lib


def check(code, what=""):
    if code != EMU_OK:
        msg = load().emu_last_error().decode(errors="replace")
        raise EmuError(code, f"{what}: {msg}" if what else msg)
    return code


def dptr(a):
    return a.ctypes.data_as(DP)


def iptr(a):
    return a.ctypes.data_as(I32P)
